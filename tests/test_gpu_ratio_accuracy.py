"""Single-electron move ratios of every precision mode against the oracle at
160 electrons (the benchmark workload), on walkers drawn from |Psi|^2.

The oracle's ratio is Psi(x')/Psi(x) from two full FP64 evaluations (the
definition); the library's comes from the maintained inverse and the streamed
P rows of the mode's storage type.  Walkers are equilibrated by one FP64
sweep (160 moves each) before the comparison, as the error metric of the
benchmark prescribes; then every mode evaluates them and proposes moves of
four up and four down electrons.  Error metric |x - y| / max(|y|, 1).

Bars: FP64 1e-10 (as every FP64 ratio test); QMC_REFINED 1e-6, the mixed bar
(its rows are the int8-refined FP64 products, and the basis functions its
screened proposal skips change the ratio by at most 1e-13, so in practice it
lands near the FP64 figure).  The modes that stream reduced-precision rows --
QMC_MIXED (FP32 rows), QMC_MIXED_BF16 (BF16 rows) and QMC_W_FP32 -- carry the
storage rounding of P amplified by the inverse column (measured 1e-4 to 1 on
this workload) and are reported, not held to the bar: the benchmark marks
them non-conforming.
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

WK = 64
ELECTRONS = (0, 27, 52, 79, 80, 101, 133, 159)


@pytest.fixture(scope="module")
def sampled():
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=WK)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, WK)
    wk.eval_batch(torch.tensor(w.r0, device="cuda"))
    d, u = C.chain_arrays(4711, 160, WK)
    wk.vmc_steps(0, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"))
    r = wk.read(P.STATE_R).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    disp = torch.tensor(C.chain_arrays(4712, len(ELECTRONS), WK)[0])
    ref = {}
    for t, e in enumerate(ELECTRONS):
        rn = r[:, e] + disp[t]
        ref[e] = (rn, O.move_ratio(sy, r, e, rn))
    return w, r, ref


def _errors(P, w, r, ref, precision):
    sysh = P.JAGPSystem(w.system, precision=precision)
    wk = P.Walkers(sysh, WK)
    errs = []
    for e in ELECTRONS:
        wk.eval_batch(r.cuda())
        rn, rr = ref[e]
        ratio = wk.propose(e, rn.cuda().contiguous())
        torch.cuda.synchronize()
        errs.append(rel_err(ratio.cpu(), rr))
    return torch.stack(errs)


@pytest.mark.parametrize("mode", ["fp64", "refined", "mixed_fp32_rows", "mixed_bf16", "w_fp32"])
def test_move_ratio_error_vs_oracle(sampled, mode):
    P = need_gpu()
    w, r, ref = sampled
    prec = {"fp64": P.QMC_FP64, "refined": P.QMC_REFINED, "mixed_fp32_rows": P.QMC_MIXED,
            "mixed_bf16": P.QMC_MIXED_BF16, "w_fp32": P.QMC_W_FP32}[mode]
    err = _errors(P, w, r, ref, prec)
    q = torch.quantile(err.flatten(), 0.999).item()
    print(f"[ratio accuracy {mode}] max {err.max().item():.3e}  p99.9 {q:.3e}  "
          f"walkers above 1e-6: {int((err > 1e-6).any(0).sum())} of {WK}")
    if mode == "fp64":
        assert err.max().item() <= 1e-10
    elif mode == "refined":
        assert err.max().item() <= 1e-6
