"""Members with unpaired orbitals (polarized AGP), a Jastrow basis (J1
inhomogeneous + J3/4) or contracted orbitals in one multi-system launch
(qmc_multi_vmc_steps), beside a plain member.

* Each member must evolve exactly as it does alone (qmc_vmc_steps with the
  same displacements and uniforms): positions, log|Psi|, sign, W and W^{-1}
  bitwise equal, in FP64 and with FP32 / BF16 move rows.
* In FP64 the chains must equal the oracle's chains (positions bitwise, the
  accept decisions being those of the definition) with log|Psi| at 1e-10.
* A captured graph must reproduce the direct launches bitwise.
"""
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

WORKLOADS = (C.polarized_4nuc_20e, C.jas3_4nuc_20e, C.contracted_4nuc_20e, C.tiny_3nuc_10e)
PRECISIONS = ("QMC_FP64", "QMC_MIXED", "QMC_MIXED_BF16")


def _members(P, Wk, precision):
    out = []
    for f in WORKLOADS:
        w = f(n_walkers=Wk)
        sysh = P.JAGPSystem(w.system, precision=getattr(P, precision))
        wk = P.Walkers(sysh, Wk)
        wk.eval_batch(torch.tensor(w.r0, device="cuda"))
        out.append((w, sysh, wk))
    return out


@pytest.mark.parametrize("precision", PRECISIONS)
def test_multi_ansatz_members_equal_single_runs(precision):
    P = need_gpu()
    Wk, n_steps = 8, 130          # several sweeps: refreshes, spin changes and P rebuilds inside
    grp = _members(P, Wk, precision)
    solo = _members(P, Wk, precision)
    draws = [C.chain_arrays(1300 + k, n_steps, Wk) for k in range(len(WORKLOADS))]
    disp = [torch.tensor(d, device="cuda") for d, _ in draws]
    unif = [torch.tensor(u, device="cuda") for _, u in draws]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, disp, unif)
    for k, (_, _, wk) in enumerate(solo):
        wk.vmc_steps(0, disp[k], unif[k])
    torch.cuda.synchronize()
    moved = 0
    for k, f in enumerate(WORKLOADS):
        a, b = grp[k][2], solo[k][2]
        for item in (P.STATE_R, P.STATE_LOGABS, P.STATE_SIGN, P.STATE_AINV, P.STATE_W):
            assert torch.equal(a.read(item), b.read(item)), (f.__name__, item)
        moved += int((a.read(P.STATE_R).cpu() != torch.tensor(grp[k][0].r0)).any(-1).sum())
    assert moved > 0
    m.close()


def test_multi_ansatz_chains_match_oracle():
    P = need_gpu()
    Wk, n_steps = 4, 60
    grp = _members(P, Wk, "QMC_FP64")
    draws = [C.chain_arrays(1500 + k, n_steps, Wk) for k in range(len(WORKLOADS))]
    m = P.MultiSystem([wk for _, _, wk in grp])
    m.vmc_steps(n_steps, [torch.tensor(d, device="cuda") for d, _ in draws],
                [torch.tensor(u, device="cuda") for _, u in draws])
    torch.cuda.synchronize()
    for k, f in enumerate(WORKLOADS):
        w, _, wk = grp[k]
        sy = O.from_workload_system(w.system)
        rf, _, _ = O.run_chain(sy, torch.tensor(w.r0), torch.tensor(draws[k][0]), torch.tensor(draws[k][1]))
        assert torch.equal(wk.read(P.STATE_R).cpu(), rf), f.__name__
        err = rel_err(wk.read(P.STATE_LOGABS).cpu(), O.log_psi(sy, rf)[0]).max().item()
        assert err <= 1e-10, (f.__name__, err)
    m.close()


def test_multi_ansatz_graph_replay_equals_direct_launches():
    P = need_gpu()
    Wk, n_steps = 8, 120
    ga = _members(P, Wk, "QMC_MIXED")
    gb = _members(P, Wk, "QMC_MIXED")
    ma = P.MultiSystem([wk for _, _, wk in ga])
    mb = P.MultiSystem([wk for _, _, wk in gb])
    for _ in range(2):
        ma.vmc_steps(n_steps, seed=91, sigma=0.3, use_graph=True)
        mb.vmc_steps(n_steps, seed=91, sigma=0.3, use_graph=False)
    torch.cuda.synchronize()
    for k, f in enumerate(WORKLOADS):
        for item in (P.STATE_R, P.STATE_LOGABS, P.STATE_AINV):
            assert torch.equal(ga[k][2].read(item), gb[k][2].read(item)), (f.__name__, item)
    ma.close(); mb.close()
