"""Systems beyond the register inverse (n > 96): the blocked Gauss-Jordan
refresh, delayed updates of n = 512 inverses and, for the 1024-electron
workload (256 nuclei, L = 4096, Lambda banded at 8 bohr), the P products that
skip Lambda's zero tiles.

* Evaluation against the oracle at the FP64 bar (relative 1e-10 on log|Psi| and
  E_loc, 1e-8 on the drift).
* Move ratios of an up and a down electron against the oracle's ratio of full
  determinants, and the updated inverse against the inverse of the updated W.
* 70 Metropolis steps (a refresh after 64 moves of one spin): the tracked log|Psi| and inverse
  equal those of a fresh evaluation at the final positions.
* n = 112, 128, 150 (the blocked elimination runs for n > 96; 112 and 150 are
  not multiples of the 64-wide panel): identity padding.
* W = 0 is reported singular (status 1).
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def large():
    return C.large_256nuc_1024e(n_walkers=4)


def _eval(P, w, Wk=None, r=None):
    Wk = w.r0.shape[0] if Wk is None else Wk
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0[:Wk], device="cuda") if r is None else r
    out = wk.eval_batch(r, drift=True)
    torch.cuda.synchronize()
    return sysh, wk, out


def _check_eval(out, w, idx):
    ref = O.evaluate(O.from_workload_system(w.system), torch.tensor(w.r0[idx]))
    e_la = rel_err(out["logabs"].cpu()[idx], ref["logabs"]).max().item()
    e_el = rel_err(out["e_loc"].cpu()[idx], ref["e_loc"]).max().item()
    d = out["drift"].cpu()[idx]
    e_dr = ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[large eval {w.system.name}] rel err logabs {e_la:.3e}, e_loc {e_el:.3e}, drift {e_dr:.3e}")
    assert e_la <= 1e-10 and e_el <= 1e-10 and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu()[idx], ref["sign"])
    assert (out["status"].cpu()[idx] == 0).all()


def test_large_eval_matches_oracle(large):
    P = need_gpu()
    _, _, out = _eval(P, large)
    _check_eval(out, large, [0, 3])


@pytest.mark.parametrize("n_elec", [224, 256, 300])
def test_blocked_eval_and_refresh(n_elec):
    # n = 112, 128, 150: one or two padded 64-column panels
    P = need_gpu()
    w = C.multi_system(n_elec, n_walkers=8)
    sysh, wk, out = _eval(P, w)
    _check_eval(out, w, [0, 7])
    d, u = C.chain_arrays(17, 40, 8)          # refresh every 32
    wk.vmc_steps(0, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"))
    r = wk.read(P.STATE_R)
    la, A = wk.read(P.STATE_LOGABS), wk.read(P.STATE_AINV)
    _, wk2, out2 = _eval(P, w, r=r)
    assert rel_err(la.cpu(), out2["logabs"].cpu()).max().item() <= 1e-10
    A2 = wk2.read(P.STATE_AINV)
    assert ((A - A2).abs().max() / A2.abs().max()).item() <= 1e-8


def test_blocked_inverse_narrow_panels():
    # n = 550 (np = 576 > 512): 32-column panels, each followed by the two
    # batched MFMA products left and right of the panel
    P = need_gpu()
    w = C.multi_system(1100, n_walkers=2)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, 2)
    out = wk.eval_batch(torch.tensor(w.r0[:2], device="cuda"))
    torch.cuda.synchronize()
    assert int(out["status"].abs().max()) == 0
    W, A = wk.read(P.STATE_W).cpu(), wk.read(P.STATE_AINV).cpu()
    Ainv = torch.linalg.inv(W)
    err = ((A - Ainv).abs().max() / Ainv.abs().max()).item()
    print(f"[blocked inverse n=550] W^-1 against LAPACK {err:.3e}")
    assert err <= 1e-8
    sg, _ = torch.linalg.slogdet(W)
    assert torch.equal(out["sign"].cpu(), sg)


def test_large_ratios_and_update(large):
    P = need_gpu()
    w = large
    sysh, wk, _ = _eval(P, w, Wk=2)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0[:2])
    disp = torch.tensor(C.chain_arrays(23, 2, 2)[0])
    for t, e in enumerate((3, 700)):
        rn = r[:, e] + disp[t]
        ratio = wk.propose(e, rn.cuda().contiguous())
        torch.cuda.synchronize()
        rr = O.move_ratio(sy, r[:1], e, rn[:1])
        err = (ratio.cpu()[:1] - rr).abs() / rr.abs().clamp(min=1.0)
        print(f"[large move e={e}] ratio {ratio.cpu()[0].item():.6e} oracle {rr[0].item():.6e} rel {err.max():.3e}")
        assert err.max().item() <= 1e-10
        wk.accept(e, torch.ones(2, dtype=torch.uint8, device="cuda"))
        r = r.clone()
        r[:, e] = rn
    torch.cuda.synchronize()
    W, A = wk.read(P.STATE_W).cpu(), wk.read(P.STATE_AINV).cpu()
    Ainv = torch.linalg.inv(W)
    assert ((A - Ainv).abs().max() / Ainv.abs().max()).item() <= 1e-8
    assert torch.equal(wk.read(P.STATE_R).cpu(), r)


def test_large_refresh_after_64_moves(large):
    P = need_gpu()
    w = large
    sysh, wk, _ = _eval(P, w, Wk=4)
    d, u = C.chain_arrays(29, 70, 4)
    cnt = torch.zeros(4, dtype=torch.int32, device="cuda")
    wk.vmc_steps(0, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"), cnt)
    r = wk.read(P.STATE_R)
    la, A = wk.read(P.STATE_LOGABS), wk.read(P.STATE_AINV)
    _, wk2, out2 = _eval(P, w, Wk=4, r=r)
    A2 = wk2.read(P.STATE_AINV)
    print(f"[large chain] accepted {cnt.cpu().tolist()} of 70 each")
    assert int(cnt.sum()) > 0
    assert rel_err(la.cpu(), out2["logabs"].cpu()).max().item() <= 1e-10
    assert ((A - A2).abs().max() / A2.abs().max()).item() <= 1e-8


def test_large_singular_status(large):
    P = need_gpu()
    w = large
    zero = dataclasses.replace(w.system, lam=np.zeros_like(w.system.lam))
    w0 = dataclasses.replace(w, system=zero)
    _, _, out = _eval(P, w0, Wk=2)
    assert (out["status"].cpu() == 1).all()
    assert torch.isinf(out["logabs"].cpu()).all()
