"""qmc_eval_batch at the walkers' current positions (r = NULL).

An evaluation at the current positions reuses the P rows of a spin none of
whose electrons has been proposed since the rows were built (FP64, FP32 and
the refined int8 products; the mixed modes with FP32 / BF16 rows rebuild both
halves).  It must give what an evaluation at the same positions passed
explicitly gives:

* after a full sweep (the up rows current from the rebuild between the two
  halves), after moves of up electrons only (the down rows current) and right
  after an evaluation (both current): log|Psi|, sign, E_kin, E_loc and drift
  within 1e-12 of the explicit evaluation on a second walker set moved by the
  same draws (a reused half comes from the accepted moves' basis rows, the
  explicit build from the evaluation's own, which agree to rounding), and the
  FP64 and refined results within the bars of the evaluation parity tests
  against the oracle;
* the same against a fresh walker set evaluated at those positions (every P
  row built anew; in QMC_REFINED a build otherwise takes only the rows whose
  electron has moved since the row was last built);
* moves after it: a sweep on both walker sets gives bitwise equal positions;
* refusal before the first evaluation; after a parameter change both halves are
  built again (results as the explicit evaluation of the changed system).
"""
import dataclasses

import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

KEYS = ("logabs", "e_kin", "e_loc")


def _close(a, b, tol):
    for k in KEYS:
        err = rel_err(a[k].cpu(), b[k].cpu()).max().item()
        assert err <= tol, (k, err)
    dr = ((a["drift"] - b["drift"]).abs() / b["drift"].abs().clamp(min=1.0)).max().item()
    assert dr <= tol, ("drift", dr)
    assert torch.equal(a["sign"].cpu(), b["sign"].cpu())


def _pair(P, w, Wk, prec):
    sysh = P.JAGPSystem(w.system, precision=prec)
    a = P.Walkers(sysh, Wk, adjoint=False)
    b = P.Walkers(sysh, Wk, adjoint=False)
    return sysh, a, b


def _moves(wk, e0, n, seed):
    d, u = C.chain_arrays(seed, n, wk.n)
    wk.vmc_steps(e0, torch.tensor(d, device="cuda"), torch.tensor(u, device="cuda"))


CASES = [("tiny", "QMC_FP64"), ("tiny", "QMC_W_FP32"), ("tiny", "QMC_REFINED"), ("tiny", "QMC_MIXED"),
         ("mol160", "QMC_FP64"), ("mol160", "QMC_REFINED")]


@pytest.mark.parametrize("name,prec", CASES)
def test_eval_at_current_positions(name, prec):
    P = need_gpu()
    w, Wk = (C.tiny_3nuc_10e(), 32) if name == "tiny" else (C.mol_40nuc_160e(n_walkers=4), 4)
    N, nu = w.system.n_up + w.system.n_dn, w.system.n_up
    sysh, a, b = _pair(P, w, Wk, getattr(P, prec))
    r0 = torch.tensor(w.r0[:Wk], device="cuda")
    a.eval_batch(r0)
    b.eval_batch(r0)
    sy = O.from_workload_system(w.system)
    oracle_bar = {"QMC_FP64": 1e-10, "QMC_REFINED": 1e-8}.get(prec)
    for label, e0, n in (("full sweep", 0, N), ("up moves only", 0, nu), ("no moves", 0, 0)):
        if n:
            _moves(a, e0, n, 700 + n)
            _moves(b, e0, n, 700 + n)
        ra, rb = a.read(P.STATE_R), b.read(P.STATE_R)
        torch.cuda.synchronize()
        assert torch.equal(ra, rb), label
        oa = a.eval_batch(None)
        ob = b.eval_batch(rb)
        torch.cuda.synchronize()
        print(f"[eval here {name} {prec}] {label}: logabs {rel_err(oa['logabs'].cpu(), ob['logabs'].cpu()).max():.2e}"
              f" e_loc {rel_err(oa['e_loc'].cpu(), ob['e_loc'].cpu()).max():.2e}")
        _close(oa, ob, 1e-12)
        if oracle_bar is not None:
            ref = O.evaluate(sy, ra.cpu())
            for k in KEYS:
                assert rel_err(oa[k].cpu(), ref[k]).max().item() <= oracle_bar, (label, k)
    # a fresh walker set (every row built from scratch) at the same positions
    c = P.Walkers(sysh, Wk, adjoint=False)
    oc = c.eval_batch(a.read(P.STATE_R))
    oa = a.eval_batch(None)
    torch.cuda.synchronize()
    _close(oa, oc, 1e-12)
    c.close()
    # moves after the evaluation at the current positions
    _moves(a, 0, N, 999)
    _moves(b, 0, N, 999)
    la, lb = a.read(P.STATE_LOGABS), b.read(P.STATE_LOGABS)
    torch.cuda.synchronize()
    assert torch.equal(a.read(P.STATE_R), b.read(P.STATE_R))
    assert rel_err(la.cpu(), lb.cpu()).max().item() <= 1e-12
    a.close(); b.close(); sysh.close()


def test_eval_at_current_positions_refusal_and_param_change():
    P = need_gpu()
    w = C.tiny_3nuc_10e()
    Wk, N = 16, w.system.n_up + w.system.n_dn
    sysh, a, b = _pair(P, w, Wk, P.QMC_FP64)
    with pytest.raises(P.QMCError) as ex:
        a.eval_batch(None)
    assert ex.value.code == -6   # QMC_ERR_STATE
    r0 = torch.tensor(w.r0[:Wk], device="cuda")
    a.eval_batch(r0)
    b.eval_batch(r0)
    _moves(a, 0, N, 17)
    _moves(b, 0, N, 17)
    # a parameter change: both halves are stale whatever the moves left
    s = w.system
    R = torch.tensor(s.R, device="cuda")
    R[1, 0] += 0.05
    sysh.set_params(R, None, None, None)
    oa = a.eval_batch(None)
    ob = b.eval_batch(b.read(P.STATE_R))
    torch.cuda.synchronize()
    _close(oa, ob, 1e-12)
    sy = dataclasses.replace(O.from_workload_system(s), R=R.cpu())
    ref = O.evaluate(sy, a.read(P.STATE_R).cpu())
    assert rel_err(oa["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-10
    a.close(); b.close(); sysh.close()
