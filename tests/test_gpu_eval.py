"""Parity of qmc_eval_batch (FP64 path) with the CPU oracle.

Tolerance: relative 1e-10 on log|Psi|, E_kin and E_loc with the metric
|x - y| / max(|y|, 1); drift 1e-8 relative to max(1, |drift|).  Walkers whose
geminal matrix has condition number above 1e10 would be reported separately
(the inverse diverges at nodes); none of the seeded inputs below reaches it.
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

TOL = 1e-10
DRIFT_TOL = 1e-8


def _compare(out, ref, idx, label):
    for key in ("logabs", "e_kin", "e_loc"):
        err = rel_err(out[key].cpu()[idx], ref[key]).max().item()
        assert err <= TOL, (label, key, err)
    assert torch.equal(out["sign"].cpu()[idx], ref["sign"]), label
    assert torch.equal(out["status"].cpu()[idx], ref["status"]), label
    d = out["drift"].cpu()[idx]
    derr = ((d - ref["drift"]).abs() / torch.clamp(ref["drift"].abs(), min=1.0)).max().item()
    assert derr <= DRIFT_TOL, (label, "drift", derr)


def _run(P, w, idx=None, n_walkers=None):
    s = w.system
    Wk = w.r0.shape[0] if n_walkers is None else n_walkers
    r = torch.tensor(w.r0[:Wk], device="cuda")
    sysh = P.JAGPSystem(s)
    wk = P.Walkers(sysh, Wk)
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    idx = list(range(Wk)) if idx is None else idx
    ref = O.evaluate(O.from_workload_system(s), torch.tensor(w.r0[idx]), with_intermediates=True)
    return out, ref, idx, wk


def test_eval_tiny_all_walkers_and_intermediates():
    P = need_gpu()
    w = C.tiny_3nuc_10e()
    out, ref, idx, wk = _run(P, w)
    _compare(out, ref, idx, "tiny")
    phi = wk.read(P.STATE_PHI).cpu()
    assert torch.allclose(phi, ref["Phi"], rtol=1e-13, atol=1e-15)
    W = wk.read(P.STATE_W).cpu()
    assert (rel_err(W, ref["W"]).max().item()) < 1e-12
    A = wk.read(P.STATE_AINV).cpu()
    assert torch.allclose(A, ref["A"], rtol=1e-9, atol=1e-9 * ref["A"].abs().max().item())
    la = wk.read(P.STATE_LOGABS).cpu()
    assert rel_err(la, ref["logabs"]).max().item() <= TOL


@pytest.mark.parametrize("n_walkers", [1, 3, 65])
def test_eval_tiny_ragged_walker_counts(n_walkers):
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=max(n_walkers, 1))
    out, ref, idx, _ = _run(P, w, n_walkers=n_walkers)
    _compare(out, ref, idx, f"tiny Wk={n_walkers}")


def test_eval_molecule_160e_sampled_walkers():
    # full size: 1024 walkers, 160 electrons, L = 600; the oracle checks a sample
    P = need_gpu()
    w = C.mol_40nuc_160e()
    idx = [0, 1, 255, 511, 512, 777, 1022, 1023]
    out, ref, idx, _ = _run(P, w, idx=idx)
    _compare(out, ref, idx, "mol160")
    assert (out["status"] == 0).all().item()
    assert torch.isfinite(out["e_loc"]).all().item()


def test_eval_forces_workload_pade_series():
    P = need_gpu()
    w = C.forces_20nuc_80e(n_walkers=64)
    out, ref, idx, _ = _run(P, w, idx=[0, 17, 40, 63])
    _compare(out, ref, idx, "forces80")


@pytest.mark.parametrize("n_elec", [16, 48, 96, 160, 192, 256])   # n_up 80 and 96: the walker-level cofactor kernel
def test_eval_multi_system_members(n_elec):
    P = need_gpu()
    w = C.multi_system(n_elec, n_walkers=32)
    out, ref, idx, _ = _run(P, w, idx=[0, 13, 31])
    _compare(out, ref, idx, f"multi{n_elec}")


def test_eval_singular_and_nonfinite_status():
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=4)
    s = w.system
    import dataclasses
    s0 = dataclasses.replace(s, lam=np.zeros_like(s.lam))
    r = torch.tensor(w.r0, device="cuda")
    wk = P.Walkers(P.JAGPSystem(s0), 4)
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    assert out["status"].cpu().tolist() == [1, 1, 1, 1]
    assert (out["sign"].cpu() == 0).all() and torch.isinf(out["logabs"].cpu()).all()
    # electron on a nucleus: infinite potential
    r2 = w.r0.copy()
    r2[1, 3] = s.R[0]
    wk = P.Walkers(P.JAGPSystem(s), 4)
    out = wk.eval_batch(torch.tensor(r2, device="cuda"))
    torch.cuda.synchronize()
    assert out["status"].cpu().tolist() == [0, 2, 0, 0]


def test_eval_deterministic():
    P = need_gpu()
    w = C.mol_40nuc_160e(n_walkers=64)
    r = torch.tensor(w.r0, device="cuda")
    wk = P.Walkers(P.JAGPSystem(w.system), 64)
    a = wk.eval_batch(r)
    b = wk.eval_batch(r)
    torch.cuda.synchronize()
    for k in ("logabs", "e_loc", "drift"):
        assert torch.equal(a[k], b[k]), k


def test_argument_errors():
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=2)
    import dataclasses
    with pytest.raises(P.QMCError) as ei:
        P.JAGPSystem(dataclasses.replace(w.system, n_up=4, n_dn=6,
                                         unpaired=np.zeros((24, 0))))
    assert ei.value.code == -5   # the majority spin must be labelled up
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, 2)
    with pytest.raises(P.QMCError) as ei:
        wk.propose(0, torch.zeros(2, 3, dtype=torch.float64, device="cuda"))
    assert ei.value.code == -6
    wk.eval_batch(torch.tensor(w.r0, device="cuda"))
    with pytest.raises(P.QMCError) as ei:
        wk.accept(0, torch.ones(2, dtype=torch.uint8, device="cuda"))
    assert ei.value.code == -6
    with pytest.raises(P.QMCError) as ei:
        wk.propose(10, torch.zeros(2, 3, dtype=torch.float64, device="cuda"))
    assert ei.value.code == -1
