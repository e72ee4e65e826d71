"""Force and optimisation estimators on the GPU path (qmc_swct, qmc_reweight,
qmc_sr_step) against the oracle, on the same seeded inputs.

Bars (FP64 on both sides):
  * space warp: |out - ref| <= 1e-12 * max(1, max|ref|) on given partials (the
    kernel and the oracle sum the same products in different orders); on the
    GPU's own per-walker partials the adjoint's 1e-8 bar carries through;
  * reweighting factor: relative 1e-10 on R and the weight (R depends on
    W^{-1}, whose relative error is about cond(W) times the rounding unit);
  * SR: the force f within 1e-12 * max|f|; delta within 1e-9 * max|delta| of
    the oracle's direct solve (CG stopped at |r| <= 1e-14 |f|, S' well
    conditioned by construction); repeated calls bitwise equal.
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import estimators as E
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

THETA = 3.0 / 8.0


def _scaled_err(a, b):
    return ((a - b).abs().max() / max(1.0, b.abs().max().item())).item()


@pytest.mark.parametrize("name", ["tiny", "forces80"])
@pytest.mark.parametrize("jacobian", [False, True])
def test_swct_matches_oracle_on_given_partials(name, jacobian):
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=6) if name == "tiny" else C.forces_20nuc_80e(n_walkers=5)
    sysh = P.JAGPSystem(w.system)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)
    Wk, N, A = r.shape[0], r.shape[1], sy.R.shape[0]
    g = torch.Generator().manual_seed(11)
    dR = torch.randn(Wk, A, 3, generator=g, dtype=torch.float64)
    dr = torch.randn(Wk, N, 3, generator=g, dtype=torch.float64)
    out = P.swct(sysh, r.cuda(), dR.cuda(), dr.cuda(), jacobian=jacobian)
    torch.cuda.synchronize()
    ref = E.swct_total(sy, r, dR, dr, jacobian=jacobian)
    err = _scaled_err(out.cpu(), ref)
    print(f"[swct {name} jac={jacobian}] err {err:.3e}")
    assert err <= 1e-12


def test_swct_on_gpu_partials_matches_oracle_total_derivatives():
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=3)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, 3)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0[:3])
    pw = O.forces_per_walker(sy, r)
    one = torch.ones(3, dtype=torch.float64, device="cuda")
    for which, (gl, ge) in enumerate(((one, None), (None, one))):
        g = wk.forces(r.cuda(), gl, ge, per_walker=True)
        tot = P.swct(sysh, r.cuda(), g["R"], g["r"], jacobian=(which == 0))
        torch.cuda.synchronize()
        ref = E.swct_total(sy, r, pw["R"][which], pw["r"][which], jacobian=(which == 0))
        err = _scaled_err(tot.cpu(), ref)
        print(f"[swct gpu partials {'logpsi' if which == 0 else 'eloc'}] err {err:.3e}")
        assert err <= 1e-8
        # the total force is a sum over nuclei of zero (translation invariance)
        assert tot.sum(1).abs().max().item() <= 1e-8 * max(1.0, ref.abs().max().item())


@pytest.mark.parametrize("name", ["tiny", "mol160"])
def test_reweight_matches_oracle(name):
    P = need_gpu()
    if name == "tiny":
        w, Wk = C.tiny_3nuc_10e(n_walkers=16), 16
    else:
        w, Wk = C.mol_40nuc_160e(n_walkers=8), 8
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, Wk)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0[:Wk])
    wk.eval_batch(r.cuda())
    R_ref, _ = E.reweight(sy, r, THETA, 0.0)
    eps = float(R_ref.median())            # half of the walkers fall below eps
    R, wt = P.reweight(wk, THETA, eps)
    torch.cuda.synchronize()
    R_ref, wt_ref = E.reweight(sy, r, THETA, eps)
    e1, e2 = rel_err(R.cpu(), R_ref).max().item(), rel_err(wt.cpu(), wt_ref).max().item()
    print(f"[reweight {name}] R {e1:.3e} weight {e2:.3e}")
    assert e1 <= 1e-10 and e2 <= 1e-10
    assert (wt_ref < 1).any() and (wt_ref == 1).any()


def test_reweight_needs_fresh_evaluation():
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=4)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, 4)
    r = torch.tensor(w.r0[:4]).cuda()
    with pytest.raises(P.QMCError):
        P.reweight(wk, THETA, 0.0)          # never evaluated
    wk.eval_batch(r)
    P.reweight(wk, THETA, 0.0)
    rn = (r[:, 0] + 0.1).contiguous()
    wk.propose(0, rn)
    wk.accept(0, torch.ones(4, dtype=torch.uint8, device="cuda"))
    with pytest.raises(P.QMCError):
        P.reweight(wk, THETA, 0.0)          # W^{-1} of the evaluation is stale
    with pytest.raises(P.QMCError):
        P.reweight(wk, -1.0, 0.0)


def _sr_inputs(M, Pn, seed, weighted):
    g = torch.Generator().manual_seed(seed)
    # correlated columns with spread-out scales, as logarithmic derivatives have
    B = torch.randn(Pn, Pn, generator=g, dtype=torch.float64) / Pn ** 0.5 + torch.eye(Pn, dtype=torch.float64)
    Ok = torch.randn(M, Pn, generator=g, dtype=torch.float64) @ B
    Ok = Ok * torch.logspace(-1, 1, Pn, dtype=torch.float64) + 0.3
    el = -5.0 + torch.randn(M, generator=g, dtype=torch.float64) + 0.5 * Ok[:, 0]
    wts = 0.5 + torch.rand(M, generator=g, dtype=torch.float64) if weighted else None
    return Ok, el, wts


@pytest.mark.parametrize("M,Pn,weighted", [(200, 50, False), (257, 300, True), (64, 1, True), (1000, 513, False)])
def test_sr_step_matches_direct_solve(M, Pn, weighted):
    P = need_gpu()
    Ok, el, wts = _sr_inputs(M, Pn, 5 + Pn, weighted)
    eps = 1e-3
    d_ref, f_ref, _ = E.sr_step(Ok, el, eps, wts)
    cu = lambda t: None if t is None else t.cuda()
    delta, f, res = P.sr_step(cu(Ok), cu(el), eps, cu(wts), max_iter=4 * Pn + 20, tol=1e-14)
    torch.cuda.synchronize()
    ef = ((f.cpu() - f_ref).abs().max() / f_ref.abs().max()).item()
    ed = ((delta.cpu() - d_ref).abs().max() / d_ref.abs().max()).item()
    print(f"[sr M={M} P={Pn} w={weighted}] f {ef:.3e} delta {ed:.3e} residual {res.item():.3e}")
    assert ef <= 1e-12 and ed <= 1e-9
    assert res.item() <= 1e-13
    d2, _, _ = P.sr_step(cu(Ok), cu(el), eps, cu(wts), max_iter=4 * Pn + 20, tol=1e-14)
    assert torch.equal(delta, d2)


def test_sr_step_edge_cases():
    P = need_gpu()
    Ok, el, _ = _sr_inputs(40, 12, 3, False)
    delta, f, res = P.sr_step(Ok.cuda(), el.cuda(), 1e-3, None, max_iter=0)
    torch.cuda.synchronize()
    assert torch.equal(delta.cpu(), torch.zeros(12, dtype=torch.float64)) and res.item() == 1.0
    _, f_ref, _ = E.sr_step(Ok, el, 1e-3)
    assert ((f.cpu() - f_ref).abs().max() / f_ref.abs().max()).item() <= 1e-12
    # constant local energy: zero force, zero step, stops before the first iteration
    delta, f, res = P.sr_step(Ok.cuda(), torch.full((40,), -3.0, dtype=torch.float64, device="cuda"), 1e-3)
    torch.cuda.synchronize()
    assert f.abs().max().item() <= 1e-12 and delta.abs().max().item() <= 1e-12
    with pytest.raises(P.QMCError):
        P.sr_step(Ok.cuda(), el.cuda(), -1.0)
    lib = P.load()
    assert lib.qmc_sr_workspace_size(0, 5) == 0


def test_sr_step_on_gpu_log_derivatives():
    # O_k from the adjoint (per-walker derivatives of log|Psi| with respect to
    # the exponents and Jastrow parameters), e_L from the evaluation
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=48)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, 48)
    r = torch.tensor(w.r0[:48])
    out = wk.eval_batch(r.cuda())
    g = wk.forces(r.cuda(), torch.ones(48, dtype=torch.float64, device="cuda"), None, per_walker=True)
    Ok = torch.cat([g["zeta"], g["jas"]], dim=1).contiguous()
    el = out["e_loc"]
    delta, f, res = P.sr_step(Ok, el, 1e-2, None, max_iter=400, tol=1e-14)
    torch.cuda.synchronize()
    d_ref, f_ref, _ = E.sr_step(Ok.cpu(), el.cpu(), 1e-2)
    ef = ((f.cpu() - f_ref).abs().max() / f_ref.abs().max()).item()
    ed = ((delta.cpu() - d_ref).abs().max() / d_ref.abs().max()).item()
    print(f"[sr adjoint O] f {ef:.3e} delta {ed:.3e} residual {res.item():.3e}")
    assert ef <= 1e-12 and ed <= 1e-8
