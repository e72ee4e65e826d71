"""Parity of the hand-written adjoint (qmc_forces) with the oracle's gradients
(reverse-mode autodiff of the plain FP64 definition) and with central
differences of the GPU's own evaluation.

Bars: against the oracle, |g_gpu - g_ref| <= 1e-8 * max(1, max|g_ref|) per
output array (FP64 on both sides; the tolerance leaves room for the condition
of W, which enters through W^{-1} twice in the local-energy gradient).  Against
central differences with h = 1e-5: 1e-6 * max(1, |g_fd|) (the gradient bar).
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

KEYS = ("R", "zeta", "lam", "jas", "r")


def _cmp(gpu, ref, tol=1e-8, label=""):
    for k in KEYS:
        a, b = gpu[k].cpu(), ref[k]
        scale = max(1.0, b.abs().max().item())
        err = (a - b).abs().max().item() / scale
        print(f"[forces {label}] {k}: max err / scale = {err:.3e} (scale {scale:.3e})")
        assert err <= tol, (label, k, err)


def _setup(P, w, Wk):
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, Wk)
    return wk, O.from_workload_system(w.system), torch.tensor(w.r0[:Wk])


@pytest.mark.parametrize("name", ["tiny", "forces80"])
def test_forces_vjp_matches_oracle(name):
    P = need_gpu()
    if name == "tiny":
        w, Wk = C.tiny_3nuc_10e(), 8
    else:
        w, Wk = C.forces_20nuc_80e(n_walkers=4), 4
    wk, sy, r = _setup(P, w, Wk)
    rng = np.random.default_rng(3)
    gl = torch.tensor(rng.normal(size=Wk))
    ge = torch.tensor(rng.normal(size=Wk))
    out = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    torch.cuda.synchronize()
    ref = O.forces_vjp(sy, r, gl, ge)
    _cmp(out, ref, label=name)


def test_forces_per_walker_matches_oracle():
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=3)
    wk, sy, r = _setup(P, w, 3)
    ref = O.forces_per_walker(sy, r)
    one = torch.ones(3, dtype=torch.float64, device="cuda")
    for which, (gl, ge) in enumerate(((one, None), (None, one))):
        out = wk.forces(r.cuda(), gl, ge, per_walker=True)
        torch.cuda.synchronize()
        _cmp(out, {k: ref[k][which] for k in KEYS}, label=f"per-walker {'logpsi' if which == 0 else 'eloc'}")


def test_forces_translation_sum_rule_and_drift():
    P = need_gpu()
    w = C.forces_20nuc_80e(n_walkers=4)
    wk, sy, r = _setup(P, w, 4)
    one = torch.ones(4, dtype=torch.float64, device="cuda")
    out = wk.forces(r.cuda(), one, None, per_walker=True)
    ev = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    # d log|Psi| / d r_i is the drift
    assert torch.allclose(out["r"].cpu(), ev["drift"].cpu(), rtol=1e-10, atol=1e-10)
    for gl, ge in ((one, None), (None, one)):
        out = wk.forces(r.cuda(), gl, ge, per_walker=True)
        torch.cuda.synchronize()
        tot = out["R"].cpu().sum(1) + out["r"].cpu().sum(1)
        scale = max(1.0, out["R"].abs().max().item())
        assert tot.abs().max().item() <= 1e-9 * scale


def test_forces_positions_match_central_differences_of_gpu_eval():
    P = need_gpu()
    w = C.forces_20nuc_80e(n_walkers=4)
    wk, sy, r = _setup(P, w, 4)
    one = torch.ones(4, dtype=torch.float64, device="cuda")
    g = wk.forces(r.cuda(), None, one, per_walker=True)["r"].cpu()
    h = 1e-5
    for (i, c) in ((0, 0), (17, 1), (55, 2), (79, 0)):
        rp = r.clone(); rp[:, i, c] += h
        rm = r.clone(); rm[:, i, c] -= h
        ep = wk.eval_batch(rp.cuda())["e_loc"].cpu()
        em = wk.eval_batch(rm.cuda())["e_loc"].cpu()
        torch.cuda.synchronize()
        fd = (ep - em) / (2 * h)
        err = ((g[:, i, c] - fd).abs() / fd.abs().clamp(min=1.0)).max().item()
        assert err <= 1e-6, (i, c, err)


def test_autograd_function_matches_oracle_and_parameter_differences():
    P = need_gpu()
    w = C.forces_20nuc_80e(n_walkers=4)
    s = w.system
    wk, sy, r = _setup(P, w, 4)
    dev = "cuda"
    R = torch.tensor(s.R, device=dev, requires_grad=True)
    zeta = torch.tensor(s.zeta, device=dev, requires_grad=True)
    lam = torch.tensor(s.lam, device=dev, requires_grad=True)
    jas = torch.tensor(s.jastrow_params, device=dev, requires_grad=True)
    rr = r.clone().to(dev).requires_grad_(True)
    la, el = P.JAGPFunction.apply(wk, rr, R, zeta, lam, jas)
    wts = torch.tensor([0.3, -1.0, 0.7, 0.2], dtype=torch.float64, device=dev)
    loss = (wts * la).sum() + (wts.flip(0) * el).sum()
    loss.backward()
    torch.cuda.synchronize()
    ref = O.forces_vjp(sy, r, wts.cpu(), wts.flip(0).cpu())
    got = dict(R=R.grad, zeta=zeta.grad, lam=lam.grad, jas=jas.grad, r=rr.grad)
    _cmp(got, ref, label="autograd")

    # central differences of the GPU evaluation (h = 1e-5) through set_params
    def F(R_=None, zeta_=None, lam_=None, jas_=None):
        wk.sys.set_params(R_, zeta_, lam_, jas_)
        out = wk.eval_batch(r.to(dev))
        v = ((wts * out["logabs"]).sum() + (wts.flip(0) * out["e_loc"]).sum()).item()
        wk.sys.set_params(R.detach(), zeta.detach(), lam.detach(), jas.detach())
        return v

    h = 1e-5
    for name, base, ix in (("R", R, (3, 1)), ("zeta", zeta, (17,)), ("lam", lam, (5, 40)), ("jas", jas, (21,)),
                           ("jas", jas, (24,))):
        p = base.detach().clone(); p[ix] += h
        fp = F(**{name + "_": p})
        p = base.detach().clone(); p[ix] -= h
        fm = F(**{name + "_": p})
        fd = (fp - fm) / (2 * h)
        g = got[name][ix].item()
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (name, ix, g, fd)
