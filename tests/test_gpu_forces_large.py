"""The adjoint (qmc_forces) on the 1024-electron workload: 256 nuclei, L = 4096
s,p,d Gaussians, Lambda banded at 8 bohr, W 512 x 512 (blocked inverse).
The basis and Jastrow backward kernels take the electrons in chunks of 256
here (the per-electron sums of the basis backward and the per-nucleus sums of
the Jastrow backward continue across the chunks).

Two walkers: the walker-summed gradients (a vector-Jacobian product with
random weights) against the oracle's reverse-mode autodiff of the plain FP64
definition (Derivatives of energy section), bar 1e-8 of scale as every
adjoint parity test; the summed outputs against the host sum of the
per-walker ones (1e-12 of scale); and central differences of the GPU
evaluation for electron and nuclear coordinates and one exponent, bar
1e-6 * max(1, |fd|).  The differences are fourth order,
(8 (F(x+h) - F(x-h)) - (F(x+2h) - F(x-2h))) / 12h with h = 1e-3: at this size
F (two walkers' log|Psi| and e_L with unit-scale weights) is some 1e4 and its
rounding, some 1e-10, divided by the 2e-5 of a second-order difference at
h = 1e-5 would reach 5e-6; the fourth-order stencil keeps the rounding term
near 1e-7 and its truncation, h^4 F^(5) / 30, below that for exponents up to
20 bohr^-2.
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu
from oracle import jagp as O
from workloads import configs as C

pytestmark = pytest.mark.gpu

KEYS = ("R", "zeta", "lam", "jas", "r")
WK = 2


def _scale_err(a, b):
    return (a - b).abs().max().item() / max(1.0, b.abs().max().item())


@pytest.fixture(scope="module")
def large():
    P = need_gpu()
    w = C.large_256nuc_1024e(n_walkers=WK)
    sysh = P.JAGPSystem(w.system)
    wk = P.Walkers(sysh, WK)
    r = torch.tensor(w.r0[:WK])
    rng = np.random.default_rng(31)
    gl = torch.tensor(rng.normal(size=WK))
    ge = torch.tensor(rng.normal(size=WK))
    yield P, w, sysh, wk, r, gl, ge
    wk.close()
    sysh.close()


def test_large_forces_vjp_matches_oracle(large):
    P, w, sysh, wk, r, gl, ge = large
    summed = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    per = wk.forces(r.cuda(), gl.cuda(), ge.cuda(), per_walker=True)
    torch.cuda.synchronize()
    for k in KEYS:
        a = summed[k].cpu()
        b = per[k].cpu() if k == "r" else per[k].cpu().sum(0)
        err = _scale_err(a, b)
        print(f"[forces 1024e] {k}: summed vs host sum of per-walker {err:.3e}")
        assert err <= 1e-12, (k, err)
    ref = O.forces_vjp(O.from_workload_system(w.system), r, gl, ge)
    for k in KEYS:
        err = _scale_err(summed[k].cpu(), ref[k])
        print(f"[forces 1024e] {k}: vs oracle {err:.3e} (scale {ref[k].abs().max().item():.3e})")
        assert err <= 1e-8, (k, err)


def test_large_forces_match_central_differences(large):
    P, w, sysh, wk, r, gl, ge = large
    g = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    torch.cuda.synchronize()
    wgt_l, wgt_e = gl.cuda(), ge.cuda()

    def F(rr):
        out = wk.eval_batch(rr.cuda())
        return ((wgt_l * out["logabs"]).sum() + (wgt_e * out["e_loc"]).sum()).item()

    h = 1e-3

    def stencil(f):   # f(t) = F at offset t
        return (8.0 * (f(h) - f(-h)) - (f(2 * h) - f(-2 * h))) / (12.0 * h)

    def moved(wi, i, c, t):
        rr = r.clone()
        rr[wi, i, c] += t
        return rr

    # electron coordinates of both spins, in the first and last chunk of 256
    for (wi, i, c) in ((0, 3, 0), (1, 300, 1), (0, 700, 2), (1, 1021, 0)):
        fd = stencil(lambda t: F(moved(wi, i, c, t)))
        got = g["r"][wi, i, c].item()
        print(f"[forces 1024e fd] r[{wi},{i},{c}]: adjoint {got:.10e} fd {fd:.10e}")
        assert abs(got - fd) <= 1e-6 * max(1.0, abs(fd)), (wi, i, c, got, fd)
    # nuclear coordinate and one exponent, through set_params
    s = w.system
    R0 = torch.tensor(s.R, device="cuda")
    z0 = torch.tensor(s.zeta, device="cuda")

    def Fp(R_=None, zeta_=None):
        sysh.set_params(R_, zeta_, None, None)
        v = F(r)
        sysh.set_params(R0, z0, None, None)
        return v

    def shifted(base, ix, t):
        p = base.clone()
        p[ix] += t
        return p

    for name, base, ix in (("R", R0, (200, 2)), ("zeta", z0, (1234,))):
        fd = stencil(lambda t: Fp(**{name + "_": shifted(base, ix, t)}))
        got = g[name][ix].item()
        print(f"[forces 1024e fd] {name}{ix}: adjoint {got:.10e} fd {fd:.10e}")
        assert abs(got - fd) <= 1e-6 * max(1.0, abs(fd)), (name, ix, got, fd)
