"""Slater-type basis functions (eq. slater) on the GPU path, in a basis that
mixes them with Gaussians (s, p and d shells of both kinds): evaluation,
single-electron moves, lattice hops and the adjoint against the oracle, at
the FP64 bars of the Gaussian tests (relative 1e-10 on log|Psi| and E_loc,
1e-8 on the drift, ratios 1e-10, gradients 1e-8 of scale against the oracle's
autodiff and 1e-6 against central differences of the GPU's own evaluation).
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from oracle import lrdmc as L
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def slater():
    return C.slater_4nuc_20e()


def _eval(P, w, Wk, precision=None):
    sysh = P.JAGPSystem(w.system) if precision is None else P.JAGPSystem(w.system, precision=precision)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0[:Wk], device="cuda")
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    return sysh, wk, r.cpu(), out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_slater_eval_matches_oracle(slater, precision):
    P = need_gpu()
    prec = {"fp64": P.QMC_FP64, "mixed": P.QMC_MIXED}[precision]
    _, _, r, out = _eval(P, slater, 32, prec)
    ref = O.evaluate(O.from_workload_system(slater.system), r)
    e_la = rel_err(out["logabs"].cpu(), ref["logabs"]).max().item()
    e_ek = rel_err(out["e_kin"].cpu(), ref["e_kin"]).max().item()
    e_el = rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item()
    d = out["drift"].cpu()
    e_dr = ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[slater eval {precision}] logabs {e_la:.3e} e_kin {e_ek:.3e} e_loc {e_el:.3e} drift {e_dr:.3e}")
    # the mixed evaluation's products carry the int8 digit expansion's error
    # (about 1e-13 of max|Phi| max|Lambda| L), amplified by cond(W): its bar is 1e-8
    bar = 1e-10 if precision == "fp64" else 1e-8
    assert e_la <= bar and e_ek <= bar and e_el <= bar and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


def test_slater_chain_matches_oracle(slater):
    P = need_gpu()
    _, wk, r, _ = _eval(P, slater, 32)
    disp, unif = torch.tensor(slater.disp), torch.tensor(slater.unif)
    cnt = torch.zeros(32, dtype=torch.int32, device="cuda")
    wk.vmc_steps(0, disp.cuda(), unif.cuda(), cnt)
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(slater.system)
    rf, _, accs = O.run_chain(sy, r, disp, unif)
    print(f"[slater chain] acceptance {accs.double().mean().item():.3f}")
    assert torch.equal(rg, rf)
    assert rel_err(la, O.evaluate(sy, rf)["logabs"]).max().item() <= 1e-10
    assert int(cnt.sum()) == int(accs.sum())


def test_slater_lattice_hops_match_oracle(slater):
    P = need_gpu()
    _, wk, r, _ = _eval(P, slater, 8)
    prm = C.LRDMC_DOUBLE
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(slater.system)
    a_i = L.mesh(sy, r, prm["a"], prm["a_valence"], prm["tf_scale"])
    ref = L.lattice_ratios(sy, r, a_i)
    e = rel_err(g["ratios"].cpu(), ref).max().item()
    print(f"[slater hops] ratio rel err {e:.3e}")
    assert e <= 1e-10


def test_slater_forces_match_oracle_and_differences(slater):
    P = need_gpu()
    Wk = 4
    sysh, wk, r, _ = _eval(P, slater, Wk)
    rng = np.random.default_rng(8)
    gl = torch.tensor(rng.normal(size=Wk))
    ge = torch.tensor(rng.normal(size=Wk))
    out = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    torch.cuda.synchronize()
    sy = O.from_workload_system(slater.system)
    ref = O.forces_vjp(sy, r, gl, ge)
    for k in ("R", "zeta", "lam", "jas", "r"):
        a, b = out[k].cpu(), ref[k]
        scale = max(1.0, b.abs().max().item())
        err = (a - b).abs().max().item() / scale
        print(f"[slater forces] {k}: {err:.3e}")
        assert err <= 1e-8, k
    # exponents of Slater functions against central differences of the GPU evaluation
    s = slater.system
    zeta0 = torch.tensor(s.zeta, device="cuda")
    h = 1e-5
    rr = r.cuda()
    for mu in np.nonzero(s.radial)[0][[0, 7, 20]]:
        f = []
        for sgn in (1.0, -1.0):
            z = zeta0.clone()
            z[mu] += sgn * h
            sysh.set_params(zeta=z)
            o = wk.eval_batch(rr, drift=False)
            f.append((gl.cuda() * o["logabs"] + ge.cuda() * o["e_loc"]).sum().item())
        sysh.set_params(zeta=zeta0)
        fd = (f[0] - f[1]) / (2 * h)
        g = out["zeta"][mu].item()
        assert abs(g - fd) <= 1e-6 * max(1.0, abs(fd)), (mu, g, fd)
