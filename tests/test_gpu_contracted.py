"""Contracted (hybrid) orbitals over a primitive basis (Contraction of the
primitive atomic basis section) on the GPU path against the oracle, at the
FP64 bars of the other tests: relative 1e-10 on log|Psi|, E_kin, E_loc and
ratios, 1e-8 on drifts; chains bitwise; an identity contraction reproduces the
uncontracted evaluation bitwise.
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from oracle import lrdmc as L
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cw():
    return C.contracted_4nuc_20e()


def _eval(P, s, r0, Wk, precision=None):
    sysh = P.JAGPSystem(s) if precision is None else P.JAGPSystem(s, precision=precision)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(r0[:Wk], device="cuda")
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    return sysh, wk, r.cpu(), out


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_bf16"])
def test_contracted_eval_matches_oracle(cw, precision):
    P = need_gpu()
    prec = {"fp64": P.QMC_FP64, "mixed": P.QMC_MIXED, "mixed_bf16": P.QMC_MIXED_BF16}[precision]
    _, _, r, out = _eval(P, cw.system, cw.r0, 32, prec)
    ref = O.evaluate(O.from_workload_system(cw.system), r)
    e = {k: rel_err(out[k].cpu(), ref[k]).max().item() for k in ("logabs", "e_kin", "e_loc")}
    d = out["drift"].cpu()
    e_dr = ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[contracted eval {precision}] {e} drift {e_dr:.3e}")
    assert max(e.values()) <= 1e-10 and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


def test_identity_contraction_equals_primitive_basis():
    P = need_gpu()
    w = C.slater_4nuc_20e(n_walkers=16)
    s = w.system
    sc = dataclasses.replace(s, contraction=np.eye(len(s.zeta)))
    a = _eval(P, sc, w.r0, 16)[3]
    b = _eval(P, s, w.r0, 16)[3]
    for k in ("logabs", "sign", "e_kin", "e_loc", "drift"):
        assert torch.equal(a[k].cpu(), b[k].cpu()), k


def test_contracted_propose_ratio_and_drift(cw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, cw.system, cw.r0, 32)
    sy = O.from_workload_system(cw.system)
    for e in (1, 14):
        rn = r[:, e] + torch.tensor(cw.disp[e])
        ratio, dn = wk.propose(e, rn.cuda().contiguous(), drift=True)
        torch.cuda.synchronize()
        assert rel_err(ratio.cpu(), O.move_ratio(sy, r, e, rn)).max().item() <= 1e-10
        r2 = r.clone(); r2[:, e] = rn
        dref = O.evaluate(sy, r2)["drift"][:, e]
        assert ((dn.cpu() - dref).abs() / dref.abs().clamp(min=1.0)).max().item() <= 1e-8


def test_contracted_chain_matches_oracle(cw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, cw.system, cw.r0, 32)
    disp, unif = torch.tensor(cw.disp), torch.tensor(cw.unif)
    wk.vmc_steps(0, disp.cuda(), unif.cuda())
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(cw.system)
    rf, _, accs = O.run_chain(sy, r, disp, unif)
    print(f"[contracted chain] acceptance {accs.double().mean().item():.3f}")
    assert torch.equal(rg, rf)
    assert rel_err(la, O.evaluate(sy, rf)["logabs"]).max().item() <= 1e-10


def test_contracted_mixed_chain_tracks_log_psi(cw):
    # FP32 move rows perturb the ratios (so a decision near the threshold may
    # differ from the FP64 chain); log|Psi| carried through the moves still
    # agrees with a fresh FP64 evaluation at the chain's positions
    P = need_gpu()
    _, wk, r, _ = _eval(P, cw.system, cw.r0, 32, P.QMC_MIXED)
    wk.vmc_steps(0, torch.tensor(cw.disp).cuda(), torch.tensor(cw.unif).cuda())
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    assert not torch.equal(rg, r)
    ref = O.evaluate(O.from_workload_system(cw.system), rg)["logabs"]
    assert rel_err(la, ref).max().item() <= 1e-6


def test_contracted_lattice_hops(cw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, cw.system, cw.r0, 8)
    prm = C.LRDMC_DOUBLE
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(cw.system)
    a_i = L.mesh(sy, r, prm["a"], prm["a_valence"], prm["tf_scale"])
    assert rel_err(g["ratios"].cpu(), L.lattice_ratios(sy, r, a_i)).max().item() <= 1e-10


def _oracle_contraction_grads(sy, r, gl, ge):
    """Autodiff of sum_w (gl log|Psi| + ge e_L) with respect to the dense contraction matrix."""
    Cm = sy.contraction.detach().clone().requires_grad_(True)
    out = O.evaluate(dataclasses.replace(sy, contraction=Cm), r)
    F = (gl * out["logabs"]).sum() + (ge * out["e_loc"]).sum()
    return torch.autograd.grad(F, Cm)[0]


def test_contracted_forces_match_oracle(cw):
    # the adjoint over contracted orbitals: orbital-level products, then the
    # basis backward over the primitives (exponent gradients per primitive)
    P = need_gpu()
    Wk = 6
    _, wk, r, _ = _eval(P, cw.system, cw.r0, Wk)
    sy = O.from_workload_system(cw.system)
    rng = np.random.default_rng(9)
    gl = torch.tensor(rng.normal(size=Wk))
    ge = torch.tensor(rng.normal(size=Wk))
    out = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    torch.cuda.synchronize()
    ref = O.forces_vjp(sy, r, gl, ge)
    assert out["zeta"].shape == (60,) and out["lam"].shape == (28, 28)
    # the coefficients C[mu][c] of the pattern, in the CSR order the binding passed
    sysh = wk.sys
    Cg = _oracle_contraction_grads(sy, r, gl, ge)
    ref["con_coef"] = Cg[torch.tensor(sysh.con_mu), torch.tensor(sysh.con_orb)]
    for k in ("R", "zeta", "lam", "jas", "r", "con_coef"):
        a, b = out[k].cpu(), ref[k]
        err = (a - b).abs().max().item() / max(1.0, b.abs().max().item())
        print(f"[contracted forces] {k}: {err:.3e}")
        assert err <= 1e-8, (k, err)
    # per walker, log|Psi| only
    one = torch.ones(Wk, dtype=torch.float64, device="cuda")
    per = wk.forces(r.cuda(), one, None, per_walker=True)
    torch.cuda.synchronize()
    for w_ in (0, Wk - 1):
        g1 = torch.zeros(Wk, dtype=torch.float64)
        g1[w_] = 1.0
        b = _oracle_contraction_grads(sy, r, g1, torch.zeros(Wk, dtype=torch.float64))
        b = b[torch.tensor(sysh.con_mu), torch.tensor(sysh.con_orb)]
        a = per["con_coef"][w_].cpu()
        assert (a - b).abs().max().item() / max(1.0, b.abs().max().item()) <= 1e-8, w_


def test_contracted_refusals(cw):
    P = need_gpu()
    sysh, wk, r, _ = _eval(P, cw.system, cw.r0, 4)
    # primitive exponents, nuclei and Lambda (over the contracted orbitals) may change
    z2 = cw.system.zeta * 1.05
    R2 = cw.system.R + 0.03
    sysh.set_params(zeta=torch.tensor(z2, device="cuda"), R=torch.tensor(R2, device="cuda"))
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    ref = O.evaluate(O.from_workload_system(dataclasses.replace(cw.system, zeta=z2, R=R2)), r)
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-10
    sysh.set_params(zeta=torch.tensor(cw.system.zeta, device="cuda"), R=torch.tensor(cw.system.R, device="cuda"))
    lam2 = torch.tensor(cw.system.lam * 1.1, device="cuda")
    sysh.set_params(lam=lam2)
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    ref = O.evaluate(O.from_workload_system(dataclasses.replace(cw.system, lam=cw.system.lam * 1.1)), r)
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-10
    # a contraction without coefficients is refused
    with pytest.raises(P.QMCError) as ex:
        P.JAGPSystem(dataclasses.replace(cw.system, contraction=np.zeros_like(cw.system.contraction)))
    assert ex.value.code == -1
