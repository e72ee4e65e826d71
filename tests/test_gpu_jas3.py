"""Jastrow-basis terms (one-body inhomogeneous and three/four-body,
onebody_J_inh and threebody_jastrow) on the GPU path against the oracle, at
the FP64 bars of the other tests: relative 1e-10 on log|Psi|, E_kin and E_loc,
1e-8 on drifts, 1e-10 on ratios; chains bitwise equal; zero coefficients
reproduce the evaluation without a Jastrow basis bitwise.
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
def jw():
    return C.jas3_4nuc_20e()


def _eval(P, s, r0, Wk, precision=None):
    sysh = P.JAGPSystem(s) if precision is None else P.JAGPSystem(s, precision=precision)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(r0[:Wk], device="cuda")
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    return sysh, wk, r.cpu(), out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_jas3_eval_matches_oracle(jw, precision):
    P = need_gpu()
    prec = {"fp64": P.QMC_FP64, "mixed": P.QMC_MIXED}[precision]
    _, _, r, out = _eval(P, jw.system, jw.r0, 32, prec)
    ref = O.evaluate(O.from_workload_system(jw.system), r)
    e = {k: rel_err(out[k].cpu(), ref[k]).max().item() for k in ("logabs", "e_kin", "e_loc")}
    d = out["drift"].cpu()
    e_dr = ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[jas3 eval {precision}] {e} drift {e_dr:.3e}")
    assert max(e.values()) <= 1e-10 and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


def test_jas3_zero_coefficients_equal_plain_jastrow(jw):
    P = need_gpu()
    s = jw.system
    s0 = dataclasses.replace(s, j1_inh=np.zeros_like(s.j1_inh), j3=np.zeros_like(s.j3))
    base = dataclasses.replace(s, jb_center=None, jb_l=None, jb_m=None, jb_radial=None, jb_zeta=None,
                               j1_inh=None, j3=None)
    a = _eval(P, s0, jw.r0, 16)[3]
    b = _eval(P, base, jw.r0, 16)[3]
    for k in ("logabs", "e_kin", "e_loc", "drift"):
        assert torch.equal(a[k].cpu(), b[k].cpu()), k


def test_jas3_propose_ratio_and_drift(jw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, jw.system, jw.r0, 32)
    sy = O.from_workload_system(jw.system)
    for e in (2, 15):
        rn = r[:, e] + torch.tensor(jw.disp[e])
        ratio, dn = wk.propose(e, rn.cuda().contiguous(), drift=True)
        torch.cuda.synchronize()
        assert rel_err(ratio.cpu(), O.move_ratio(sy, r, e, rn)).max().item() <= 1e-10
        r2 = r.clone(); r2[:, e] = rn
        dref = O.evaluate(sy, r2)["drift"][:, e]
        assert ((dn.cpu() - dref).abs() / dref.abs().clamp(min=1.0)).max().item() <= 1e-8


def test_jas3_chain_matches_oracle(jw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, jw.system, jw.r0, 32)
    disp, unif = torch.tensor(jw.disp), torch.tensor(jw.unif)
    wk.vmc_steps(0, disp.cuda(), unif.cuda())
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(jw.system)
    rf, _, accs = O.run_chain(sy, r, disp, unif)
    print(f"[jas3 chain] acceptance {accs.double().mean().item():.3f}")
    assert torch.equal(rg, rf)
    assert rel_err(la, O.evaluate(sy, rf)["logabs"]).max().item() <= 1e-10
    # the maintained Jastrow-basis sums agree with a fresh evaluation: the next
    # proposal's ratio equals the oracle's
    e = 7
    rn = rf[:, e] + torch.tensor(jw.disp[0])
    ratio = wk.propose(e, rn.cuda().contiguous())
    torch.cuda.synchronize()
    assert rel_err(ratio.cpu(), O.move_ratio(sy, rf, e, rn)).max().item() <= 1e-10


def test_jas3_lattice_hops(jw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, jw.system, jw.r0, 8)
    prm = C.LRDMC_DOUBLE
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(jw.system)
    a_i = L.mesh(sy, r, prm["a"], prm["a_valence"], prm["tf_scale"])
    assert rel_err(g["ratios"].cpu(), L.lattice_ratios(sy, r, a_i)).max().item() <= 1e-10


def _oracle_j3_param_grads(sy, r, gl, ge):
    """Autodiff of sum_w (gl log|Psi| + ge e_L) with respect to the Jastrow-basis
    coefficients and exponents (same-spin blocks symmetrised)."""
    j1 = sy.j1_inh.detach().clone().requires_grad_(True)
    j3 = sy.j3.detach().clone().requires_grad_(True)
    jz = sy.jb_zeta.detach().clone().requires_grad_(True)
    sw = dataclasses.replace(sy, j1_inh=j1, j3=j3, jb_zeta=jz)
    out = O.evaluate(sw, r)
    F = (gl * out["logabs"] + ge * out["e_loc"]).sum()
    g1, g3, gz = torch.autograd.grad(F, [j1, j3, jz])
    g3 = g3.clone()
    g3[0] = 0.5 * (g3[0] + g3[0].T)
    g3[1] = 0.5 * (g3[1] + g3[1].T)
    return g1, g3, gz


def test_jas3_forces_match_oracle(jw):
    # the adjoint through the Jastrow-basis terms (positions, nuclei, coefficients, exponents)
    P = need_gpu()
    Wk = 6
    _, wk, r, _ = _eval(P, jw.system, jw.r0, Wk)
    sy = O.from_workload_system(jw.system)
    rng = np.random.default_rng(21)
    gl = torch.tensor(rng.normal(size=Wk))
    ge = torch.tensor(rng.normal(size=Wk))
    out = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    torch.cuda.synchronize()
    ref = O.forces_vjp(sy, r, gl, ge)
    g1, g3, gz = _oracle_j3_param_grads(sy, r, gl, ge)
    ref.update(j1_inh=g1, j3=g3, jb_zeta=gz)
    for k in ("R", "zeta", "lam", "jas", "r", "j1_inh", "j3", "jb_zeta"):
        a, b = out[k].cpu(), ref[k]
        err = (a - b).abs().max().item() / max(1.0, b.abs().max().item())
        print(f"[jas3 forces] {k}: {err:.3e}")
        assert err <= 1e-8, (k, err)
    # per walker, log|Psi| only: the coefficients' part equals the closed-form log-derivatives
    one = torch.ones(Wk, dtype=torch.float64, device="cuda")
    per = wk.forces(r.cuda(), one, None, per_walker=True)
    dm, dM = wk.jastrow_basis_logderiv()
    torch.cuda.synchronize()
    assert ((per["j1_inh"] - dm).abs().max() / dm.abs().max()).item() <= 1e-12
    assert ((per["j3"] - dM).abs().max() / dM.abs().max()).item() <= 1e-12


def test_jas3_refusals(jw):
    P = need_gpu()
    s = jw.system
    bad = s.j3.copy()
    bad[0, 0, 1] += 1.0
    with pytest.raises(P.QMCError) as ex:
        P.JAGPSystem(dataclasses.replace(s, j3=bad))
    assert ex.value.code == -1


def _oracle_logderiv(sy, r):
    """Per-walker autodiff of log|Psi| with respect to j1_inh and j3 (same-spin
    blocks symmetrised: the gradient with respect to a symmetric matrix)."""
    dm, dM = [], []
    for w in range(r.shape[0]):
        j1 = sy.j1_inh.detach().clone().requires_grad_(True)
        j3 = sy.j3.detach().clone().requires_grad_(True)
        sw = dataclasses.replace(sy, j1_inh=j1, j3=j3)
        lp, _ = O.log_psi(sw, r[w:w + 1])
        g1, g3 = torch.autograd.grad(lp.sum(), [j1, j3])
        g3 = g3.clone()
        g3[0] = 0.5 * (g3[0] + g3[0].T)
        g3[1] = 0.5 * (g3[1] + g3[1].T)
        dm.append(g1)
        dM.append(g3)
    return torch.stack(dm), torch.stack(dM)


def test_jas3_logderiv_matches_oracle(jw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, jw.system, jw.r0, 8)
    sy = O.from_workload_system(jw.system)
    dm, dM = wk.jastrow_basis_logderiv()
    torch.cuda.synchronize()
    rm, rM = _oracle_logderiv(sy, r)
    e1 = ((dm.cpu() - rm).abs().max() / rm.abs().max()).item()
    e2 = ((dM.cpu() - rM).abs().max() / rM.abs().max()).item()
    print(f"[jas3 logderiv] j1_inh {e1:.3e} j3 {e2:.3e}")
    assert e1 <= 1e-12 and e2 <= 1e-12
    # after a chain: the maintained chi rows give the derivatives at the new positions
    disp, unif = torch.tensor(jw.disp[:40, :8]).contiguous(), torch.tensor(jw.unif[:40, :8]).contiguous()
    wk.vmc_steps(0, disp.cuda(), unif.cuda())
    dm, dM = wk.jastrow_basis_logderiv()
    rg = wk.read(P.STATE_R).cpu()
    torch.cuda.synchronize()
    rm, rM = _oracle_logderiv(sy, rg)
    assert ((dm.cpu() - rm).abs().max() / rm.abs().max()).item() <= 1e-10
    assert ((dM.cpu() - rM).abs().max() / rM.abs().max()).item() <= 1e-10


def test_jas3_parameter_updates(jw):
    # moved nuclei carry the Jastrow basis with them; new coefficients and exponents
    P = need_gpu()
    sysh, wk, r, _ = _eval(P, jw.system, jw.r0, 8)
    s = jw.system
    rng = np.random.default_rng(33)
    R2 = s.R + 0.05 * rng.standard_normal(s.R.shape)
    sysh.set_params(R=torch.tensor(R2, device="cuda"))
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    s2 = dataclasses.replace(s, R=R2)
    ref = O.evaluate(O.from_workload_system(s2), r)
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-10
    assert rel_err(out["logabs"].cpu(), ref["logabs"]).max().item() <= 1e-10
    j1 = s.j1_inh * 1.3
    j3 = s.j3 + 0.02 * np.stack([C._sym_gaussian(rng, len(s.jb_zeta), 1.0), C._sym_gaussian(rng, len(s.jb_zeta), 1.0),
                                 rng.standard_normal((len(s.jb_zeta),) * 2)])
    jz = s.jb_zeta * 1.1
    sysh.set_jastrow_basis(torch.tensor(j1, device="cuda"), torch.tensor(j3, device="cuda"),
                           torch.tensor(jz, device="cuda"))
    with pytest.raises(P.QMCError) as ex:      # walkers must re-evaluate after a parameter change
        wk.propose(0, r[:, 0].cuda().contiguous())
    assert ex.value.code == -6
    out = wk.eval_batch(r.cuda())
    torch.cuda.synchronize()
    s3 = dataclasses.replace(s2, j1_inh=j1, j3=j3, jb_zeta=jz)
    ref = O.evaluate(O.from_workload_system(s3), r)
    assert rel_err(out["e_loc"].cpu(), ref["e_loc"]).max().item() <= 1e-10
    assert rel_err(out["logabs"].cpu(), ref["logabs"]).max().item() <= 1e-10

