"""Spin-polarized geminal with unpaired orbitals (eq:wfAGPunpaired) on the GPU
path against the oracle: W is n_up x n_up with n_up - n_dn columns
psi(r_i) . U[:, l].  Bars as for the paired systems: relative 1e-10 on
log|Psi|, E_kin, E_loc and ratios, 1e-8 on drifts; chains bitwise.
"""
import dataclasses

import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import estimators as E
from oracle import jagp as O
from oracle import lrdmc as L
from workloads import configs as C

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pw():
    return C.polarized_4nuc_20e()


def _eval(P, s, r0, Wk, precision=None):
    sysh = P.JAGPSystem(s) if precision is None else P.JAGPSystem(s, precision=precision)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(r0[:Wk], device="cuda")
    out = wk.eval_batch(r)
    torch.cuda.synchronize()
    return sysh, wk, r.cpu(), out


def _check_eval(out, ref, label):
    e = {k: rel_err(out[k].cpu(), ref[k]).max().item() for k in ("logabs", "e_kin", "e_loc")}
    d = out["drift"].cpu()
    e_dr = ((d - ref["drift"]).abs() / ref["drift"].abs().clamp(min=1.0)).max().item()
    print(f"[polarized eval {label}] {e} drift {e_dr:.3e}")
    assert max(e.values()) <= 1e-10 and e_dr <= 1e-8
    assert torch.equal(out["sign"].cpu(), ref["sign"])


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_bf16"])
def test_polarized_eval_matches_oracle(pw, precision):
    P = need_gpu()
    prec = {"fp64": P.QMC_FP64, "mixed": P.QMC_MIXED, "mixed_bf16": P.QMC_MIXED_BF16}[precision]
    _, wk, r, out = _eval(P, pw.system, pw.r0, 32, prec)
    sy = O.from_workload_system(pw.system)
    _check_eval(out, O.evaluate(sy, r), precision)
    if precision == "fp64":
        W = wk.read(P.STATE_W).cpu()
        Wref = O.geminal(sy, O.agp_basis(sy, r)[0])
        assert W.shape == (32, 11, 11)
        assert ((W - Wref).abs().max() / Wref.abs().max()).item() <= 1e-13


def test_polarized_propose_ratio_and_drift(pw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, pw.system, pw.r0, 32)
    sy = O.from_workload_system(pw.system)
    for e in (0, 10, 11, 19):   # up (paired and unpaired columns change), down
        rn = r[:, e] + torch.tensor(pw.disp[e])
        ratio, dn = wk.propose(e, rn.cuda().contiguous(), drift=True)
        torch.cuda.synchronize()
        assert rel_err(ratio.cpu(), O.move_ratio(sy, r, e, rn)).max().item() <= 1e-10, e
        r2 = r.clone(); r2[:, e] = rn
        dref = O.evaluate(sy, r2)["drift"][:, e]
        assert ((dn.cpu() - dref).abs() / dref.abs().clamp(min=1.0)).max().item() <= 1e-8, e


def test_polarized_chain_matches_oracle(pw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, pw.system, pw.r0, 32)
    disp, unif = torch.tensor(pw.disp), torch.tensor(pw.unif)
    wk.vmc_steps(0, disp.cuda(), unif.cuda())
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    sy = O.from_workload_system(pw.system)
    rf, _, accs = O.run_chain(sy, r, disp, unif)
    print(f"[polarized chain] acceptance {accs.double().mean().item():.3f}")
    assert torch.equal(rg, rf)
    assert rel_err(la, O.evaluate(sy, rf)["logabs"]).max().item() <= 1e-10
    # the inverse carried through the delayed updates
    A = wk.read(P.STATE_AINV).cpu()
    Aref = torch.linalg.inv(O.geminal(sy, O.agp_basis(sy, rf)[0]))
    assert ((A - Aref).abs().max() / Aref.abs().max()).item() <= 1e-9


def test_polarized_mixed_chain_tracks_log_psi(pw):
    # FP32 rows, including the unpaired orbitals' rows, in the proposals
    P = need_gpu()
    _, wk, r, _ = _eval(P, pw.system, pw.r0, 32, P.QMC_MIXED)
    wk.vmc_steps(0, torch.tensor(pw.disp).cuda(), torch.tensor(pw.unif).cuda())
    rg = wk.read(P.STATE_R).cpu()
    la = wk.read(P.STATE_LOGABS).cpu()
    torch.cuda.synchronize()
    ref = O.evaluate(O.from_workload_system(pw.system), rg)["logabs"]
    assert rel_err(la, ref).max().item() <= 1e-6


def test_polarized_lattice_hops(pw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, pw.system, pw.r0, 8)
    prm = C.LRDMC_DOUBLE
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(pw.system)
    a_i = L.mesh(sy, r, prm["a"], prm["a_valence"], prm["tf_scale"])
    assert rel_err(g["ratios"].cpu(), L.lattice_ratios(sy, r, a_i)).max().item() <= 1e-10


def test_polarized_reweight(pw):
    P = need_gpu()
    _, wk, r, _ = _eval(P, pw.system, pw.r0, 16)
    R, wt = P.reweight(wk, 3.0 / 8.0, 0.0)
    torch.cuda.synchronize()
    R_ref, _ = E.reweight(O.from_workload_system(pw.system), r, 3.0 / 8.0, 0.0)
    assert ((R.cpu() - R_ref).abs() / R_ref.abs()).max().item() <= 1e-10


def test_polarized_contracted_and_jastrow_basis():
    # unpaired orbitals over contracted orbitals, with a Jastrow basis
    P = need_gpu()
    w = C.contracted_4nuc_20e(n_walkers=16)
    rng = np.random.default_rng(23)
    s = dataclasses.replace(w.system, n_up=11, n_dn=9,
                            unpaired=rng.standard_normal((w.system.lam.shape[0], 2)) / 5.0)
    s = C.add_jastrow_basis(s, rng)
    r0 = C.random_positions(31, s, 16)
    _, wk, r, out = _eval(P, s, r0, 16)
    sy = O.from_workload_system(s)
    _check_eval(out, O.evaluate(sy, r), "contracted+J3")
    rn = r[:, 4] + 0.2
    ratio = wk.propose(4, rn.cuda().contiguous())
    torch.cuda.synchronize()
    assert rel_err(ratio.cpu(), O.move_ratio(sy, r, 4, rn)).max().item() <= 1e-10


def _oracle_unpaired_grads(sy, r, gl, ge):
    """Autodiff of sum_w (gl log|Psi| + ge e_L) with respect to the unpaired orbitals U [L, k]."""
    U = sy.unpaired.detach().clone().requires_grad_(True)
    out = O.evaluate(dataclasses.replace(sy, unpaired=U), r)
    F = (gl * out["logabs"]).sum() + (ge * out["e_loc"]).sum()
    return torch.autograd.grad(F, U)[0]


def test_polarized_forces_match_oracle(pw):
    # the adjoint with unpaired orbitals: G_W's unpaired columns feed dF/dPhi_up
    P = need_gpu()
    Wk = 6
    _, wk, r, _ = _eval(P, pw.system, pw.r0, Wk)
    sy = O.from_workload_system(pw.system)
    rng = np.random.default_rng(5)
    gl = torch.tensor(rng.normal(size=Wk))
    ge = torch.tensor(rng.normal(size=Wk))
    out = wk.forces(r.cuda(), gl.cuda(), ge.cuda())
    torch.cuda.synchronize()
    ref = O.forces_vjp(sy, r, gl, ge)
    ref["unpaired"] = _oracle_unpaired_grads(sy, r, gl, ge)
    for k in ("R", "zeta", "lam", "jas", "r", "unpaired"):
        a, b = out[k].cpu(), ref[k]
        err = (a - b).abs().max().item() / max(1.0, b.abs().max().item())
        print(f"[polarized forces] {k}: {err:.3e}")
        assert err <= 1e-8, (k, err)
    one = torch.ones(Wk, dtype=torch.float64, device="cuda")
    per = wk.forces(r.cuda(), one, None, per_walker=True)
    pref = O.forces_per_walker(sy, r)
    for k in ("zeta", "jas"):
        a, b = per[k].cpu(), pref[k][0]
        assert (a - b).abs().max().item() / max(1.0, b.abs().max().item()) <= 1e-8, k
    for w_ in (0, Wk - 1):   # log|Psi| of one walker with respect to U
        g1 = torch.zeros(Wk, dtype=torch.float64)
        g1[w_] = 1.0
        b = _oracle_unpaired_grads(sy, r, g1, torch.zeros(Wk, dtype=torch.float64))
        a = per["unpaired"][w_].cpu()
        assert (a - b).abs().max().item() / max(1.0, b.abs().max().item()) <= 1e-8, w_


def test_fully_polarized_determinant():
    # n_dn = 0: W = Phi_up U, a Slater determinant of the k = n_up unpaired orbitals
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=8, n_steps=60)
    L_ = len(w.system.lam)
    rng = np.random.default_rng(3)
    s = dataclasses.replace(w.system, n_up=4, n_dn=0, unpaired=rng.standard_normal((L_, 4)) / np.sqrt(L_))
    r0 = C.random_positions(5, s, 8)
    _, wk, r, out = _eval(P, s, r0, 8)
    sy = O.from_workload_system(s)
    _check_eval(out, O.evaluate(sy, r), "n_dn = 0")
    disp = torch.tensor(w.disp[:60, :8, :]).contiguous()
    unif = torch.tensor(w.unif[:60, :8]).contiguous()
    wk.vmc_steps(0, disp.cuda(), unif.cuda())
    rg = wk.read(P.STATE_R).cpu()
    torch.cuda.synchronize()
    rf, _, _ = O.run_chain(sy, r, disp, unif)
    assert torch.equal(rg, rf)
    one = torch.ones(8, dtype=torch.float64, device="cuda")
    g = wk.forces(rf.cuda(), one, one)
    torch.cuda.synchronize()
    ref = O.forces_vjp(sy, rf, torch.ones(8, dtype=torch.float64), torch.ones(8, dtype=torch.float64))
    ref["unpaired"] = _oracle_unpaired_grads(sy, rf, torch.ones(8, dtype=torch.float64),
                                             torch.ones(8, dtype=torch.float64))
    for k in ("R", "zeta", "jas", "r", "unpaired"):
        a, b = g[k].cpu(), ref[k]
        assert (a - b).abs().max().item() / max(1.0, b.abs().max().item()) <= 1e-8, k


def test_polarized_refusals(pw):
    P = need_gpu()
    sysh, wk, r, _ = _eval(P, pw.system, pw.r0, 4)
    swapped = dataclasses.replace(pw.system, n_up=9, n_dn=11, unpaired=np.zeros((44, 0)))
    with pytest.raises(P.QMCError) as ex:
        P.JAGPSystem(swapped)
    assert ex.value.code == -5
