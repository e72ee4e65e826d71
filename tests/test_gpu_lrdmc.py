"""Parity of the lattice-regularised DMC step (qmc_lrdmc_hops,
qmc_lrdmc_advance) with the CPU oracle (oracle/lrdmc.py), whose hop ratios
are Psi(x')/Psi(x) from two full evaluations.

Tolerances.  Hop ratios: relative 1e-10 in the metric |x-y|/max(|y|,1), the
bar of the move ratios.  Per-walker terms are sums of ratios divided by
2 a_i^2 (or a_i^2), so their bound is derived from the ratio bar:
  |d term| <= 1e-10 * sum_k max(|ratio_k|, 1) / a_k^2  +  1e-10 max(|E_kin|, |E_loc|, 1).
The continuous-time step: the hop index must be equal, unless the oracle's
running sum at the chosen boundary lies within the same bound of the target;
r_next bitwise equal (one FP64 addition of +-a_i on both sides); weight and
tau_left relative 1e-9 (the exponent tau_xi e_L inherits the escape-rate
error).

At the 160-electron, 1024-walker size the oracle cannot re-evaluate all
6N x 1024 configurations; there the ratios of sampled walkers and electrons
are compared with the oracle, and the terms and the step of every walker with
the oracle's formulas applied to the GPU's own ratios.
"""
import numpy as np
import pytest
import torch

from gpu_util import need_gpu, rel_err
from oracle import jagp as O
from oracle import lrdmc as L
from workloads import configs as C

pytestmark = pytest.mark.gpu

TERMS = ("e_loc", "e_kin", "lap_a", "va_shift", "v_sf", "escape", "hfn_diag")
ORACLE_KEY = {"lap_a": "lap_a", "v_sf": "V_sf", "escape": "escape", "hfn_diag": "HFN_diag"}


def _eval(P, w, Wk, precision=None):
    sysh = P.JAGPSystem(w.system) if precision is None else P.JAGPSystem(w.system, precision=precision)
    wk = P.Walkers(sysh, Wk)
    r = torch.tensor(w.r0[:Wk], device="cuda")
    out = wk.eval_batch(r)
    return sysh, wk, r, out


def _term_tol(ratios, a_i, e_kin, e_loc, bar=1e-10):
    s = (ratios.abs().clamp(min=1.0) / (a_i * a_i).unsqueeze(-1)).sum(dim=(1, 2))
    return bar * s + bar * torch.stack([e_kin.abs(), e_loc.abs(), torch.ones_like(e_kin)]).max(0).values


def _check_terms(gpu, col, a_i, bar=1e-10):
    """bar: relative bar of the hop ratios and energies the terms are built from
    (1e-10 FP64; 1e-8 for the mixed evaluation's int8 digit products)."""
    tol = _term_tol(col["ratios"], a_i, col["e_kin"], col["e_loc"], bar)
    for k in ("lap_a", "v_sf", "escape", "hfn_diag"):
        d = (gpu[k].cpu() - col[ORACLE_KEY[k]]).abs()
        assert (d <= tol).all(), (k, d.max().item(), tol.min().item())
    d = (gpu["va_shift"].cpu() - (col["V_a"] - col["V"])).abs()
    assert (d <= tol).all(), ("va_shift", d.max().item())
    for k in ("e_loc", "e_kin"):
        assert rel_err(gpu[k].cpu(), col[k]).max().item() <= bar


def _check_step(r, a_i, col, xi, w0, t0, rn, wt, tl, hop, tol):
    ro, wo, to, ho = L.advance(r, a_i, col, xi, w0, t0)
    hop = hop.cpu().long()
    same = hop == ho
    for w in torch.nonzero(~same).flatten().tolist():
        # a different hop is only allowed where the target sits on a boundary
        cum = torch.cumsum(col["G_off"][w].reshape(-1), 0)
        target = float(xi[w, 1]) * float(col["escape"][w])
        k = int(ho[w])
        edge = min(abs(float(cum[k]) - target), abs(float(cum[k - 1]) - target) if k > 0 else 1e300)
        assert edge <= float(tol[w]), (w, int(hop[w]), k, edge)
    assert int(same.sum()) >= len(same) - 1
    idx = torch.nonzero(same).flatten()
    assert torch.equal(rn.cpu()[idx], ro[idx])
    assert rel_err(wt.cpu()[idx], wo[idx]).max().item() <= 1e-9
    assert rel_err(tl.cpu()[idx], to[idx]).max().item() <= 1e-9
    return ho


@pytest.mark.parametrize("grid,precision", [("single", "fp64"), ("double", "fp64"), ("double", "mixed")])
def test_lrdmc_tiny_all_walkers(grid, precision):
    P = need_gpu()
    w = C.tiny_3nuc_10e()
    prm = C.LRDMC_SINGLE if grid == "single" else C.LRDMC_DOUBLE
    prec = {"fp64": P.QMC_FP64, "mixed": P.QMC_MIXED}[precision]
    Wk = 64
    sysh, wk, r, out = _eval(P, w, Wk, prec)
    g = wk.lrdmc_hops(**prm)
    xi = torch.tensor(C.lrdmc_draws(5, 1, Wk)[0], device="cuda")
    weight = torch.ones(Wk, dtype=torch.float64, device="cuda")
    tau = torch.full((Wk,), C.LRDMC_TAU, dtype=torch.float64, device="cuda")
    tau[:4] = 0.0                                         # no time left: untouched
    w0, t0 = weight.cpu().clone(), tau.cpu().clone()
    rn, hop = wk.lrdmc_advance(xi, weight, tau)
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    rc = r.cpu()
    a_i = L.mesh(sy, rc, prm["a"], prm["a_valence"], prm["tf_scale"])
    col = L.green_column(sy, rc, a_i, prm["gamma"])
    e = rel_err(g["ratios"].cpu(), col["ratios"]).max().item()
    print(f"[lrdmc tiny {grid} {precision}] ratio rel err {e:.3e}; negative hops "
          f"{int((col['ratios'] < 0).sum())}; hops made {int((hop >= 0).sum())}")
    # mixed: the cofactor rows come from the int8 digit products (about 1e-13 of
    # max|Phi| max|Lambda| L before the cond(W) amplification): bar 1e-8
    bar = 1e-10 if precision == "fp64" else 1e-8
    assert e <= bar
    _check_terms(g, col, a_i, bar)
    # the fixed-node lattice local energy is e_L for every gamma (oracle identity)
    assert torch.equal(g["e_loc"].cpu(), out["e_loc"].cpu())
    tol = _term_tol(col["ratios"], a_i, col["e_kin"], col["e_loc"], bar)
    _check_step(rc, a_i, col, xi.cpu(), w0, t0, rn, weight, tau, hop, tol)
    assert (hop.cpu()[:4] == -1).all() and torch.equal(rn.cpu()[:4], rc[:4])
    assert torch.equal(weight.cpu()[:4], w0[:4]) and (tau.cpu()[:4] == 0).all()


def test_lrdmc_80e_pade_series():
    P = need_gpu()
    w = C.forces_20nuc_80e(n_walkers=4)
    prm = dict(C.LRDMC_DOUBLE)
    sysh, wk, r, out = _eval(P, w, 4)
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    rc = r.cpu()
    a_i = L.mesh(sy, rc, prm["a"], prm["a_valence"], prm["tf_scale"])
    col = L.green_column(sy, rc, a_i, prm["gamma"])
    e = rel_err(g["ratios"].cpu(), col["ratios"]).max().item()
    print(f"[lrdmc 80e] ratio rel err {e:.3e}")
    assert e <= 1e-10
    _check_terms(g, col, a_i)


def test_lrdmc_chain_of_steps_tiny():
    # eval -> hops -> advance, five times; the oracle runs the same chain
    P = need_gpu()
    w = C.tiny_3nuc_10e()
    prm = C.LRDMC_SINGLE
    Wk = 32
    sysh, wk, r, _ = _eval(P, w, Wk)
    sy = O.from_workload_system(w.system)
    xi = C.lrdmc_draws(9, 5, Wk)
    weight = torch.ones(Wk, dtype=torch.float64, device="cuda")
    tau = torch.full((Wk,), 4 * C.LRDMC_TAU, dtype=torch.float64, device="cuda")
    ro, wo, to = r.cpu().clone(), weight.cpu().clone(), tau.cpu().clone()
    for t in range(5):
        g = wk.lrdmc_hops(**prm, ratios=False)
        rn, hop = wk.lrdmc_advance(torch.tensor(xi[t], device="cuda"), weight, tau)
        wk.eval_batch(rn)
        a_i = L.mesh(sy, ro, prm["a"])
        col = L.green_column(sy, ro, a_i, prm["gamma"])
        ro, wo, to, ho = L.advance(ro, a_i, col, torch.tensor(xi[t]), wo, to)
        assert torch.equal(hop.cpu().long(), ho), t
    torch.cuda.synchronize()
    assert torch.equal(wk.read(P.STATE_R).cpu(), ro)
    assert rel_err(weight.cpu(), wo).max().item() <= 1e-9
    assert rel_err(tau.cpu(), to).max().item() <= 1e-9


def test_lrdmc_full_size_160e():
    P = need_gpu()
    w = C.mol_40nuc_160e()
    Wk = w.r0.shape[0]
    prm = C.LRDMC_DOUBLE
    sysh, wk, r, out = _eval(P, w, Wk)
    g = wk.lrdmc_hops(**prm)
    xi = torch.tensor(C.lrdmc_draws(13, 1, Wk)[0], device="cuda")
    weight = torch.ones(Wk, dtype=torch.float64, device="cuda")
    tau = torch.full((Wk,), C.LRDMC_TAU, dtype=torch.float64, device="cuda")
    rn, hop = wk.lrdmc_advance(xi, weight, tau)
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    rc = r.cpu()
    a_i = L.mesh(sy, rc, prm["a"], prm["a_valence"], prm["tf_scale"])
    ah = g["ratios"].cpu()
    # sampled walkers and electrons (both spins) against full re-evaluation
    for wi in (0, Wk - 1):
        for e in (0, 79, 80, 159):
            for k, (sg, ax) in enumerate(L.DIRS):
                rnew = rc[wi:wi + 1, e].clone()
                rnew[0, ax] += sg * a_i[wi, e]
                ref = O.move_ratio(sy, rc[wi:wi + 1], e, rnew)
                assert rel_err(ah[wi, e, k], ref[0]).item() <= 1e-10, (wi, e, k)
    # every walker: the terms and the step from the oracle's formulas on the GPU's ratios
    ev = dict(e_kin=out["e_kin"].cpu(), e_loc=out["e_loc"].cpu(), V=(out["e_loc"] - out["e_kin"]).cpu())
    col = L.green_column(sy, rc, a_i, prm["gamma"], ratios=ah, ev=ev)
    _check_terms(g, col, a_i)
    tol = _term_tol(col["ratios"], a_i, col["e_kin"], col["e_loc"])
    w0 = torch.ones(Wk, dtype=torch.float64)
    t0 = torch.full((Wk,), C.LRDMC_TAU, dtype=torch.float64)
    ho = _check_step(rc, a_i, col, xi.cpu(), w0, t0, rn, weight, tau, hop, tol)
    print(f"[lrdmc 160e x {Wk}] hops made {int((ho >= 0).sum())}, double-grid fraction with a "
          f"{float((a_i == prm['a']).double().mean()):.3f}")


def test_lrdmc_blocked_inverse_sizes():
    # n = 112 per spin: the cofactor rows come from the blocked elimination
    P = need_gpu()
    w = C.multi_system(224, n_walkers=2)
    prm = C.LRDMC_SINGLE
    sysh, wk, r, _ = _eval(P, w, 2)
    g = wk.lrdmc_hops(**prm)
    torch.cuda.synchronize()
    sy = O.from_workload_system(w.system)
    rc = r.cpu()
    for e in (0, 111, 112, 223):
        for k, (sg, ax) in enumerate(L.DIRS):
            rnew = rc[:, e].clone()
            rnew[:, ax] += sg * prm["a"]
            ref = O.move_ratio(sy, rc, e, rnew)
            assert rel_err(g["ratios"].cpu()[:, e, k], ref).max().item() <= 1e-10, (e, k)


def test_lrdmc_state_and_argument_errors():
    P = need_gpu()
    w = C.tiny_3nuc_10e(n_walkers=8, n_steps=4)
    sysh, wk, r, _ = _eval(P, w, 8)
    xi = torch.zeros(8, 2, dtype=torch.float64, device="cuda")
    one = torch.ones(8, dtype=torch.float64, device="cuda")
    with pytest.raises(P.QMCError) as ex:
        wk.lrdmc_advance(xi, one.clone(), one.clone())          # no hops yet
    assert ex.value.code == -6
    for bad in (dict(a=0.0), dict(a=0.1, gamma=-1.0), dict(a=0.1, a_valence=0.4, tf_scale=0.0)):
        with pytest.raises(P.QMCError) as ex:
            wk.lrdmc_hops(**bad)
        assert ex.value.code == -1
    wk.lrdmc_hops(a=0.2)
    d = torch.tensor(w.disp[:1], device="cuda")
    u = torch.tensor(w.unif[:1], device="cuda")
    wk.vmc_steps(0, d, u)                                       # a move makes the cofactor rows stale
    with pytest.raises(P.QMCError) as ex:
        wk.lrdmc_hops(a=0.2)
    assert ex.value.code == -6
    with pytest.raises(P.QMCError) as ex:
        wk.lrdmc_advance(xi, one.clone(), one.clone())
    assert ex.value.code == -6
    wk.eval_batch(wk.read(P.STATE_R))
    wk.lrdmc_hops(a=0.2)
    wk.lrdmc_advance(xi, one.clone(), one.clone())
    torch.cuda.synchronize()
