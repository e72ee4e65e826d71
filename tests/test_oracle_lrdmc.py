"""Pins of the LRDMC oracle (Lattice regularized Monte Carlo section) against
closed forms, limits and identities that the paper's definitions fix.

* Hydrogen-like ion with its exact ground state e^{-Z r}: the six hop ratios,
  the lattice Laplacian and V^a in closed form; the fixed-node local energy is
  the eigenvalue -Z^2/2 for every gamma (zero variance).
* The lattice Laplacian tends to the continuous one at O(a^2) (second-order
  finite differences): error ratio ~4 when a halves, Richardson limit equals
  -2 E_kin of the continuous evaluation.
* Fixed-node identity: sum_{x'} H^{FN,gamma}_{x',x} Psi(x')/Psi(x) equals the
  continuous local energy for every gamma, with hops that cross the node.
* Fixed-node Green's function off-diagonal elements are never negative.
* Continuous time against the discrete-time chain: for large lambda the
  probability of staying M = lambda tau steps, (G~_xx / b~_x)^M, tends to the
  oracle's exp(-escape tau), and the weight prod b~_x / lambda tends to
  exp(-tau e_L).
* Hop selection: over a fine grid of the uniform, each hop is chosen with
  frequency G~_{x',x} / escape; the chosen configuration's Psi ratio is the
  hop ratio.
* Double grid: the mesh follows the Thomas-Fermi length 0.8853 Z^{-1/3}.
"""
import math

import numpy as np
import pytest
import torch

from oracle import jagp as O
from oracle import lrdmc as L
from test_oracle_pins import make_system
from workloads import configs as C

DT = torch.float64


def hydrogenic(Z):
    # Slater 1s with zeta = Z, no Jastrow: exact eigenfunction, eigenvalue -Z^2/2
    return make_system([[0.0, 0.0, 0.0]], [Z], [(0, 0)], 1, 0, lam=np.zeros((1, 1)),
                       unpaired=np.ones((1, 1)), zetas=[Z], radial=1)[1]


@pytest.mark.parametrize("Z,a", [(1.0, 0.2), (2.0, 0.1), (3.0, 0.05)])
def test_hydrogenic_closed_forms(Z, a):
    sy = hydrogenic(Z)
    rng = np.random.default_rng(11)
    r = torch.tensor(rng.normal(size=(12, 1, 3)) * 1.2, dtype=DT)
    a_i = torch.full((12, 1), a, dtype=DT)
    col = L.green_column(sy, r, a_i, gamma=0.0)
    x = r[:, 0].numpy()
    rn = np.linalg.norm(x, axis=1)
    ratios = np.zeros((12, 6))
    for k, (sg, ax) in enumerate(L.DIRS):
        y = x.copy()
        y[:, ax] += sg * a
        ratios[:, k] = np.exp(-Z * (np.linalg.norm(y, axis=1) - rn))
    assert np.allclose(col["ratios"][:, 0].numpy(), ratios, rtol=1e-13, atol=0)
    lap_a = (ratios - 1.0).sum(1) / a ** 2
    assert np.allclose(col["lap_a"].numpy(), lap_a, rtol=1e-11, atol=1e-11)
    # lap psi / psi = Z^2 - 2Z/r ; V = -Z/r ; V^a = V + (lap_a - lap)/2
    V_a = -Z / rn + 0.5 * (lap_a - (Z * Z - 2.0 * Z / rn))
    assert np.allclose(col["V_a"].numpy(), V_a, rtol=1e-11, atol=1e-11)
    # a nodeless state: nothing flips sign
    assert (col["V_sf"] == 0).all()
    for gamma in (0.0, 0.5, 2.0):
        c = L.green_column(sy, r, a_i, gamma=gamma, ratios=col["ratios"])
        assert np.allclose(c["e_L_fn"].numpy(), -0.5 * Z * Z, rtol=0, atol=1e-11)


def test_lattice_laplacian_second_order_limit():
    w = C.tiny_3nuc_10e(n_walkers=4, n_steps=1)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)
    ev = O.evaluate(sy, r)
    target = -2.0 * ev["e_kin"]
    f = {}
    for a in (0.04, 0.02, 0.01):
        a_i = torch.full(r.shape[:2], a, dtype=DT)
        f[a] = L.green_column(sy, r, a_i, 0.0, ev=ev)["lap_a"]
    e1, e2, e3 = f[0.04] - target, f[0.02] - target, f[0.01] - target
    # O(a^2): halving a divides the error by ~4
    q1, q2 = e1 / e2, e2 / e3
    assert ((q1 > 3.6) & (q1 < 4.4)).all() and ((q2 > 3.8) & (q2 < 4.2)).all(), (q1, q2)
    rich = (4.0 * f[0.01] - f[0.02]) / 3.0
    assert ((rich - target).abs() <= 1e-5 * target.abs().clamp(min=1.0)).all()


@pytest.mark.parametrize("gamma", [0.0, 0.5, 1.0])
def test_fixed_node_local_energy_identity(gamma):
    w = C.tiny_3nuc_10e(n_walkers=16, n_steps=1)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)
    # long hops so that some of them cross the nodal surface
    a_i = L.mesh(sy, r, 0.3, a_valence=0.9, tf_scale=1.0)
    col = L.green_column(sy, r, a_i, gamma)
    assert int((col["ratios"] < 0).sum()) > 0
    assert (col["V_sf"] > 0).any()
    tol = 1e-10 * col["e_loc"].abs().clamp(min=1.0) + 1e-12 * (col["ratios"].abs() / a_i.unsqueeze(-1) ** 2).sum(dim=(1, 2))
    assert ((col["e_L_fn"] - col["e_loc"]).abs() <= tol).all()
    # no sign problem: every off-diagonal element of G~^FN is >= 0
    assert (col["G_off"] >= 0).all()
    # gamma = 0 drops the node-crossing hops altogether
    if gamma == 0.0:
        assert (col["G_off"][col["ratios"] < 0] == 0).all()


def test_continuous_time_limit_of_discrete_chain():
    w = C.tiny_3nuc_10e(n_walkers=6, n_steps=1)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)
    a_i = L.mesh(sy, r, 0.2)
    col = L.green_column(sy, r, a_i, 0.5)
    tau = 2e-3                      # escape * tau = 1.5 - 3: staying and hopping both likely
    lam = 1e10
    diag, b = L.discrete_column(col, lam)
    M = int(lam * tau)
    p_stay = torch.exp(M * torch.log(diag / b))            # probability of M diagonal steps
    w_stay = torch.exp(M * torch.log(b / lam))             # weight of those steps, / lambda^M
    # the oracle's continuous-time step: the uniform that makes tau_xi = tau exactly
    # separates staying from hopping
    xi_edge = -torch.expm1(-col["escape"] * tau)
    assert torch.allclose(p_stay, torch.exp(-col["escape"] * tau), rtol=1e-6, atol=0)
    assert ((p_stay > 0.01) & (p_stay < 0.99)).all()
    xi = torch.stack([xi_edge * 0.999999, torch.full_like(xi_edge, 0.5)], dim=1)
    ones = torch.ones(r.shape[0], dtype=DT)
    _, wt, tl, hop = L.advance(r, a_i, col, xi, ones, torch.full_like(ones, tau))
    assert (hop >= 0).all()
    xi[:, 0] = xi_edge * 1.000001
    _, wt, tl, hop = L.advance(r, a_i, col, xi, ones, torch.full_like(ones, tau))
    assert (hop == -1).all() and (tl == 0).all()
    assert torch.allclose(wt, w_stay, rtol=1e-6, atol=0)
    assert torch.allclose(wt, torch.exp(-tau * col["e_loc"]), rtol=1e-13, atol=0)


def test_hop_selection_frequencies_and_geometry():
    w = C.tiny_3nuc_10e(n_walkers=3, n_steps=1)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)
    a_i = L.mesh(sy, r, 0.3, a_valence=0.9)
    col = L.green_column(sy, r, a_i, 0.5)
    Wk, N = r.shape[:2]
    M = 20000
    for wk in range(Wk):
        counts = np.zeros(6 * N)
        sel = {wk}
        rr = r[wk:wk + 1].expand(M, N, 3)
        c1 = {k: v[wk:wk + 1].expand(M, *v.shape[1:]) for k, v in col.items()}
        xi = torch.stack([torch.zeros(M, dtype=DT), (torch.arange(M, dtype=DT) + 0.5) / M], 1)
        rn, _, _, hop = L.advance(rr, a_i[wk:wk + 1].expand(M, N), c1, xi,
                                  torch.ones(M, dtype=DT), torch.full((M,), 1e9, dtype=DT))
        np.add.at(counts, hop.numpy(), 1)
        p = (col["G_off"][wk].reshape(-1) / col["escape"][wk]).numpy()
        assert np.abs(counts / M - p).max() <= 1.0 / M + 1e-12, sel
        # geometry of three chosen hops and their ratios from scratch
        for j in (0, M // 2, M - 1):
            k = int(hop[j])
            i, d = divmod(k, 6)
            sg, ax = L.DIRS[d]
            delta = rn[j] - r[wk]
            expect = torch.zeros(N, 3, dtype=DT)
            expect[i, ax] = sg * a_i[wk, i]
            assert torch.allclose(delta, expect, atol=1e-15, rtol=0)
            ratio = O.move_ratio(sy, r[wk:wk + 1], i, rn[j:j + 1, i])
            assert torch.allclose(ratio, col["ratios"][wk, i, d].view(1), rtol=1e-12, atol=0)


def test_double_grid_mesh_thomas_fermi():
    R = [[0.0, 0.0, 0.0], [10.0, 0.0, 0.0]]
    s, sy = make_system(R, [8.0, 1.0], [(0, 0), (1, 0)], 1, 1)
    tf8 = 0.8853 / 2.0              # 8^{-1/3} = 1/2
    tf1 = 0.8853
    r = torch.tensor([[[tf8 * 0.99, 0.0, 0.0], [0.0, tf8 * 1.01, 0.0]],
                      [[10.0 + tf1 * 0.99, 0.0, 0.0], [10.0, 0.0, tf1 * 1.01]]], dtype=DT)
    m = L.mesh(sy, r, 0.1, a_valence=0.4, tf_scale=1.0)
    assert m.tolist() == [[0.1, 0.4], [0.1, 0.4]]
    m2 = L.mesh(sy, r, 0.1, a_valence=0.4, tf_scale=2.0)
    assert m2.tolist() == [[0.1, 0.1], [0.1, 0.1]]
    assert (L.mesh(sy, r, 0.2) == 0.2).all()
