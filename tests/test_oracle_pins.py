"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, brute force on tiny inputs, identities of determinants, symmetries of
the wave function, the exact hydrogenic energy and finite differences.
"""
import itertools
import math
import os

import numpy as np
import pytest
import torch

from oracle import jagp as O
from workloads import configs as C

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
DT = torch.float64


def golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split("=")
                vals[k.strip()] = float(v)
    return vals


def tiny():
    w = C.tiny_3nuc_10e(n_walkers=8, n_steps=4)
    return w, O.from_workload_system(w.system), torch.tensor(w.r0)


def make_system(R, Z, shells, n_up, n_dn, lam=None, unpaired=None, j1_form=0,
                j1_b=None, j2_form=0, j2=None, zetas=None, radial=0, seed=0):
    """A hand-built system: shells = list of (center, l); one zeta per shell."""
    rng = np.random.default_rng(seed)
    center, l, m, zeta = [], [], [], []
    for si, (a, ll) in enumerate(shells):
        z = zetas[si] if zetas is not None else float(np.exp(rng.uniform(np.log(0.3), np.log(3.0))))
        for mm in range(C.N_COMP[ll]):
            center.append(a); l.append(ll); m.append(mm); zeta.append(z)
    L = len(zeta)
    if lam is None:
        lam = rng.standard_normal((L, L)) / L
    if unpaired is None:
        unpaired = np.zeros((L, n_up - n_dn))
    R = np.asarray(R, float)
    s = C.System(name="hand", R=R, Z=np.asarray(Z, float), center=np.array(center, np.int32),
                 l=np.array(l, np.int32), m=np.array(m, np.int32), zeta=np.array(zeta),
                 radial=np.full(L, radial, np.int32), lam=np.asarray(lam, float),
                 n_up=n_up, n_dn=n_dn, unpaired=np.asarray(unpaired, float),
                 j1_form=j1_form, j1_b=np.ones(len(Z)) if j1_b is None else np.asarray(j1_b, float),
                 j2_form=j2_form, j2=np.array([1.0, 1.0]) if j2 is None else np.asarray(j2, float))
    return s, O.from_workload_system(s)


# ---------------------------------------------------------------------------
# basis (eq. gaussian / eq. slater)
# ---------------------------------------------------------------------------

def test_basis_at_center():
    _, sy, _ = tiny()
    for a in range(3):
        psi, _, _ = O.basis(sy, sy.R[a].view(1, 3))
        own = (sy.center == a)
        s_own = own & (sy.l == 0)
        p_own = own & (sy.l == 1)
        assert torch.allclose(psi[0, s_own], torch.ones(int(s_own.sum()), dtype=DT), atol=0, rtol=1e-15)
        assert torch.all(psi[0, p_own] == 0)


def test_basis_gaussian_laplacian_closed_form():
    # real solid harmonics are harmonic and homogeneous of degree l, so
    # lap(P e^{-z r^2}) = (4 z^2 r^2 - (4 l + 6) z) P e^{-z r^2}
    s, sy = make_system([[0.1, -0.2, 0.3]], [1.0], [(0, 0), (0, 1), (0, 2)], 1, 1)
    r = torch.tensor(np.random.default_rng(1).normal(size=(50, 3)), dtype=DT)
    psi, _, lap = O.basis(sy, r)
    d2 = ((r.unsqueeze(1) - sy.R[sy.center]) ** 2).sum(-1)
    ref = (4 * sy.zeta ** 2 * d2 - (4 * sy.l.to(DT) + 6) * sy.zeta) * psi
    assert torch.allclose(lap, ref, rtol=1e-12, atol=1e-13)


def test_basis_slater_laplacian_closed_form():
    s, sy = make_system([[0.0, 0.0, 0.0]], [1.0], [(0, 0), (0, 1), (0, 2)], 1, 1, radial=1)
    r = torch.tensor(np.random.default_rng(2).normal(size=(50, 3)), dtype=DT)
    psi, _, lap = O.basis(sy, r)
    rr = torch.sqrt(((r.unsqueeze(1) - sy.R[sy.center]) ** 2).sum(-1))
    ref = (sy.zeta ** 2 - 2 * sy.zeta * (sy.l.to(DT) + 1) / rr) * psi
    assert torch.allclose(lap, ref, rtol=1e-12, atol=1e-13)


def test_basis_angular_factors_are_solid_harmonics():
    # unnormalised r^l Re[Y_lm] in Cartesian form: check homogeneity of degree l
    # and the explicit l = 2 combinations at a point
    s, sy = make_system([[0.0, 0.0, 0.0]], [1.0], [(0, 1), (0, 2)], 1, 1, zetas=[0.0, 0.0])
    x, y, z = 0.3, -0.7, 1.1
    psi, _, _ = O.basis(sy, torch.tensor([[x, y, z]], dtype=DT))
    ref = [x, y, z, x * y, y * z, z * x, x * x - y * y, 2 * z * z - x * x - y * y]
    assert np.allclose(psi[0].numpy(), ref, rtol=0, atol=1e-15)
    psi2, _, _ = O.basis(sy, torch.tensor([[2 * x, 2 * y, 2 * z]], dtype=DT))
    deg = sy.l.to(DT)
    assert torch.allclose(psi2[0], psi[0] * 2 ** deg, rtol=1e-14)


def test_basis_finite_differences():
    w, sy, r = tiny()
    pts = r[:2].reshape(-1, 3)
    psi, grad, lap = O.basis(sy, pts)
    h = 1e-5
    for ax in range(3):
        e = torch.zeros(3, dtype=DT); e[ax] = h
        fd = (O.basis(sy, pts + e)[0] - O.basis(sy, pts - e)[0]) / (2 * h)
        assert torch.allclose(grad[..., ax], fd, rtol=1e-6, atol=1e-8)
    # Richardson-extrapolated second differences
    def lap_fd(hh):
        tot = 0
        for ax in range(3):
            e = torch.zeros(3, dtype=DT); e[ax] = hh
            tot = tot + (O.basis(sy, pts + e)[0] - 2 * psi + O.basis(sy, pts - e)[0]) / hh ** 2
        return tot
    fd2 = (4 * lap_fd(5e-4) - lap_fd(1e-3)) / 3
    assert torch.allclose(lap, fd2, rtol=1e-5, atol=1e-6)


# ---------------------------------------------------------------------------
# Jastrow (onebody_J_hom, onebody_u, twobody_v)
# ---------------------------------------------------------------------------

def test_jastrow_cusps():
    g = golden("jastrow_cusps.txt")
    for Z in (1.0, 3.0, 8.0):
        for form in (1, 2):
            s, sy = make_system([[0.0, 0.0, 0.0]], [Z], [(0, 0)], 1, 0, j1_form=form, j1_b=[1.3])
            h = 1e-7
            r = torch.tensor([[[0.0, 0.0, h]], [[0.0, 0.0, 2 * h]]], dtype=DT)
            J, _, _ = O.jastrow(sy, r)
            slope = float((J[1] - J[0]) / h)
            assert abs(slope / (-Z) - g["j1_slope_over_minus_Z"]) < 1e-5
    for same, key in ((True, "v_slope_parallel"), (False, "v_slope_antiparallel")):
        n_up, n_dn = (2, 0) if same else (1, 1)
        s, sy = make_system([[50.0, 50.0, 50.0]], [1.0], [(0, 0)], n_up, n_dn,
                            j2_form=1, j2=[1.7, 0.9],
                            unpaired=np.zeros((1, n_up - n_dn)) if n_up > n_dn else None)
        h = 1e-7
        r = torch.tensor([[[0, 0, 0], [0, 0, h]], [[0, 0, 0], [0, 0, 2 * h]]], dtype=DT)
        J, _, _ = O.jastrow(sy, r)
        assert abs(float((J[1] - J[0]) / h) - g[key]) < 1e-6


def test_jastrow_large_distance_limits():
    g = golden("jastrow_limits.txt")
    big = 1e9
    s, sy = make_system([[0.0, 0.0, 0.0]], [2.0], [(0, 0)], 1, 0, j1_form=1, j1_b=[1.0])
    J, _, _ = O.jastrow(sy, torch.tensor([[[0.0, 0.0, big]]], dtype=DT))
    assert abs(float(J[0]) / (-(4.0 ** 0.75)) - g["u_inf_b1"]) < 1e-8
    for b, sfx in ((1.0, "b1"), (2.0, "b2")):
        for same, key in ((True, "v_inf_parallel_"), (False, "v_inf_antiparallel_")):
            n_up, n_dn = (2, 0) if same else (1, 1)
            s, sy = make_system([[0.0, 0.0, 0.0]], [1.0], [(0, 0)], n_up, n_dn, j2_form=1, j2=[b, b],
                                unpaired=np.zeros((1, n_up - n_dn)) if n_up > n_dn else None)
            J, _, _ = O.jastrow(sy, torch.tensor([[[0, 0, 0], [0, 0, big]]], dtype=DT))
            assert abs(float(J[0]) - g[key + sfx]) < 1e-7


def test_jastrow_pade_series_reduces_to_pade():
    s, sy1 = make_system([[0.0, 0.0, 0.0]], [1.0], [(0, 0)], 2, 2, j2_form=1, j2=[1.3, 0.7])
    s, sy2 = make_system([[0.0, 0.0, 0.0]], [1.0], [(0, 0)], 2, 2, j2_form=2,
                         j2=[1.3, 0, 0, 0, 0.7, 0, 0, 0])
    r = torch.tensor(np.random.default_rng(3).normal(size=(5, 4, 3)), dtype=DT)
    for a, b in zip(O.jastrow(sy1, r), O.jastrow(sy2, r)):
        assert torch.allclose(a, b, rtol=1e-14, atol=1e-15)


def _fd_grad_lap(f, r, h=2e-4, h2=2e-4):
    """Richardson-extrapolated central differences: gradient and Laplacian."""
    Wk, N, _ = r.shape
    g = torch.zeros(Wk, N, 3, dtype=DT)
    lap = torch.zeros(Wk, N, dtype=DT)
    f0 = f(r)
    for i in range(N):
        for ax in range(3):
            e = torch.zeros_like(r); e[:, i, ax] = 1.0
            g1 = (f(r + h * e) - f(r - h * e)) / (2 * h)
            g2 = (f(r + 0.5 * h * e) - f(r - 0.5 * h * e)) / h
            g[:, i, ax] = (4 * g2 - g1) / 3
            d1 = (f(r + h2 * e) - 2 * f0 + f(r - h2 * e)) / h2 ** 2
            hh = h2 / 2
            d2 = (f(r + hh * e) - 2 * f0 + f(r - hh * e)) / hh ** 2
            lap[:, i] += (4 * d2 - d1) / 3
    return g, lap


def test_jastrow_finite_differences():
    w, sy, r = tiny()
    J, gJ, hJ = O.jastrow(sy, r)
    g, lap = _fd_grad_lap(lambda x: O.jastrow(sy, x)[0], r, h2=1e-3)
    assert torch.allclose(gJ, g, rtol=1e-7, atol=1e-7)
    assert torch.allclose(hJ, lap, rtol=1e-5, atol=1e-5)
    # the eight-parameter two-body form
    wf = C.forces_20nuc_80e(n_walkers=2)
    syf = O.from_workload_system(wf.system)
    rf = torch.tensor(wf.r0)[:, :6]
    syf.n_up, syf.n_dn = 3, 3
    J, gJ, hJ = O.jastrow(syf, rf)
    g, lap = _fd_grad_lap(lambda x: O.jastrow(syf, x)[0], rf, h2=1e-3)
    assert torch.allclose(gJ, g, rtol=1e-7, atol=1e-7)
    assert torch.allclose(hJ, lap, rtol=1e-5, atol=1e-5)


def test_coulomb_hand_value():
    g = golden("h2_coulomb.txt")
    s, sy = make_system([[0, 0, 0], [0, 0, 2]], [1.0, 1.0], [(0, 0)], 1, 1)
    V = O.potential(sy, torch.tensor([[[0, 0, 1.0], [1.0, 0, 0]]], dtype=DT))
    assert abs(float(V[0]) - g["v_total"]) < 1e-14


# ---------------------------------------------------------------------------
# geminal and determinant (agp_expansion, eq:wfAGPs, eq:wfAGPunpaired)
# ---------------------------------------------------------------------------

def test_geminal_entries_by_definition_nonsymmetric_lambda():
    rng = np.random.default_rng(4)
    s, sy = make_system([[0, 0, 0], [1.5, 0, 0]], [1.0, 2.0], [(0, 0), (0, 1), (1, 0), (1, 2)], 3, 3,
                        lam=rng.standard_normal((10, 10)))
    r = torch.tensor(rng.normal(size=(2, 6, 3)), dtype=DT)
    Phi, _, _ = O.basis(sy, r)
    W = O.geminal(sy, Phi)
    lam = s.lam
    for w in range(2):
        for i in range(3):
            for j in range(3):
                f = sum(lam[mu, nu] * Phi[w, i, mu].item() * Phi[w, 3 + j, nu].item()
                        for mu in range(10) for nu in range(10))
                assert abs(W[w, i, j].item() - f) < 1e-13 * max(1.0, abs(f))


def _leibniz_det(M):
    n = M.shape[0]
    tot = 0.0
    for p in itertools.permutations(range(n)):
        inv = sum(1 for a in range(n) for b in range(a + 1, n) if p[a] > p[b])
        prod = 1.0
        for i in range(n):
            prod *= M[i, p[i]]
        tot += (-1) ** inv * prod
    return tot


def test_determinant_brute_force_leibniz():
    w, sy, r = tiny()
    out = O.evaluate(sy, r, with_intermediates=True)
    J = out["J"]
    for k in range(r.shape[0]):
        d = _leibniz_det(out["W"][k].numpy())
        assert np.sign(d) == out["sign"][k].item()
        assert abs(math.log(abs(d)) + J[k].item() - out["logabs"][k].item()) < 1e-10


def test_antisymmetry_same_spin_swap():
    w, sy, r = tiny()
    a = O.evaluate(sy, r)
    for (i, j) in ((0, 3), (5, 9)):
        r2 = r.clone(); r2[:, [i, j]] = r[:, [j, i]]
        b = O.evaluate(sy, r2)
        assert torch.equal(b["sign"], -a["sign"])
        assert torch.allclose(b["logabs"], a["logabs"], rtol=1e-13)
        assert torch.allclose(b["e_loc"], a["e_loc"], rtol=1e-10)


def test_lambda_scaling():
    w, sy, r = tiny()
    a = O.evaluate(sy, r)
    c = -2.5
    b = O.evaluate(sy, r, lam=c * sy.lam)
    assert torch.allclose(b["logabs"], a["logabs"] + sy.n_up * math.log(abs(c)), rtol=1e-13)
    assert torch.equal(b["sign"], a["sign"] * (-1) ** sy.n_up)
    assert torch.allclose(b["e_loc"], a["e_loc"], rtol=1e-10)
    assert torch.allclose(b["drift"], a["drift"], rtol=1e-9, atol=1e-9)


def test_spin_exchange_symmetric_lambda():
    w, sy, r = tiny()
    a = O.evaluate(sy, r)
    r2 = torch.cat([r[:, sy.n_up:], r[:, :sy.n_up]], dim=1)
    b = O.evaluate(sy, r2)
    assert torch.allclose(b["logabs"], a["logabs"], rtol=1e-13)
    assert torch.equal(b["sign"], a["sign"])
    assert torch.allclose(b["e_loc"], a["e_loc"], rtol=1e-10)


def test_slater_reduction():
    # Lambda = sum_{k<=N/2} c_k c_k^T: det W = det(Phi_up C) det(Phi_dn C)  (SD section)
    w, sy, r = tiny()
    rng = np.random.default_rng(5)
    Cm = rng.standard_normal((24, sy.n_up))
    lam = torch.tensor(Cm @ Cm.T, dtype=DT)
    Phi, _, _ = O.basis(sy, r)
    sign, logdet = torch.linalg.slogdet(O.geminal(sy, Phi, lam))
    du = np.linalg.det(Phi[:, :sy.n_up].numpy() @ Cm)
    dd = np.linalg.det(Phi[:, sy.n_up:].numpy() @ Cm)
    prod = du * dd
    assert np.allclose(sign.numpy(), np.sign(prod))
    assert np.allclose(logdet.numpy(), np.log(np.abs(prod)), rtol=1e-12, atol=1e-12)


def test_multiconfiguration_cauchy_binet():
    # Lambda = C D C^T of rank r > N/2: det W = sum over N/2-subsets S of
    # prod_{k in S} d_k det(Phi_up C)[:, S] det(Phi_dn C)[:, S]  (eq:gtop_exp)
    rng = np.random.default_rng(6)
    s, sy = make_system([[0, 0, 0], [1.2, 0.3, 0], [0, 1.4, 0.5]], [1.0, 1.0, 1.0],
                        [(0, 0), (0, 1), (1, 0), (1, 1), (2, 0)], 3, 3)
    L = s.zeta.shape[0]
    rank = 7
    Cm = rng.standard_normal((L, rank))
    dvec = rng.standard_normal(rank)
    lam = torch.tensor(Cm @ np.diag(dvec) @ Cm.T, dtype=DT)
    r = torch.tensor(rng.normal(size=(3, 6, 3)), dtype=DT)
    Phi, _, _ = O.basis(sy, r)
    detW = torch.linalg.det(O.geminal(sy, Phi, lam)).numpy()
    Mu = Phi[:, :3].numpy() @ Cm
    Md = Phi[:, 3:].numpy() @ Cm
    tot = np.zeros(3)
    for S in itertools.combinations(range(rank), 3):
        S = list(S)
        tot += np.prod(dvec[S]) * np.linalg.det(Mu[:, :, S]) * np.linalg.det(Md[:, :, S])
    assert np.allclose(detW, tot, rtol=1e-11, atol=0)


# ---------------------------------------------------------------------------
# local energy and drift
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("Z", [1.0, 2.0, 3.0])
def test_hydrogenic_exact_energy(Z):
    g = golden("hydrogenic_exact.txt")
    key = {1.0: "e_loc_Z1", 2.0: "e_loc_Z2", 3.0: "e_loc_Z3"}[Z]
    rng = np.random.default_rng(7)
    r = torch.tensor(rng.normal(size=(20, 1, 3)) * 1.5, dtype=DT)
    # zeta = 0 Gaussian (constant orbital) x one-body Pade Jastrow with b = 0
    s, sy = make_system([[0.2, -0.1, 0.4]], [Z], [(0, 0)], 1, 0, lam=np.zeros((1, 1)),
                        unpaired=np.ones((1, 1)), zetas=[0.0], j1_form=2, j1_b=[0.0])
    out = O.evaluate(sy, r + sy.R[0])
    assert torch.allclose(out["e_loc"], torch.full((20,), g[key], dtype=DT), atol=1e-12, rtol=0)
    # Slater 1s with zeta = Z and no Jastrow
    s, sy = make_system([[0.0, 0.0, 0.0]], [Z], [(0, 0)], 1, 0, lam=np.zeros((1, 1)),
                        unpaired=np.ones((1, 1)), zetas=[Z], radial=1)
    out = O.evaluate(sy, r)
    assert torch.allclose(out["e_loc"], torch.full((20,), g[key], dtype=DT), atol=1e-12, rtol=0)


def test_drift_and_kinetic_match_finite_differences():
    w, sy, r = tiny()
    r = r[:4]
    out = O.evaluate(sy, r)
    f = lambda x: O.log_psi(sy, x)[0]
    g, lap = _fd_grad_lap(f, r)
    assert torch.allclose(out["drift"], g, rtol=1e-6, atol=1e-6)
    # -1/2 lap Psi / Psi = -1/2 (lap log|Psi| + |grad log|Psi||^2)
    ekin_fd = -0.5 * (lap.sum(-1) + (g * g).sum(dim=(1, 2)))
    assert torch.allclose(out["e_kin"], ekin_fd, rtol=1e-5, atol=1e-4)


def test_drift_and_kinetic_pade_series_and_d_shells():
    wf = C.forces_20nuc_80e(n_walkers=1)
    s = wf.system
    keep_nuc = 3
    keep = np.isin(s.center, np.arange(keep_nuc))
    idx = np.nonzero(keep)[0]
    s2 = C.System(name="cut", R=s.R[:keep_nuc], Z=s.Z[:keep_nuc], center=s.center[idx], l=s.l[idx],
                  m=s.m[idx], zeta=s.zeta[idx], radial=s.radial[idx],
                  lam=s.lam[np.ix_(idx, idx)], n_up=3, n_dn=3, unpaired=np.zeros((len(idx), 0)),
                  j1_form=2, j1_b=np.ones(keep_nuc), j2_form=2, j2=s.j2)
    sy = O.from_workload_system(s2)
    r = torch.tensor(C.random_positions(8, s2, 2))
    out = O.evaluate(sy, r)
    g, lap = _fd_grad_lap(lambda x: O.log_psi(sy, x)[0], r)
    assert torch.allclose(out["drift"], g, rtol=1e-6, atol=1e-6)
    ekin_fd = -0.5 * (lap.sum(-1) + (g * g).sum(dim=(1, 2)))
    assert torch.allclose(out["e_kin"], ekin_fd, rtol=1e-5, atol=1e-4)
    # d shells: one more system with l = 2
    s3, sy3 = make_system([[0, 0, 0], [1.1, 0.4, -0.3]], [2.0, 1.0], [(0, 0), (0, 2), (1, 1), (1, 2)],
                          2, 2, j1_form=1, j2_form=1, j2=[0.8, 1.2])
    r3 = torch.tensor(np.random.default_rng(9).normal(size=(3, 4, 3)), dtype=DT)
    out3 = O.evaluate(sy3, r3)
    g, lap = _fd_grad_lap(lambda x: O.log_psi(sy3, x)[0], r3)
    assert torch.allclose(out3["drift"], g, rtol=1e-6, atol=1e-6)
    assert torch.allclose(out3["e_kin"], -0.5 * (lap.sum(-1) + (g * g).sum(dim=(1, 2))), rtol=1e-5, atol=1e-4)


def test_coalescence_bounded():
    w, sy, r = tiny()
    r = r[:1].clone()
    # electron 0 onto nucleus 0; electrons 1 (up) and 5 (down) together
    vals = []
    for eps in (1e-3, 1e-5, 1e-7):
        x = r.clone()
        x[0, 0] = sy.R[0] + torch.tensor([eps, 0.0, 0.0], dtype=DT)
        x[0, 5] = x[0, 1] + torch.tensor([0.0, eps, 0.0], dtype=DT)
        vals.append(O.evaluate(sy, x)["e_loc"].item())
    assert abs(vals[2] - vals[1]) < 1e-2 and abs(vals[1] - vals[0]) < 0.5


def test_singular_and_nonfinite_status():
    w, sy, r = tiny()
    x = r[:2].clone()
    # Lambda = 0 makes every geminal entry zero: det = 0 exactly -> status 1
    out = O.evaluate(sy, x, lam=torch.zeros_like(sy.lam))
    assert out["status"].tolist() == [1, 1]
    assert out["sign"][0].item() == 0 and out["logabs"][0].item() == -math.inf
    # an electron on a nucleus makes the potential infinite -> status 2
    x[0, 2] = sy.R[1]
    out = O.evaluate(sy, x)
    assert out["status"].tolist() == [2, 0]


# ---------------------------------------------------------------------------
# moves: the definition ratio against the matrix-determinant lemma
# ---------------------------------------------------------------------------

def test_move_ratio_matches_determinant_lemma():
    w, sy, r = tiny()
    out = O.evaluate(sy, r, with_intermediates=True)
    A = out["A"]
    rng = np.random.default_rng(10)
    for e in (0, 4, 5, 9):
        rn = r[:, e] + torch.tensor(rng.normal(size=(r.shape[0], 3)) * 0.3, dtype=DT)
        ratio = O.move_ratio(sy, r, e, rn)
        psi_new, _, _ = O.basis(sy, rn)
        Phi = out["Phi"]
        if e < sy.n_up:
            wrow = torch.einsum('wm,mn,wjn->wj', psi_new, sy.lam, Phi[:, sy.n_up:])
            rdet = torch.einsum('wj,wj->w', wrow, A[:, :, e])
        else:
            jd = e - sy.n_up
            wcol = torch.einsum('wim,mn,wn->wi', Phi[:, :sy.n_up], sy.lam, psi_new)
            rdet = torch.einsum('wi,wi->w', A[:, jd, :], wcol)
        r2 = r.clone(); r2[:, e] = rn
        dJ = O.jastrow(sy, r2)[0] - out["J"]
        assert torch.allclose(ratio, rdet * torch.exp(dJ), rtol=1e-10, atol=1e-14)


# ---------------------------------------------------------------------------
# derivatives: finite differences, Jacobi's formula, translation invariance
# ---------------------------------------------------------------------------

def test_forces_match_central_differences():
    w, sy, r = tiny()
    r = r[:3]
    gl = torch.tensor([0.7, -0.2, 1.1], dtype=DT)
    ge = torch.tensor([0.3, 0.5, -0.4], dtype=DT)
    g = O.forces_vjp(sy, r, gl, ge)
    A = sy.R.shape[0]

    def F(**kw):
        out = O.evaluate(sy, kw.get("r", r), R=kw.get("R"), zeta=kw.get("zeta"), lam=kw.get("lam"),
                         j1_b=kw["jas"][:A] if "jas" in kw else None,
                         j2=kw["jas"][A:] if "jas" in kw else None)
        return float((gl * out["logabs"]).sum() + (ge * out["e_loc"]).sum())

    base = dict(R=sy.R, zeta=sy.zeta, lam=sy.lam, jas=torch.cat([sy.j1_b, sy.j2]), r=r)
    h = 1e-5
    checks = [("R", (0, 0)), ("R", (2, 1)), ("zeta", (3,)), ("zeta", (20,)), ("lam", (1, 5)),
              ("lam", (7, 7)), ("jas", (0,)), ("jas", (3,)), ("jas", (4,)), ("r", (1, 2, 0)),
              ("r", (0, 7, 2))]
    for key, ix in checks:
        p = base[key].clone(); p[ix] += h
        fp = F(**{key: p})
        p = base[key].clone(); p[ix] -= h
        fm = F(**{key: p})
        fd = (fp - fm) / (2 * h)
        val = g[key][ix].item()
        assert abs(val - fd) <= 1e-6 * max(1.0, abs(fd)), (key, ix, val, fd)


def test_jacobi_formula_lambda():
    w, sy, r = tiny()
    r = r[:2]
    out = O.evaluate(sy, r, with_intermediates=True)
    g = O.forces_vjp(sy, r, torch.ones(2, dtype=DT), torch.zeros(2, dtype=DT))
    Phi, A = out["Phi"], out["A"]
    # d log|det W| / d Lambda = Phi_up^T W^{-T} Phi_dn, summed over walkers
    ref = torch.einsum('wim,wji,wjn->mn', Phi[:, :sy.n_up], A, Phi[:, sy.n_up:])
    assert torch.allclose(g["lam"], ref, rtol=1e-10, atol=1e-12)


def test_translation_sum_rule():
    w, sy, r = tiny()
    r = r[:2]
    for gl, ge in ((1.0, 0.0), (0.0, 1.0)):
        g = O.forces_vjp(sy, r, torch.full((2,), gl, dtype=DT), torch.full((2,), ge, dtype=DT))
        tot = g["R"].sum(0) + g["r"].sum(dim=(0, 1))
        scale = g["R"].abs().max().item()
        assert tot.abs().max().item() < 1e-9 * max(1.0, scale)


def test_basis_slater_finite_differences():
    # Slater s, p and d functions (eq. slater): gradients against central
    # differences of the values, Laplacians against Richardson second differences
    s, sy = make_system([[0.2, -0.1, 0.3]], [1.0], [(0, 0), (0, 1), (0, 2)], 1, 1, radial=1)
    pts = torch.tensor(np.random.default_rng(4).normal(size=(20, 3)), dtype=DT)
    psi, grad, lap = O.basis(sy, pts)
    h = 1e-5
    for ax in range(3):
        e = torch.zeros(3, dtype=DT); e[ax] = h
        fd = (O.basis(sy, pts + e)[0] - O.basis(sy, pts - e)[0]) / (2 * h)
        assert torch.allclose(grad[..., ax], fd, rtol=1e-6, atol=1e-9)
    def lap_fd(hh):
        tot = 0
        for ax in range(3):
            e = torch.zeros(3, dtype=DT); e[ax] = hh
            tot = tot + (O.basis(sy, pts + e)[0] - 2 * psi + O.basis(sy, pts - e)[0]) / hh ** 2
        return tot
    fd2 = (4 * lap_fd(5e-4) - lap_fd(1e-3)) / 3
    assert torch.allclose(lap, fd2, rtol=1e-5, atol=1e-6)
