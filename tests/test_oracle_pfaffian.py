"""Pins of the Pfaffian oracle (Pfaffian wave function section).

  * Parlett-Reid against the definition (expansion along a row) for n <= 8,
    zero for odd n;
  * Pf(G)^2 = det(G); Pf(B M B^T) = det(B) Pf(M);
  * Pf([[0, X], [-X^T, 0]]) = (-1)^(n(n-1)/2) det(X) (eq:pfafftodet);
  * a Pfaffian whose pairing is singlet-only with unpaired orbitals of the up
    electrons only is the AGP determinant (the AGP section's special case):
    log|Psi|, E_loc and drift equal the determinant oracle's, signs related
    by (-1)^(n(n-1)/2);
  * drift and Laplacian of log Pf against finite differences with all four
    pairing components and unpaired orbitals of both spins;
  * exchanging two like-spin electrons changes the sign only.
"""
import dataclasses
import math

import numpy as np
import torch

from oracle import jagp as O
from oracle import pfaffian as PF
from workloads import configs as C

DT = torch.float64


def _skew(n, seed):
    g = torch.Generator().manual_seed(seed)
    a = torch.randn(n, n, generator=g, dtype=DT)
    return a - a.T


def test_parlett_reid_matches_definition():
    for n, seed in ((2, 1), (4, 2), (6, 3), (8, 4)):
        G = _skew(n, seed)
        ref = PF.pfaffian_expansion(G)
        s, l = PF.pfaffian_parlett_reid(G)
        assert s.item() == math.copysign(1.0, ref.item())
        assert abs(l.item() - math.log(abs(ref.item()))) <= 1e-12 * max(1.0, abs(l.item()))
    s, l = PF.pfaffian_parlett_reid(torch.zeros(5, 5, dtype=DT))
    assert s.item() == 0.0 and l.item() == -math.inf
    # the 2x2 case is the upper entry
    assert PF.pfaffian_expansion(torch.tensor([[0.0, 3.5], [-3.5, 0.0]], dtype=DT)).item() == 3.5


def test_pfaffian_square_congruence_and_block_form():
    G = _skew(22, 7)
    s, l = PF.pfaffian_parlett_reid(G)
    sd, ld = torch.linalg.slogdet(G)
    assert sd.item() > 0 and abs(2 * l.item() - ld.item()) <= 1e-11 * abs(ld.item())
    g = torch.Generator().manual_seed(8)
    B = torch.randn(22, 22, generator=g, dtype=DT)
    s2, l2 = PF.pfaffian_parlett_reid(B @ G @ B.T)
    sb, lb = torch.linalg.slogdet(B)
    assert s2.item() == s.item() * sb.item()
    assert abs(l2.item() - (l.item() + lb.item())) <= 1e-10 * max(1.0, abs(l2.item()))
    for n in (3, 4, 5, 11):
        X = torch.randn(n, n, generator=g, dtype=DT)
        M = torch.cat([torch.cat([torch.zeros(n, n, dtype=DT), X], 1),
                       torch.cat([-X.T, torch.zeros(n, n, dtype=DT)], 1)], 0)
        s3, l3 = PF.pfaffian_parlett_reid(M)
        sx, lx = torch.linalg.slogdet(X)
        assert s3.item() == sx.item() * (-1) ** (n * (n - 1) // 2)
        assert abs(l3.item() - lx.item()) <= 1e-11 * max(1.0, abs(lx.item()))


def _as_pfaffian(s):
    L = len(s.lam)
    k = s.n_up - s.n_dn
    return dataclasses.replace(s, pairing=1, pf_uu=np.zeros((L, L)), pf_dd=np.zeros((L, L)),
                               unpaired=np.asarray(s.unpaired).reshape(L, k), unpaired_dn=np.zeros((L, k)))


def test_singlet_pfaffian_is_the_agp_determinant():
    for w in (C.tiny_3nuc_10e(n_walkers=4), C.polarized_4nuc_20e(n_walkers=4)):
        s = w.system
        r = torch.tensor(w.r0)
        a = O.evaluate(O.from_workload_system(s), r)
        b = O.evaluate(O.from_workload_system(_as_pfaffian(s)), r)
        n = s.n_up
        for key in ("logabs", "e_kin", "e_loc", "drift"):
            err = ((a[key] - b[key]).abs() / a[key].abs().clamp(min=1.0)).max().item()
            assert err <= 1e-10, (s.name, key, err)
        assert torch.equal(b["sign"], a["sign"] * (-1) ** (n * (n - 1) // 2))


def test_pfaffian_derivatives_by_differences():
    w = C.pfaffian_4nuc_20e(n_walkers=2)
    sy = O.from_workload_system(w.system)
    assert sy.pf_uu.abs().max() > 0 and sy.unpaired_dn.abs().max() > 0
    r = torch.tensor(w.r0)
    out = O.evaluate(sy, r, with_intermediates=True)
    Jd = O.jastrow(sy, r)
    h = 1e-4
    for i in (0, 10, 11, 19):
        lap = torch.zeros(r.shape[0], dtype=DT)
        for ax in range(3):
            rp, rm = r.clone(), r.clone()
            rp[:, i, ax] += h
            rm[:, i, ax] -= h
            lp_, _ = O.log_psi(sy, rp)
            lm_, _ = O.log_psi(sy, rm)
            l0, _ = O.log_psi(sy, r)
            # central differences converge as h^2 (1.5e-6 at h = 1e-4, 1.5e-8 at 1e-5)
            hg = 1e-5
            rp2, rm2 = r.clone(), r.clone()
            rp2[:, i, ax] += hg
            rm2[:, i, ax] -= hg
            fd = (O.log_psi(sy, rp2)[0] - O.log_psi(sy, rm2)[0]) / (2 * hg)
            err = ((out["drift"][:, i, ax] - fd).abs() / fd.abs().clamp(min=1.0)).max().item()
            assert err <= 1e-7, (i, ax, err)
            # second differences of log Pf give lap log Pf = lap Pf / Pf - |grad log Pf|^2
            lap += (lp_ - 2 * l0 + lm_) / (h * h)
        D = out["D"][:, i]
        lapJ = Jd[2][:, i]
        ref = out["Ldet"][:, i] - (D * D).sum(-1) + lapJ
        assert torch.allclose(lap, ref, rtol=1e-4, atol=1e-3), (i, lap, ref)


def test_exchange_of_like_spin_electrons_changes_sign():
    w = C.pfaffian_4nuc_20e(n_walkers=3)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)
    l0, s0 = O.log_psi(sy, r)
    for a, b in ((0, 5), (12, 17)):
        rx = r.clone()
        rx[:, [a, b]] = rx[:, [b, a]]
        l1, s1 = O.log_psi(sy, rx)
        assert torch.allclose(l1, l0, rtol=1e-12, atol=1e-12)
        assert torch.equal(s1, -s0)
