"""Pins of the oracle's contracted basis (Contraction of the primitive atomic
basis section).  A contracted geminal is the primitive geminal with the
pairing matrix C Lambda C^T (and unpaired orbitals C U): W is built from
phi_c = sum_mu C[mu, c] psi_mu, so
    phi_c(r_i)^T Lambda phi_c(r_j) = psi(r_i)^T (C Lambda C^T) psi(r_j).
The pins evaluate both forms (the second through the uncontracted path, which
the other pins tie to closed forms and finite differences) and an identity
contraction.
"""
import dataclasses

import numpy as np
import torch

from oracle import jagp as O
from workloads import configs as C

KEYS = ("logabs", "e_kin", "e_loc", "drift")


def _rel(a, b):
    return ((a - b).abs() / b.abs().clamp(min=1.0)).max().item()


def _primitive_twin(s, unpaired=None):
    Cm = s.contraction
    lam_q = Cm @ s.lam @ Cm.T
    U = s.unpaired if unpaired is None else unpaired
    return dataclasses.replace(s, contraction=None, lam=lam_q, unpaired=Cm @ U)


def test_contracted_equals_primitive_with_transformed_pairing():
    w = C.contracted_4nuc_20e(n_walkers=6)
    s = w.system
    assert s.contraction.shape == (60, 28) and s.lam.shape == (28, 28)
    r = torch.tensor(w.r0)
    a = O.evaluate(O.from_workload_system(s), r)
    b = O.evaluate(O.from_workload_system(_primitive_twin(s)), r)
    for k in KEYS:
        assert _rel(a[k], b[k]) <= 1e-11, k
    assert torch.equal(a["sign"], b["sign"])
    # a move ratio through both forms
    rn = r[:, 3] + torch.tensor([0.2, -0.1, 0.3], dtype=torch.float64)
    ra = O.move_ratio(O.from_workload_system(s), r, 3, rn)
    rb = O.move_ratio(O.from_workload_system(_primitive_twin(s)), r, 3, rn)
    assert _rel(ra, rb) <= 1e-11


def test_identity_contraction_is_the_primitive_basis():
    w = C.slater_4nuc_20e(n_walkers=4)
    s = w.system
    L = len(s.zeta)
    sc = dataclasses.replace(s, contraction=np.eye(L))
    r = torch.tensor(w.r0)
    a = O.evaluate(O.from_workload_system(sc), r)
    b = O.evaluate(O.from_workload_system(s), r)
    for k in KEYS:
        assert _rel(a[k], b[k]) <= 1e-14, k


def test_contracted_unpaired_orbitals():
    # 11 up / 9 down: two unpaired columns phi_c(r_i)^T U
    w = C.contracted_4nuc_20e(n_walkers=4)
    s = w.system
    rng = np.random.default_rng(17)
    U = rng.standard_normal((s.lam.shape[0], 2)) / 5.0
    sp = dataclasses.replace(s, n_up=11, n_dn=9, unpaired=U)
    r = torch.tensor(w.r0)
    a = O.evaluate(O.from_workload_system(sp), r)
    b = O.evaluate(O.from_workload_system(_primitive_twin(sp)), r)
    for k in KEYS:
        assert _rel(a[k], b[k]) <= 1e-11, k


def test_contracted_orbital_derivatives_by_differences():
    # gradient and Laplacian of the contracted orbitals against central
    # differences of their values
    w = C.contracted_4nuc_20e(n_walkers=2)
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0)[:, :5]
    v, g, lap = O.agp_basis(sy, r)
    h = 1e-4
    fd_lap = torch.zeros_like(v)
    for ax in range(3):
        e = torch.zeros(3, dtype=torch.float64); e[ax] = h
        vp, vm = O.agp_basis(sy, r + e)[0], O.agp_basis(sy, r - e)[0]
        assert torch.allclose(g[..., ax], (vp - vm) / (2 * h), rtol=1e-6, atol=1e-7)
        fd_lap += (vp - 2 * v + vm) / (h * h)
    assert torch.allclose(lap, fd_lap, rtol=1e-4, atol=1e-4)
