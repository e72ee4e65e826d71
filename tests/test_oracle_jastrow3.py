"""Pins of the oracle's Jastrow-basis terms (onebody_J_inh, threebody_jastrow)
against closed forms, symmetries and finite differences.

* Zero coefficients reproduce the J1 + J2 Jastrow exactly.
* Rank one: with every M = v v^T the pair sum is
  sum_{i<j} a_i a_j = ((sum a)^2 - sum a^2) / 2, a_i = v . chi(r_i).
* One s orbital per nucleus with coefficients c: J1inh = c sum_i e^{-zeta r_ia^2}.
* Exchanging two same-spin electrons leaves J unchanged (and flips Psi).
* With M_uu = M_dd, symmetric M_ud and equal one-body coefficients, exchanging
  the up and down sets leaves J unchanged.
* Gradients and Laplacians against Richardson central differences.
"""
import dataclasses

import numpy as np
import torch

from oracle import jagp as O
from test_oracle_pins import _fd_grad_lap
from workloads import configs as C

DT = torch.float64


def _w():
    return C.jas3_4nuc_20e(n_walkers=4, n_steps=1)


def test_zero_coefficients_reduce_to_j1_j2():
    w = _w()
    s = w.system
    s0 = dataclasses.replace(s, j1_inh=np.zeros_like(s.j1_inh), j3=np.zeros_like(s.j3))
    base = dataclasses.replace(s, jb_center=None, jb_l=None, jb_m=None, jb_radial=None, jb_zeta=None,
                               j1_inh=None, j3=None)
    r = torch.tensor(w.r0)
    a = O.jastrow(O.from_workload_system(s0), r)
    b = O.jastrow(O.from_workload_system(base), r)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_rank_one_closed_form():
    w = _w()
    s = w.system
    LJ = s.n_jbasis
    v = np.random.default_rng(3).normal(size=LJ)
    M = np.outer(v, v)
    s1 = dataclasses.replace(s, j1_inh=np.zeros((2, LJ)), j3=np.stack([M, M, M]),
                             j1_form=0, j2_form=0)
    sy = O.from_workload_system(s1)
    r = torch.tensor(w.r0)
    J = O.jastrow(sy, r)[0]
    chi = O.basis(O._JBasisView(sy, sy.R), r)[0]
    a = chi @ torch.tensor(v)
    ref = 0.5 * (a.sum(1) ** 2 - (a * a).sum(1))
    assert torch.allclose(J, ref, rtol=1e-13, atol=1e-13)


def test_one_body_inhomogeneous_single_s_closed_form():
    w = _w()
    s = w.system
    A = len(s.Z)
    z = np.array([0.7, 1.1, 0.4, 2.0])
    c = np.array([0.3, -0.2])
    s1 = dataclasses.replace(
        s, jb_center=np.arange(A, dtype=np.int32), jb_l=np.zeros(A, np.int32), jb_m=np.zeros(A, np.int32),
        jb_radial=np.zeros(A, np.int32), jb_zeta=z, j1_inh=np.array([[c[0]] * A, [c[1]] * A]),
        j3=np.zeros((3, A, A)), j1_form=0, j2_form=0)
    r = w.r0
    d2 = ((r[:, :, None, :] - s.R[None, None]) ** 2).sum(-1)              # [Wk, N, A]
    e = np.exp(-z[None, None] * d2).sum(-1)                                 # [Wk, N]
    ref = c[0] * e[:, :s.n_up].sum(1) + c[1] * e[:, s.n_up:].sum(1)
    J = O.jastrow(O.from_workload_system(s1), torch.tensor(r))[0]
    assert np.allclose(J.numpy(), ref, rtol=1e-13, atol=1e-13)


def test_same_spin_exchange_and_spin_swap_symmetry():
    w = _w()
    s = w.system
    sy = O.from_workload_system(s)
    r = torch.tensor(w.r0)
    J = O.jastrow(sy, r)[0]
    for i, j in ((0, 3), (10, 17)):
        r2 = r.clone()
        r2[:, [i, j]] = r[:, [j, i]]
        assert torch.allclose(O.jastrow(sy, r2)[0], J, rtol=1e-13, atol=1e-12)
        la, sa = O.log_psi(sy, r)
        lb, sb = O.log_psi(sy, r2)
        assert torch.allclose(la, lb, rtol=1e-12) and torch.equal(sa, -sb)
    Mud = 0.5 * (s.j3[2] + s.j3[2].T)
    s2 = dataclasses.replace(s, j3=np.stack([s.j3[0], s.j3[0], Mud]), j1_inh=np.stack([s.j1_inh[0]] * 2))
    sy2 = O.from_workload_system(s2)
    nu = s.n_up
    swapped = torch.cat([r[:, nu:], r[:, :nu]], dim=1)
    assert torch.allclose(O.jastrow(sy2, swapped)[0], O.jastrow(sy2, r)[0], rtol=1e-13, atol=1e-12)


def test_gradient_and_laplacian_finite_differences():
    w = _w()
    sy = O.from_workload_system(w.system)
    r = torch.tensor(w.r0[:2])
    J, gJ, hJ = O.jastrow(sy, r)
    g, lap = _fd_grad_lap(lambda x: O.jastrow(sy, x)[0], r, h2=1e-3)
    assert torch.allclose(gJ, g, rtol=1e-7, atol=1e-7)
    assert torch.allclose(hJ, lap, rtol=1e-5, atol=1e-5)
