"""The seeded input generator: deterministic, shapes and distributions as documented."""
import hashlib

import numpy as np

from workloads import configs as C


def _digest(w):
    h = hashlib.sha256()
    s = w.system
    for a in (s.R, s.Z, s.center, s.l, s.m, s.zeta, s.lam, s.j1_b, s.j2, w.r0):
        h.update(np.ascontiguousarray(a).tobytes())
    for a in (w.disp, w.unif):
        if a is not None:
            h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def test_deterministic():
    assert _digest(C.tiny_3nuc_10e()) == _digest(C.tiny_3nuc_10e())
    assert _digest(C.mol_40nuc_160e(n_walkers=8)) == _digest(C.mol_40nuc_160e(n_walkers=8))


def test_shapes_and_counts():
    w = C.tiny_3nuc_10e()
    s = w.system
    assert s.n_basis == 24 and (s.n_up, s.n_dn) == (5, 5) and w.r0.shape == (64, 10, 3)
    assert w.disp.shape == (1000, 64, 3) and w.unif.shape == (1000, 64)
    assert np.allclose(s.lam, s.lam.T)
    w = C.mol_40nuc_160e(n_walkers=4)
    s = w.system
    assert s.n_basis == 600 and s.Z.sum() == 160 and (s.n_up, s.n_dn) == (80, 80)
    assert np.allclose(s.lam, s.lam.T)
    d = np.linalg.norm(s.R[:, None] - s.R[None], axis=-1) + np.eye(40) * 10
    assert d.min() >= 1.0
    w = C.forces_20nuc_80e(n_walkers=4)
    assert w.system.n_basis == 300 and w.system.j2.shape == (8,)
    for n in C.MULTI_SIZES:
        s = C.multi_system(n, n_walkers=2).system
        assert s.n_basis == 4 * n and s.n_up == s.n_dn == n // 2


def test_electron_counts_largest_remainder():
    counts = C._electron_counts(np.array([2.0, 3.0, 5.0]), 10)
    assert counts.tolist() == [2, 3, 5]
    counts = C._electron_counts(np.array([1.0, 1.0, 1.0]), 4)
    assert counts.sum() == 4 and counts.max() - counts.min() <= 1
