"""Pins of the oracle's random-number path and of its Metropolis accept rule.

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) against the known-answer
vectors distributed with the authors' library (tests/golden); the map of two
32-bit words to a 53-bit uniform at closed-form points; the Box-Muller normals
by their distribution (a dropped factor, a wrong sign or a swapped cos/sin
changes a moment or a tail); and the chain's strict u < ratio^2 rule (VMC
section: the walk samples |Psi|^2) on hand-built steps whose ratios are known.
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import jagp as O
from oracle import philox as PH
from workloads import configs as C

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox4x32_10_kat.txt")


def kat_rows():
    rows = []
    for line in open(GOLD):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        assert len(w) == 10
        rows.append(w)
    return rows


def test_philox_known_answers():
    rows = kat_rows()
    assert len(rows) == 3
    for w in rows:
        ctr = np.array([w[0:4]], dtype=np.uint64)
        key = np.array([w[4:6]], dtype=np.uint64)
        out = PH.philox4x32_10(ctr, key)[0]
        assert [int(x) for x in out] == w[6:10], [hex(int(x)) for x in out]


def test_philox_is_a_bijection_of_the_counter_sample():
    # a keyed bijection: distinct counters give distinct blocks
    ctr = np.zeros((4096, 4), np.uint64)
    ctr[:, 0] = np.arange(4096)
    key = np.tile(np.array([[0x12345678, 0x9abcdef0]], np.uint64), (4096, 1))
    out = PH.philox4x32_10(ctr, key)
    assert len({tuple(int(x) for x in r) for r in out}) == 4096


def test_words_to_uniform_closed_forms():
    u = PH.words_to_uniform
    assert u(0, 0) == 0.0
    assert u(0x80000000, 0) == 0.5
    assert u(0x40000000, 0) == 0.25
    # the 11 low bits are dropped: 53 random bits
    assert u(0, 0x7FF) == 0.0
    assert u(0, 0x800) == 2.0 ** -53
    # the largest value is 1 - 2^-53 < 1
    top = u(0xFFFFFFFF, 0xFFFFFFFF)
    assert top == 1.0 - 2.0 ** -53 and top < 1.0
    # monotone in the 64-bit integer
    assert u(0x12345678, 0x9ABCDEF0) < u(0x12345678, 0x9ABCE000)


def _ks_normal(x):
    x = np.sort(np.asarray(x))
    n = len(x)
    cdf = 0.5 * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    d = max(np.max(np.arange(1, n + 1) / n - cdf), np.max(cdf - np.arange(0, n) / n))
    return d * math.sqrt(n)


def test_metropolis_draws_distribution():
    n = 60000
    sigma = 0.3
    disp, unif = PH.metropolis_draws(20020, 3, np.arange(n), 17, sigma)
    assert disp.shape == (n, 3) and unif.shape == (n,)
    assert np.all(unif >= 0.0) and np.all(unif < 1.0)
    z = disp / sigma
    for k in range(3):
        # mean 0, variance 1, zero skew and excess kurtosis 0 within a few
        # standard errors of n draws
        assert abs(z[:, k].mean()) < 5 / math.sqrt(n)
        assert abs(z[:, k].var() - 1.0) < 5 * math.sqrt(2.0 / n)
        assert abs((z[:, k] ** 3).mean()) < 5 * math.sqrt(15.0 / n)
        assert abs((z[:, k] ** 4).mean() - 3.0) < 5 * math.sqrt(96.0 / n)
        # Kolmogorov statistic well below its 0.1 % quantile (1.95)
        assert _ks_normal(z[:, k]) < 1.95
    # the Box-Muller pair (components 0, 1) is uncorrelated, also in squares
    c = np.corrcoef(z[:, 0], z[:, 1])[0, 1]
    c2 = np.corrcoef(z[:, 0] ** 2, z[:, 1] ** 2)[0, 1]
    assert abs(c) < 5 / math.sqrt(n) and abs(c2) < 5 / math.sqrt(n)
    # the acceptance uniform: Kolmogorov statistic against U[0, 1)
    s = np.sort(unif)
    d = max(np.max(np.arange(1, n + 1) / n - s), np.max(s - np.arange(0, n) / n)) * math.sqrt(n)
    assert d < 1.95


def test_metropolis_draws_depend_on_every_counter_field():
    base = PH.metropolis_draws(7, 1, np.arange(8), 5, 1.0)
    for args in ((8, 1, 5), (7, 2, 5), (7, 1, 6)):
        other = PH.metropolis_draws(args[0], args[1], np.arange(8), args[2], 1.0)
        assert not np.allclose(base[0], other[0]) and not np.allclose(base[1], other[1])
    shifted = PH.metropolis_draws(7, 1, np.arange(1, 9), 5, 1.0)
    assert np.array_equal(shifted[0][:-1], base[0][1:]) and np.array_equal(shifted[1][:-1], base[1][1:])


def _one_walker():
    w = C.tiny_3nuc_10e(n_walkers=1, n_steps=1)
    sy = O.from_workload_system(w.system)
    return sy, torch.tensor(w.r0)


def test_run_chain_accepts_strictly_below_ratio_squared():
    sy, r0 = _one_walker()
    zero = torch.zeros(1, 1, 3, dtype=torch.float64)
    # no displacement: ratio is exactly 1, so u = 1 (not below 1) must reject
    # and the largest uniform below 1 must accept
    r, ratios, acc = O.run_chain(sy, r0, zero, torch.tensor([[1.0]], dtype=torch.float64))
    assert ratios[0, 0].item() == 1.0 and not bool(acc[0, 0])
    r, ratios, acc = O.run_chain(sy, r0, zero, torch.tensor([[1.0 - 2.0 ** -53]], dtype=torch.float64))
    assert bool(acc[0, 0])


def test_run_chain_compares_with_the_square_of_the_ratio():
    sy, r0 = _one_walker()
    e = 0
    # a displacement whose |ratio| lies well inside (0, 1)
    d = None
    for step in np.linspace(0.2, 3.0, 60):
        cand = torch.tensor([[[step, -0.5 * step, 0.3 * step]]], dtype=torch.float64)
        q = O.move_ratio(sy, r0, e, r0[:, e] + cand[0]).abs().item()
        if 0.3 < q < 0.8:
            d, ratio = cand, q
            break
    assert d is not None
    between = torch.tensor([[0.5 * (ratio * ratio + ratio)]], dtype=torch.float64)   # ratio^2 < u < |ratio|
    r, ratios, acc = O.run_chain(sy, r0, d, between)
    assert abs(abs(ratios[0, 0].item()) - ratio) < 1e-12
    assert not bool(acc[0, 0]) and torch.equal(r, r0)
    below = torch.tensor([[0.5 * ratio * ratio]], dtype=torch.float64)
    r, ratios, acc = O.run_chain(sy, r0, d, below)
    assert bool(acc[0, 0])
    moved = r0.clone()
    moved[:, e] += d[0]
    assert torch.equal(r, moved)


def test_run_chain_ratios_chain_through_accepted_states():
    # two steps of the same electron: the second ratio is taken from the
    # accepted state, so the product of the ratios is Psi(final)/Psi(initial)
    sy, r0 = _one_walker()
    d = torch.tensor([[[0.1, 0.0, -0.05]], [[-0.02, 0.07, 0.0]]], dtype=torch.float64)
    u = torch.zeros(2, 1, dtype=torch.float64)   # always accept (ratio^2 > 0)
    r, ratios, acc = O.run_chain(sy, r0, d, u, e_start=4, n_steps=2)
    assert bool(acc.all())
    # electron 4 then electron 5
    la, sa = O.log_psi(sy, r0)
    lb, sb = O.log_psi(sy, r)
    full = (sa * sb * torch.exp(lb - la)).item()
    assert abs(ratios.prod().item() - full) <= 1e-12 * max(1.0, abs(full))
    assert torch.equal(r[:, 4], r0[:, 4] + d[0, 0]) and torch.equal(r[:, 5], r0[:, 5] + d[1, 0])
