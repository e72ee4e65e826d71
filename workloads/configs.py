"""Seeded synthetic JAGP systems and walker/move arrays.

This module draws inputs only: nuclear geometry, the basis specification,
the pairing matrix Lambda, Jastrow parameters, initial electron positions and
the random numbers of a Metropolis chain.  It computes nothing of the wave
function, so both the CPU oracle and the HIP path can take their inputs from
it without sharing any of the method's arithmetic.

Conventions (shared by both sides):
  * Hartree atomic units (bohr, Hartree).
  * Electrons 0..n_up-1 have spin up, n_up..N-1 spin down (the paper's AGP
    section orders the electrons this way).
  * A basis function is (center, l, m, zeta, radial).  The angular factor is
    an unnormalised real solid harmonic; component index m means
        l=0: 1
        l=1: x, y, z                          (m = 0, 1, 2)
        l=2: xy, yz, zx, x^2-y^2, 2z^2-x^2-y^2 (m = 0..4)
    radial 0 is Gaussian exp(-zeta r^2), radial 1 is Slater exp(-zeta r).
  * Jastrow one-body form: 0 none, 1 exponential u, 2 Pade u; one b per nucleus.
  * Jastrow two-body form: 0 none, 1 Pade (params b_para, b_anti),
    2 Pade series (params b, a1, a2, a3 for parallel spins then the same four
    for antiparallel spins).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Dict, List, Optional

import numpy as np

SEED_BASE = 200207401

# Shell-component counts per angular momentum (real solid harmonics).
N_COMP = {0: 1, 1: 3, 2: 5}


@dataclass
class System:
    """One molecular system: nuclei, basis, pairing matrix and Jastrow."""
    name: str
    R: np.ndarray            # [n_nuc, 3] float64
    Z: np.ndarray            # [n_nuc]    float64
    center: np.ndarray       # [L] int32 index into R
    l: np.ndarray            # [L] int32
    m: np.ndarray            # [L] int32 component index
    zeta: np.ndarray         # [L] float64
    radial: np.ndarray       # [L] int32 (0 Gaussian, 1 Slater)
    lam: np.ndarray          # [L, L] float64 pairing coefficients
    n_up: int
    n_dn: int
    unpaired: np.ndarray     # [L, n_up - n_dn] float64 (empty when paired)
    j1_form: int
    j1_b: np.ndarray         # [n_nuc] float64
    j2_form: int
    j2: np.ndarray           # [n_j2] float64
    refresh_every: int = 32
    band_cutoff: float = 0.0  # 0 means dense Lambda
    # Jastrow basis chi (onebody_J_inh, threebody_jastrow); absent when jb_zeta is None
    jb_center: Optional[np.ndarray] = None   # [LJ] int32
    jb_l: Optional[np.ndarray] = None        # [LJ] int32
    jb_m: Optional[np.ndarray] = None        # [LJ] int32
    jb_radial: Optional[np.ndarray] = None   # [LJ] int32
    jb_zeta: Optional[np.ndarray] = None     # [LJ] float64
    j1_inh: Optional[np.ndarray] = None      # [2, LJ] coefficients of chi for up / down electrons
    j3: Optional[np.ndarray] = None          # [3, LJ, LJ] up-up, down-down (symmetric), up-down
    # contraction of the primitive basis: center .. radial describe the
    # primitives, lam / unpaired act on phi_c = sum_mu C[mu, c] psi_mu
    contraction: Optional[np.ndarray] = None  # [L_primitive, L] float64
    # Pfaffian pairing (pairing = 1, eq:g): lam is the unlike-spin block A^{ud},
    # pf_uu / pf_dd the skew-symmetric same-spin blocks, unpaired / unpaired_dn
    # the unpaired orbitals of up / down electrons (k columns, N + k even)
    pairing: int = 0
    pf_uu: Optional[np.ndarray] = None       # [L, L]
    pf_dd: Optional[np.ndarray] = None       # [L, L]
    unpaired_dn: Optional[np.ndarray] = None  # [L, k]

    @property
    def n_jbasis(self) -> int:
        return 0 if self.jb_zeta is None else int(self.jb_zeta.shape[0])

    @property
    def n_elec(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_basis(self) -> int:
        return int(self.zeta.shape[0])

    @property
    def n_nuc(self) -> int:
        return int(self.Z.shape[0])

    @property
    def jastrow_params(self) -> np.ndarray:
        """The Jastrow parameter vector: one-body b per nucleus, then two-body."""
        return np.concatenate([self.j1_b, self.j2]).astype(np.float64)


@dataclass
class Workload:
    """A system plus its walkers and the random numbers of a chain."""
    system: System
    r0: np.ndarray                       # [Wk, N, 3] float64 initial positions
    disp: Optional[np.ndarray] = None    # [n_steps, Wk, 3] Gaussian displacements
    unif: Optional[np.ndarray] = None    # [n_steps, Wk] uniforms in [0, 1)
    sigma: float = 0.3
    extra: Dict[str, object] = field(default_factory=dict)

    @property
    def n_walkers(self) -> int:
        return int(self.r0.shape[0])


# --------------------------------------------------------------------------
# geometry and basis drawing
# --------------------------------------------------------------------------

def _place_nuclei(rng, n, box, min_sep=1.0):
    """Uniform positions in [0, box)^3, rejecting pairs closer than min_sep."""
    pts: List[np.ndarray] = []
    while len(pts) < n:
        p = rng.uniform(0.0, box, size=3)
        if all(np.linalg.norm(p - q) >= min_sep for q in pts):
            pts.append(p)
    return np.array(pts, dtype=np.float64)


def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size=size))


def _shell_basis(rng, n_nuc, shells, zlo, zhi):
    """Per nucleus, the listed shells (angular momenta); one zeta per shell,
    shared by the shell's components."""
    center, l, m, zeta = [], [], [], []
    for a in range(n_nuc):
        for ll in shells:
            z = float(_log_uniform(rng, zlo, zhi, 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a)
                l.append(ll)
                m.append(mm)
                zeta.append(z)
    return (np.array(center, np.int32), np.array(l, np.int32),
            np.array(m, np.int32), np.array(zeta, np.float64))


def _sym_gaussian(rng, L, scale):
    """Symmetric matrix: upper triangle (with diagonal) N(0,1)*scale, mirrored."""
    a = rng.standard_normal((L, L)) * scale
    u = np.triu(a)
    return u + np.triu(u, 1).T


def _electron_counts(Z, n_elec):
    """Electrons per nucleus in proportion to Z (largest-remainder rounding)."""
    share = Z / Z.sum() * n_elec
    base = np.floor(share).astype(int)
    rem = n_elec - base.sum()
    order = np.argsort(-(share - base), kind="stable")
    base[order[:rem]] += 1
    return base


def _initial_positions(rng, R, Z, n_up, n_dn, n_walkers, spread=1.0):
    """Electrons at R_a + N(0, spread^2); spins alternate over the per-nucleus
    list (the electrons past 2 n_dn are up), then up electrons are put first."""
    counts = _electron_counts(Z, n_up + n_dn)
    owner = np.repeat(np.arange(len(Z)), counts)
    if n_up == n_dn:
        up_idx = owner[0::2]
        dn_idx = owner[1::2]
    else:
        pair = owner[:2 * n_dn]
        up_idx = np.concatenate([pair[0::2], owner[2 * n_dn:]])
        dn_idx = pair[1::2]
    assert len(up_idx) == n_up and len(dn_idx) == n_dn, (len(up_idx), len(dn_idx))
    order = np.concatenate([up_idx, dn_idx])
    r0 = R[order][None, :, :] + spread * rng.standard_normal((n_walkers, len(order), 3))
    return r0.astype(np.float64)


def _chain_arrays(rng, n_steps, n_walkers, sigma):
    disp = sigma * rng.standard_normal((n_steps, n_walkers, 3))
    unif = rng.random((n_steps, n_walkers))
    return disp.astype(np.float64), unif.astype(np.float64)


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------

def tiny_3nuc_10e(n_walkers=64, n_steps=1000, seed_offset=1) -> Workload:
    """3 nuclei (Z = 2, 3, 5) in a 6-bohr cube, 10 electrons (5 up / 5 down),
    per atom 6 s functions and 2 single p functions whose axes cycle over the
    system (x,y | z,x | y,z), zeta log-uniform in [0.1, 10] (L = 24),
    Lambda symmetric N(0,1)/24, Pade one- and two-body Jastrow with b = 1."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([2.0, 3.0, 5.0])
    R = _place_nuclei(rng, 3, 6.0)
    p_axes = [(0, 1), (2, 0), (1, 2)]
    center, l, m = [], [], []
    for a in range(3):
        for _ in range(6):
            center.append(a); l.append(0); m.append(0)
        for ax in p_axes[a]:
            center.append(a); l.append(1); m.append(ax)
    L = len(center)
    zeta = _log_uniform(rng, 0.1, 10.0, L)
    lam = _sym_gaussian(rng, L, 1.0 / 24.0)
    sysd = System(
        name="tiny_3nuc_10e", R=R, Z=Z,
        center=np.array(center, np.int32), l=np.array(l, np.int32),
        m=np.array(m, np.int32), zeta=zeta.astype(np.float64),
        radial=np.zeros(L, np.int32), lam=lam, n_up=5, n_dn=5,
        unpaired=np.zeros((L, 0)), j1_form=2, j1_b=np.ones(3),
        j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32)
    r0 = _initial_positions(rng, R, Z, 5, 5, n_walkers)
    disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def slater_4nuc_20e(n_walkers=32, n_steps=200, seed_offset=5) -> Workload:
    """Mixed Slater / Gaussian basis (eq. slater, eq. gaussian): 4 nuclei
    (Z = 2, 4, 6, 8) in an 8-bohr cube, 20 electrons (10 up / 10 down), per
    atom 2 Slater s + 1 Gaussian s + 1 Slater p + 1 Gaussian p + 1 Slater d
    shells (14 functions, L = 56); Slater zeta log-uniform in [0.5, 5], Gaussian
    zeta log-uniform in [0.1, 10]; Lambda symmetric N(0,1)/56; Pade one- and
    two-body Jastrow with b = 1."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([2.0, 4.0, 6.0, 8.0])
    R = _place_nuclei(rng, 4, 8.0)
    shells = [(0, 1), (0, 1), (0, 0), (1, 1), (1, 0), (2, 1)]   # (l, radial)
    center, l, m, zeta, radial = [], [], [], [], []
    for a in range(4):
        for ll, rad in shells:
            z = float(_log_uniform(rng, 0.5, 5.0, 1)[0] if rad else _log_uniform(rng, 0.1, 10.0, 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a); l.append(ll); m.append(mm); zeta.append(z); radial.append(rad)
    L = len(center)
    lam = _sym_gaussian(rng, L, 1.0 / L)
    sysd = System(
        name="slater_4nuc_20e", R=R, Z=Z,
        center=np.array(center, np.int32), l=np.array(l, np.int32),
        m=np.array(m, np.int32), zeta=np.array(zeta, np.float64),
        radial=np.array(radial, np.int32), lam=lam, n_up=10, n_dn=10,
        unpaired=np.zeros((L, 0)), j1_form=2, j1_b=np.ones(4),
        j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32)
    r0 = _initial_positions(rng, R, Z, 10, 10, n_walkers)
    disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def add_jastrow_basis(sysd: System, rng, shells=((0, 0), (0, 0), (1, 0)), zrange=(0.2, 3.0),
                      scale_1=0.1, scale_3=0.05) -> System:
    """A copy of sysd with a Jastrow basis of the given (l, radial) shells on
    every nucleus (zeta log-uniform in zrange, one per shell), one-body
    inhomogeneous coefficients N(0, scale_1^2) per spin, and three/four-body
    matrices: up-up and down-down symmetric N(0, scale_3^2) (upper triangle
    mirrored), up-down N(0, scale_3^2)."""
    center, l, m, radial, zeta = [], [], [], [], []
    for a in range(len(sysd.Z)):
        for ll, rad in shells:
            z = float(_log_uniform(rng, zrange[0], zrange[1], 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a); l.append(ll); m.append(mm); radial.append(rad); zeta.append(z)
    LJ = len(center)
    j3 = np.stack([_sym_gaussian(rng, LJ, scale_3), _sym_gaussian(rng, LJ, scale_3),
                   rng.standard_normal((LJ, LJ)) * scale_3])
    return replace(sysd, name=sysd.name + "_j3", jb_center=np.array(center, np.int32),
                   jb_l=np.array(l, np.int32), jb_m=np.array(m, np.int32),
                   jb_radial=np.array(radial, np.int32), jb_zeta=np.array(zeta, np.float64),
                   j1_inh=rng.standard_normal((2, LJ)) * scale_1, j3=j3)


def jas3_4nuc_20e(n_walkers=32, n_steps=200, seed_offset=6) -> Workload:
    """The geometry and Gaussian geminal basis of a 4-nucleus, 20-electron
    system (Z = 2, 4, 6, 8, 8-bohr cube, per atom 3 s + 1 p + 1 d Gaussian
    shells, L = 44, Lambda symmetric N(0,1)/44, Pade J1 and J2 with b = 1) with
    a Jastrow basis of 2 s + 1 p Gaussian shells per atom (LJ = 20), J1
    inhomogeneous and J3/4 terms (onebody_J_inh, threebody_jastrow)."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([2.0, 4.0, 6.0, 8.0])
    R = _place_nuclei(rng, 4, 8.0)
    center, l, m = [], [], []
    zeta = []
    for a in range(4):
        for ll in (0, 0, 0, 1, 2):
            z = float(_log_uniform(rng, 0.1, 10.0, 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a); l.append(ll); m.append(mm); zeta.append(z)
    L = len(center)
    sysd = System(
        name="jas3_4nuc_20e", R=R, Z=Z, center=np.array(center, np.int32), l=np.array(l, np.int32),
        m=np.array(m, np.int32), zeta=np.array(zeta, np.float64), radial=np.zeros(L, np.int32),
        lam=_sym_gaussian(rng, L, 1.0 / L), n_up=10, n_dn=10, unpaired=np.zeros((L, 0)),
        j1_form=2, j1_b=np.ones(4), j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32)
    sysd = add_jastrow_basis(sysd, rng)
    r0 = _initial_positions(rng, R, Z, 10, 10, n_walkers)
    disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def contracted_4nuc_20e(n_walkers=32, n_steps=200, seed_offset=7) -> Workload:
    """A contracted (hybrid) basis (Contraction of the primitive atomic basis
    section): 4 nuclei (Z = 2, 4, 6, 8) in an 8-bohr cube, 20 electrons
    (10 up / 10 down); per atom 15 primitives (3 Gaussian s, 1 Slater s,
    2 Gaussian p, 1 Gaussian d shells; Gaussian zeta log-uniform in [0.1, 10],
    Slater in [0.5, 5]) and 7 contracted orbitals, each a combination of all of
    its atom's primitives with N(0, 1/16) coefficients (60 primitives, L = 28);
    Lambda symmetric N(0,1)/28; Pade J1 and J2 with b = 1."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([2.0, 4.0, 6.0, 8.0])
    R = _place_nuclei(rng, 4, 8.0)
    shells = [(0, 0), (0, 0), (0, 0), (0, 1), (1, 0), (1, 0), (2, 0)]   # (l, radial)
    center, l, m, zeta, radial = [], [], [], [], []
    for a in range(4):
        for ll, rad in shells:
            z = float(_log_uniform(rng, 0.5, 5.0, 1)[0] if rad else _log_uniform(rng, 0.1, 10.0, 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a); l.append(ll); m.append(mm); zeta.append(z); radial.append(rad)
    Lq, n_con = len(center), 7
    center = np.array(center, np.int32)
    C = np.zeros((Lq, 4 * n_con))
    for a in range(4):
        prim = np.nonzero(center == a)[0]
        C[np.ix_(prim, np.arange(a * n_con, (a + 1) * n_con))] = rng.standard_normal((len(prim), n_con)) / 4.0
    L = C.shape[1]
    sysd = System(
        name="contracted_4nuc_20e", R=R, Z=Z, center=center, l=np.array(l, np.int32),
        m=np.array(m, np.int32), zeta=np.array(zeta, np.float64), radial=np.array(radial, np.int32),
        lam=_sym_gaussian(rng, L, 1.0 / L), n_up=10, n_dn=10, unpaired=np.zeros((L, 0)),
        j1_form=2, j1_b=np.ones(4), j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32, contraction=C)
    r0 = _initial_positions(rng, R, Z, 10, 10, n_walkers)
    disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def polarized_4nuc_20e(n_walkers=32, n_steps=200, seed_offset=8) -> Workload:
    """A spin-polarized geminal with unpaired orbitals (eq:wfAGPunpaired):
    4 nuclei (Z = 2, 4, 6, 8) in an 8-bohr cube, 20 electrons, 11 up / 9 down
    (two unpaired orbitals); per atom 3 s + 1 p + 1 d Gaussian shells (L = 44,
    zeta log-uniform in [0.1, 10]); Lambda symmetric N(0,1)/44; unpaired
    coefficients N(0, 1/44); Pade J1 and J2 with b = 1."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([2.0, 4.0, 6.0, 8.0])
    R = _place_nuclei(rng, 4, 8.0)
    center, l, m, zeta = [], [], [], []
    for a in range(4):
        for ll in (0, 0, 0, 1, 2):
            z = float(_log_uniform(rng, 0.1, 10.0, 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a); l.append(ll); m.append(mm); zeta.append(z)
    L = len(center)
    sysd = System(
        name="polarized_4nuc_20e", R=R, Z=Z, center=np.array(center, np.int32), l=np.array(l, np.int32),
        m=np.array(m, np.int32), zeta=np.array(zeta, np.float64), radial=np.zeros(L, np.int32),
        lam=_sym_gaussian(rng, L, 1.0 / L), n_up=11, n_dn=9,
        unpaired=rng.standard_normal((L, 2)) / np.sqrt(L),
        j1_form=2, j1_b=np.ones(4), j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32)
    r0 = _initial_positions(rng, R, Z, 11, 9, n_walkers)
    disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def _skew_gaussian(rng, L, scale):
    u = rng.standard_normal((L, L)) * scale
    return np.triu(u, 1) - np.triu(u, 1).T


def pfaffian_4nuc_20e(n_walkers=32, n_steps=200, seed_offset=9) -> Workload:
    """A Pfaffian wave function with all four pairing components (eq:g):
    4 nuclei (Z = 2, 4, 6, 8) in an 8-bohr cube, 20 electrons, 11 up / 9 down
    with k = 2 unpaired orbitals per spin (G~ is 22 x 22); per atom
    3 s + 1 p + 1 d Gaussian shells (L = 44, zeta log-uniform in [0.1, 10]);
    A^{ud} = singlet (symmetric N(0,1)/44) + triplet-zero part (skew N(0, 0.3^2)/44);
    A^{uu}, A^{dd} skew N(0, 0.5^2)/44; unpaired coefficients N(0, 1/44) for
    each spin; Pade J1 and J2 with b = 1."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([2.0, 4.0, 6.0, 8.0])
    R = _place_nuclei(rng, 4, 8.0)
    center, l, m, zeta = [], [], [], []
    for a in range(4):
        for ll in (0, 0, 0, 1, 2):
            z = float(_log_uniform(rng, 0.1, 10.0, 1)[0])
            for mm in range(N_COMP[ll]):
                center.append(a); l.append(ll); m.append(mm); zeta.append(z)
    L = len(center)
    aud = _sym_gaussian(rng, L, 1.0 / L) + _skew_gaussian(rng, L, 0.3 / L)
    sysd = System(
        name="pfaffian_4nuc_20e", R=R, Z=Z, center=np.array(center, np.int32), l=np.array(l, np.int32),
        m=np.array(m, np.int32), zeta=np.array(zeta, np.float64), radial=np.zeros(L, np.int32),
        lam=aud, n_up=11, n_dn=9, unpaired=rng.standard_normal((L, 2)) / np.sqrt(L),
        j1_form=2, j1_b=np.ones(4), j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32,
        pairing=1, pf_uu=_skew_gaussian(rng, L, 0.5 / L), pf_dd=_skew_gaussian(rng, L, 0.5 / L),
        unpaired_dn=rng.standard_normal((L, 2)) / np.sqrt(L))
    r0 = _initial_positions(rng, R, Z, 11, 9, n_walkers)
    disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def mol_40nuc_160e(n_walkers=1024, n_steps=0, seed_offset=2) -> Workload:
    """40 nuclei (20 H, 10 C, 10 O) in a 20-bohr cube (min separation 1 bohr),
    160 electrons (80/80), per atom 4 s + 2 p + 1 d shells (15 functions,
    L = 600), zeta log-uniform in [0.05, 20], Lambda = C C^T (C 600x80,
    N(0,1)/sqrt(600)) plus 1e-3 times a symmetric N(0,1) matrix, Pade
    Jastrow b = 1, refresh every 32 moves."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([1.0] * 20 + [6.0] * 10 + [8.0] * 10)
    R = _place_nuclei(rng, 40, 20.0)
    center, l, m, zeta = _shell_basis(rng, 40, [0, 0, 0, 0, 1, 1, 2], 0.05, 20.0)
    L = len(zeta)
    C = rng.standard_normal((L, 80)) / np.sqrt(L)
    lam = C @ C.T + 1e-3 * _sym_gaussian(rng, L, 1.0)
    sysd = System(
        name="mol_40nuc_160e", R=R, Z=Z, center=center, l=l, m=m, zeta=zeta,
        radial=np.zeros(L, np.int32), lam=lam, n_up=80, n_dn=80,
        unpaired=np.zeros((L, 0)), j1_form=2, j1_b=np.ones(40),
        j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32)
    r0 = _initial_positions(rng, R, Z, 80, 80, n_walkers)
    disp = unif = None
    if n_steps:
        disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def forces_20nuc_80e(n_walkers=512, n_steps=0, seed_offset=3) -> Workload:
    """20 nuclei (10 H, 5 C, 5 O) in a 15.9-bohr cube, 80 electrons (40/40),
    per atom 6 s + 3 p shells (15 functions, L = 300), zeta log-uniform in
    [0.05, 20], Lambda symmetric N(0,1)/300, one-body Pade b = 1, two-body
    8-parameter Pade series."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = np.array([1.0] * 10 + [6.0] * 5 + [8.0] * 5)
    R = _place_nuclei(rng, 20, 15.9)
    center, l, m, zeta = _shell_basis(rng, 20, [0] * 6 + [1] * 3, 0.05, 20.0)
    L = len(zeta)
    lam = _sym_gaussian(rng, L, 1.0 / 300.0)
    # b, a1, a2, a3 for parallel spins, then for antiparallel spins
    j2 = np.array([1.0, 0.05, -0.02, 0.01, 1.0, 0.08, -0.03, 0.01])
    sysd = System(
        name="forces_20nuc_80e", R=R, Z=Z, center=center, l=l, m=m, zeta=zeta,
        radial=np.zeros(L, np.int32), lam=lam, n_up=40, n_dn=40,
        unpaired=np.zeros((L, 0)), j1_form=2, j1_b=np.ones(20),
        j2_form=2, j2=j2, refresh_every=32)
    r0 = _initial_positions(rng, R, Z, 40, 40, n_walkers)
    disp = unif = None
    if n_steps:
        disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def pfaffian_20nuc_80e(n_walkers=512, n_steps=0, seed_offset=10) -> Workload:
    """The 80-electron system of forces_20nuc_80e (20 nuclei, 40/40 electrons,
    L = 300) as a Pfaffian (G~ 80 x 80): A^{ud} = its singlet Lambda plus a
    triplet-zero part skew N(0, 0.3^2)/300, A^{uu}, A^{dd} skew N(0, 0.5^2)/300,
    no unpaired orbitals."""
    w = forces_20nuc_80e(n_walkers=n_walkers, n_steps=n_steps)
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    s = w.system
    L = len(s.lam)
    sysd = replace(s, name="pfaffian_20nuc_80e", lam=s.lam + _skew_gaussian(rng, L, 0.3 / L), pairing=1,
                   pf_uu=_skew_gaussian(rng, L, 0.5 / L), pf_dd=_skew_gaussian(rng, L, 0.5 / L),
                   unpaired_dn=np.zeros((L, 0)))
    disp, unif = w.disp, w.unif
    if n_steps and disp is None:
        disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, w.r0, disp, unif, 0.3)


MULTI_SIZES = (16, 32, 48, 64, 96, 128, 192, 256)


def multi_system(n_elec: int, n_walkers=256, n_steps=0, seed_offset=4) -> Workload:
    """One member of the uneven multi-system batch: n_elec electrons (equal
    spins), n_elec/2 helium-like nuclei (Z = 2) in a cube of side
    (100 n_elec)^(1/3), 5 s + 1 p shells per nucleus (L = 4 n_elec), zeta
    log-uniform in [0.1, 10], Lambda symmetric N(0,1)/L, Pade Jastrow b = 1."""
    rng = np.random.default_rng(SEED_BASE + seed_offset * 1000 + n_elec)
    n_nuc = n_elec // 2
    Z = np.full(n_nuc, 2.0)
    R = _place_nuclei(rng, n_nuc, (100.0 * n_elec) ** (1.0 / 3.0))
    center, l, m, zeta = _shell_basis(rng, n_nuc, [0] * 5 + [1], 0.1, 10.0)
    L = len(zeta)
    lam = _sym_gaussian(rng, L, 1.0 / L)
    sysd = System(
        name=f"multi_{n_elec}e", R=R, Z=Z, center=center, l=l, m=m, zeta=zeta,
        radial=np.zeros(L, np.int32), lam=lam, n_up=n_elec // 2, n_dn=n_elec // 2,
        unpaired=np.zeros((L, 0)), j1_form=2, j1_b=np.ones(n_nuc),
        j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=32)
    r0 = _initial_positions(rng, R, Z, n_elec // 2, n_elec // 2, n_walkers)
    disp = unif = None
    if n_steps:
        disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def large_256nuc_1024e(n_walkers=256, n_steps=0, seed_offset=5) -> Workload:
    """256 nuclei (Z uniform on 1..8) in a 40-bohr cube, 1024 electrons
    (512/512), per atom 5 s + 2 p + 1 d shells (16 functions, L = 4096),
    zeta log-uniform in [0.05, 20], Lambda symmetric N(0,1)/sqrt(nnz per
    row), zero between functions whose centres are 8 bohr or more apart,
    Pade Jastrow b = 1, refresh every 64 moves."""
    rng = np.random.default_rng(SEED_BASE + seed_offset)
    Z = rng.integers(1, 9, size=256).astype(np.float64)
    R = _place_nuclei(rng, 256, 40.0)
    center, l, m, zeta = _shell_basis(rng, 256, [0] * 5 + [1, 1, 2], 0.05, 20.0)
    L = len(zeta)
    dist = np.linalg.norm(R[:, None, :] - R[None, :, :], axis=-1)
    near = dist[center][:, center] < 8.0
    nnz_row = near.sum(axis=1).mean()
    lam = _sym_gaussian(rng, L, 1.0 / np.sqrt(nnz_row)) * near
    sysd = System(
        name="large_256nuc_1024e", R=R, Z=Z, center=center, l=l, m=m, zeta=zeta,
        radial=np.zeros(L, np.int32), lam=lam, n_up=512, n_dn=512,
        unpaired=np.zeros((L, 0)), j1_form=2, j1_b=np.ones(256),
        j2_form=1, j2=np.array([1.0, 1.0]), refresh_every=64, band_cutoff=8.0)
    r0 = _initial_positions(rng, R, Z, 512, 512, n_walkers)
    disp = unif = None
    if n_steps:
        disp, unif = _chain_arrays(rng, n_steps, n_walkers, 0.3)
    return Workload(sysd, r0, disp, unif, 0.3)


def chain_arrays(seed: int, n_steps: int, n_walkers: int, sigma: float = 0.3):
    """Displacements N(0, sigma^2) [n_steps, Wk, 3] and uniforms [n_steps, Wk]."""
    return _chain_arrays(np.random.default_rng(seed), n_steps, n_walkers, sigma)


# Lattice-regularised DMC settings of the synthetic runs: single grid with
# hop length 0.2 bohr, and a double grid with 0.1 bohr hops within one
# Thomas-Fermi length of a nucleus and 0.4 bohr hops elsewhere; fixed-node
# gamma 0 and 0.5; projection time 0.05 Ha^-1 between branchings.
LRDMC_SINGLE = dict(a=0.2, a_valence=0.0, tf_scale=1.0, gamma=0.0)
LRDMC_DOUBLE = dict(a=0.1, a_valence=0.4, tf_scale=1.0, gamma=0.5)
LRDMC_TAU = 0.05


def lrdmc_draws(seed: int, n_steps: int, n_walkers: int):
    """Uniforms in [0, 1) [n_steps, Wk, 2] for the continuous-time LRDMC step
    (time spent in the configuration, then the hop)."""
    return np.random.default_rng(seed).random((n_steps, n_walkers, 2))


def random_positions(seed: int, sysd: System, n_walkers: int, spread=1.0):
    """Fresh walker positions for sysd drawn like the initial ones."""
    rng = np.random.default_rng(seed)
    return _initial_positions(rng, sysd.R, sysd.Z, sysd.n_up, sysd.n_dn, n_walkers, spread)


def with_walkers(w: Workload, n_walkers: int) -> Workload:
    """The first n_walkers walkers (and their chain arrays) of w."""
    return replace(
        w, r0=w.r0[:n_walkers].copy(),
        disp=None if w.disp is None else w.disp[:, :n_walkers].copy(),
        unif=None if w.unif is None else w.unif[:, :n_walkers].copy())


WORKLOADS = {
    "tiny_3nuc_10e": tiny_3nuc_10e,
    "slater_4nuc_20e": slater_4nuc_20e,
    "jas3_4nuc_20e": jas3_4nuc_20e,
    "mol_40nuc_160e": mol_40nuc_160e,
    "forces_20nuc_80e": forces_20nuc_80e,
    "large_256nuc_1024e": large_256nuc_1024e,
}
