"""CPU oracle for the batched JAGP wave function (test infrastructure only).

THIS MODULE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.

It is a plain, slow, FP64 evaluation of what the paper defines, batched only
over independent walkers:

  * Psi = Phi_AS * exp(J)                              (Wave functions section)
  * Phi_AS = det(G_S) with G_S[i, j] = f_S(r_i, r_j) over up electrons i and
    down electrons j (eq:wfAGPs); with k = n_up - n_dn > 0 unpaired orbitals
    the k extra columns hold phi_l(r_i) (eq:wfAGPunpaired)
  * f_S(r_i, r_j) = sum_{mu,nu} Lambda[mu, nu] psi_mu(r_i) psi_nu(r_j)
    (agp_expansion, Lambda being the coefficient matrix A of that equation)
  * psi_mu = |r - R|^l e^{-zeta |r-R|^2} x (real solid harmonic), or the Slater
    form with e^{-zeta |r-R|} (eq. gaussian / eq. slater)
  * optionally contracted orbitals phi_c = sum_mu C[mu, c] psi_mu in place of
    psi in f_S and the unpaired columns (Contraction of the primitive atomic
    basis section)
  * J = J1 + J2 with the homogeneous one-body term (onebody_J_hom), the
    bounded function u (onebody_u, plus a Pade variant) and the spin-dependent
    two-body term (twobody_jastrow, twobody_v, plus a Pade-series variant)
  * e_L = H Psi / Psi with H the all-electron Coulomb Hamiltonian in Hartree
    units (the local energy of the Variational Monte Carlo section)

Nothing here is blocked, fused or reordered beyond what the definitions say.
Library primitives used as single steps: matmul/einsum, torch.linalg.slogdet
(an LU factorisation), torch.linalg.inv, and torch.autograd for parameter
derivatives of the plain definition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, Optional

import numpy as np
import torch

DT = torch.float64


def _t(x, dtype=DT):
    return torch.as_tensor(np.asarray(x), dtype=dtype)


@dataclass
class OSystem:
    """A system held as FP64 CPU tensors (parameters may require grad)."""
    R: torch.Tensor        # [A, 3]
    Z: torch.Tensor        # [A]
    center: torch.Tensor   # [L] long
    l: torch.Tensor        # [L] long
    m: torch.Tensor        # [L] long
    zeta: torch.Tensor     # [L]
    radial: torch.Tensor   # [L] long
    lam: torch.Tensor      # [L, L]
    unpaired: torch.Tensor  # [L, k]
    n_up: int
    n_dn: int
    j1_form: int
    j1_b: torch.Tensor     # [A]
    j2_form: int
    j2: torch.Tensor       # [n_j2]
    # Jastrow basis chi and the coefficients of onebody_J_inh / threebody_jastrow
    # (LJ = 0: absent)
    jb_center: Optional[torch.Tensor] = None   # [LJ] long
    jb_l: Optional[torch.Tensor] = None
    jb_m: Optional[torch.Tensor] = None
    jb_radial: Optional[torch.Tensor] = None
    jb_zeta: Optional[torch.Tensor] = None     # [LJ]
    j1_inh: Optional[torch.Tensor] = None      # [2, LJ] up, down
    j3: Optional[torch.Tensor] = None          # [3, LJ, LJ] up-up, down-down, up-down
    # contraction of the primitive basis (Contraction of the primitive atomic
    # basis section): the geminal's orbitals are phi_c = sum_mu C[mu, c] psi_mu;
    # center .. zeta then describe the primitives and lam / unpaired the
    # contracted functions (None: lam / unpaired act on the primitives)
    contraction: Optional[torch.Tensor] = None  # [L_primitive, L]
    # Pfaffian pairing (pairing = 1): lam is A^{ud}, pf_uu / pf_dd the
    # skew-symmetric same-spin blocks, unpaired / unpaired_dn the unpaired
    # orbitals of up / down electrons (k = unpaired.shape[1], N + k even)
    pairing: int = 0
    pf_uu: Optional[torch.Tensor] = None       # [L, L]
    pf_dd: Optional[torch.Tensor] = None       # [L, L]
    unpaired_dn: Optional[torch.Tensor] = None  # [L, k]

    @property
    def n_elec(self):
        return self.n_up + self.n_dn

    @property
    def n_jbasis(self):
        return 0 if self.jb_zeta is None else int(self.jb_zeta.shape[0])


def from_workload_system(s) -> OSystem:
    """Wrap a workloads.System as tensors."""
    return OSystem(
        R=_t(s.R), Z=_t(s.Z), center=_t(s.center, torch.long), l=_t(s.l, torch.long),
        m=_t(s.m, torch.long), zeta=_t(s.zeta), radial=_t(s.radial, torch.long),
        lam=_t(s.lam), unpaired=_t(s.unpaired).reshape(len(s.lam), -1),
        n_up=int(s.n_up), n_dn=int(s.n_dn), j1_form=int(s.j1_form), j1_b=_t(s.j1_b),
        j2_form=int(s.j2_form), j2=_t(s.j2),
        **({} if getattr(s, "jb_zeta", None) is None else dict(
            jb_center=_t(s.jb_center, torch.long), jb_l=_t(s.jb_l, torch.long), jb_m=_t(s.jb_m, torch.long),
            jb_radial=_t(s.jb_radial, torch.long), jb_zeta=_t(s.jb_zeta), j1_inh=_t(s.j1_inh), j3=_t(s.j3))),
        **({} if getattr(s, "contraction", None) is None else dict(contraction=_t(s.contraction))),
        **({} if not getattr(s, "pairing", 0) else dict(
            pairing=int(s.pairing), pf_uu=_t(s.pf_uu), pf_dd=_t(s.pf_dd),
            unpaired_dn=_t(s.unpaired_dn).reshape(len(s.lam), -1))))


# ---------------------------------------------------------------------------
# atomic basis (eq. gaussian, eq. slater)
# ---------------------------------------------------------------------------

def _angular(d):
    """All nine unnormalised real solid harmonics up to l = 2 at displacement
    d [..., 3]: values [..., 9], gradients [..., 9, 3], Laplacians [..., 9].
    Order: 1 | x, y, z | xy, yz, zx, x^2-y^2, 2z^2-x^2-y^2."""
    x, y, z = d[..., 0], d[..., 1], d[..., 2]
    one, zero = torch.ones_like(x), torch.zeros_like(x)
    P = torch.stack([one, x, y, z, x * y, y * z, z * x, x * x - y * y,
                     2 * z * z - x * x - y * y], dim=-1)
    g = [
        (zero, zero, zero),
        (one, zero, zero), (zero, one, zero), (zero, zero, one),
        (y, x, zero), (zero, z, y), (z, zero, x),
        (2 * x, -2 * y, zero), (-2 * x, -2 * y, 4 * z),
    ]
    G = torch.stack([torch.stack(c, dim=-1) for c in g], dim=-2)
    # second derivatives summed: 0 for 1, x, y, z, xy, yz, zx; 2-2 for x^2-y^2;
    # -2-2+4 for 2z^2-x^2-y^2
    lapP = torch.stack([zero] * 7 + [2 * one - 2 * one, -2 * one - 2 * one + 4 * one], dim=-1)
    return P, G, lapP


def _kind(sy: OSystem):
    """Index into the nine angular factors for each basis function."""
    off = torch.tensor([0, 1, 4], dtype=torch.long)
    return off[sy.l] + sy.m


def basis(sy: OSystem, r, R=None, zeta=None):
    """psi_mu(r), grad psi_mu(r), lap psi_mu(r) for r [..., 3].

    Returns values [..., L], gradients [..., L, 3], Laplacians [..., L].
    The Laplacian is the product rule written out:
      lap(P e) = e lap P + 2 grad P . grad e + P lap e.
    """
    R = sy.R if R is None else R
    zeta = sy.zeta if zeta is None else zeta
    d = r.unsqueeze(-2) - R[sy.center]                      # [..., L, 3]
    P9, G9, H9 = _angular(d)
    k = _kind(sy)
    idx = k.expand(P9.shape[:-1])
    P = torch.gather(P9, -1, idx.unsqueeze(-1)).squeeze(-1)  # [..., L]
    gidx = idx.unsqueeze(-1).unsqueeze(-1).expand(*idx.shape, 1, 3)
    # G9 is [..., L, 9, 3]; pick the row of each function's own kind
    gP = torch.gather(G9, -2, gidx).squeeze(-2)              # [..., L, 3]
    lP = torch.gather(H9, -1, idx.unsqueeze(-1)).squeeze(-1)
    r2 = (d * d).sum(-1)
    gauss = sy.radial == 0
    # Gaussian radial factor e^{-zeta r^2}
    eg = torch.exp(-zeta * r2)
    ge_g = -2.0 * zeta.unsqueeze(-1) * d * eg.unsqueeze(-1)
    le_g = (4.0 * zeta * zeta * r2 - 6.0 * zeta) * eg
    # Slater radial factor e^{-zeta r}; its derivatives are singular at r = 0
    rr = torch.sqrt(torch.where(gauss, torch.ones_like(r2), r2))
    es = torch.exp(-zeta * rr)
    ge_s = -zeta.unsqueeze(-1) * d / rr.unsqueeze(-1) * es.unsqueeze(-1)
    le_s = (zeta * zeta - 2.0 * zeta / rr) * es
    e = torch.where(gauss, eg, es)
    ge = torch.where(gauss.unsqueeze(-1), ge_g, ge_s)
    le = torch.where(gauss, le_g, le_s)
    psi = P * e
    grad = gP * e.unsqueeze(-1) + P.unsqueeze(-1) * ge
    lap = lP * e + 2.0 * (gP * ge).sum(-1) + P * le
    return psi, grad, lap


def agp_basis(sy: OSystem, r, R=None, zeta=None):
    """The orbitals the geminal is built from: the primitive basis, or its
    contraction phi_c = sum_mu C[mu, c] psi_mu (values, gradients and
    Laplacians are linear in psi, so each is contracted the same way)."""
    psi, grad, lap = basis(sy, r, R, zeta)
    C = sy.contraction
    if C is None:
        return psi, grad, lap
    return psi @ C, torch.einsum('...mx,mc->...cx', grad, C), lap @ C


# ---------------------------------------------------------------------------
# Jastrow factor (onebody_J_hom, onebody_u, twobody_jastrow, twobody_v)
# ---------------------------------------------------------------------------

def _u_and_derivs(form, s, b):
    """One-body bounded function u(s) and its first two derivatives in s.
    form 1: u = (1 - e^{-b s}) / (2 b)          (onebody_u)
    form 2: u = s / (2 (1 + b s))               (Pade variant, same cusp)"""
    if form == 1:
        e = torch.exp(-b * s)
        return -torch.expm1(-b * s) / (2.0 * b), 0.5 * e, -0.5 * b * e
    if form == 2:
        q = 1.0 + b * s
        return s / (2.0 * q), 0.5 / (q * q), -b / (q * q * q)
    raise ValueError(form)


def _v_and_derivs(form, params, r, same_spin):
    """Two-body function v(r) for each pair and its first two derivatives.
    form 1 (twobody_v): v = c r / (1 + b r), c = 1/4 (parallel) or 1/2
    (antiparallel), b = b_para or b_anti.
    form 2: v = c t + sum_{k=1..3} a_k t^{k+1}, t = r / (1 + b r), with one
    (b, a1, a2, a3) set per spin relation."""
    c = torch.where(same_spin, torch.full_like(r, 0.25), torch.full_like(r, 0.5))
    if form == 1:
        b = torch.where(same_spin, params[0], params[1])
        a = [torch.zeros_like(r)] * 3
    elif form == 2:
        b = torch.where(same_spin, params[0], params[4])
        a = [torch.where(same_spin, params[1 + k], params[5 + k]) for k in range(3)]
    else:
        raise ValueError(form)
    q = 1.0 + b * r
    t = r / q
    t1 = 1.0 / (q * q)
    t2 = -2.0 * b / (q * q * q)
    v = c * t
    dv_dt = c.clone()
    d2v_dt2 = torch.zeros_like(r)
    for k in range(3):
        v = v + a[k] * t ** (k + 2)
        dv_dt = dv_dt + (k + 2) * a[k] * t ** (k + 1)
        d2v_dt2 = d2v_dt2 + (k + 2) * (k + 1) * a[k] * t ** k
    v1 = dv_dt * t1
    v2 = d2v_dt2 * t1 * t1 + dv_dt * t2
    return v, v1, v2


def jastrow(sy: OSystem, r, R=None, j1_b=None, j2=None):
    """J [Wk], grad_i J [Wk, N, 3], lap_i J [Wk, N] for positions r [Wk, N, 3].

    For a radial term f(|x|): grad f = f'(r) x / r and lap f = f'' + 2 f' / r.
    """
    R = sy.R if R is None else R
    j1_b = sy.j1_b if j1_b is None else j1_b
    j2 = sy.j2 if j2 is None else j2
    Wk, N, _ = r.shape
    J = torch.zeros(Wk, dtype=DT)
    g = torch.zeros(Wk, N, 3, dtype=DT)
    h = torch.zeros(Wk, N, dtype=DT)
    if sy.j1_form:
        d = r.unsqueeze(2) - R.unsqueeze(0).unsqueeze(0)    # [Wk, N, A, 3]
        ria = torch.sqrt((d * d).sum(-1))
        twoZ = 2.0 * sy.Z
        s = twoZ ** 0.25 * ria
        u, u1, u2 = _u_and_derivs(sy.j1_form, s, j1_b)
        f = -(twoZ ** 0.75) * u
        f1 = -(twoZ ** 0.75) * (twoZ ** 0.25) * u1
        f2 = -(twoZ ** 0.75) * (twoZ ** 0.5) * u2
        J = J + f.sum(dim=(1, 2))
        g = g + (f1 / ria).unsqueeze(-1).mul(d).sum(2)
        h = h + (f2 + 2.0 * f1 / ria).sum(2)
    if sy.n_jbasis:
        Jx, gx, hx = _jastrow_basis_terms(sy, r, R)
        J, g, h = J + Jx, g + gx, h + hx
    if sy.j2_form and N > 1:
        d = r.unsqueeze(2) - r.unsqueeze(1)                   # [Wk, N, N, 3]
        eye = torch.eye(N, dtype=torch.bool)
        rij = torch.sqrt((d * d).sum(-1) + eye.to(DT))          # 1 on the diagonal
        spin = torch.arange(N) < sy.n_up
        same = (spin.unsqueeze(0) == spin.unsqueeze(1)).expand(Wk, N, N)
        v, v1, v2 = _v_and_derivs(sy.j2_form, j2, rij, same)
        off = (~eye).to(DT)
        J = J + 0.5 * (v * off).sum(dim=(1, 2))
        g = g + ((v1 / rij) * off).unsqueeze(-1).mul(d).sum(2)
        h = h + ((v2 + 2.0 * v1 / rij) * off).sum(2)
    return J, g, h


class _JBasisView:
    """The Jastrow basis dressed as a system for basis()."""
    def __init__(self, sy: OSystem, R):
        self.R, self.center, self.l, self.m = R, sy.jb_center, sy.jb_l, sy.jb_m
        self.zeta, self.radial = sy.jb_zeta, sy.jb_radial


def _jastrow_basis_terms(sy: OSystem, r, R=None):
    """J1 inhomogeneous and J3/4 (onebody_J_inh, threebody_jastrow) with
    per-electron gradients and Laplacians.

      J1inh = sum_i m_{s_i} . chi(r_i)
      J3/4  = sum_{i<j} chi(r_i)^T M^{s_i s_j} chi(r_j)
    Up electrons come first, so a pair i < j of unlike spins is (up, down) and
    uses M^{ud}; same-spin matrices are symmetric (the pair term must not
    depend on the order of two same-spin electrons), M^{du} = (M^{ud})^T.
    The pair sum is written out over all pairs; electron i's term is linear
    in chi(r_i), so grad_i and lap_i act on chi(r_i) alone.
    """
    R = sy.R if R is None else R
    chi, gchi, lchi = basis(_JBasisView(sy, R), r)          # [Wk, N, LJ], [.., 3], [..]
    Wk, N, LJ = chi.shape
    nu = sy.n_up
    up = torch.arange(N) < nu
    m = torch.where(up.view(1, N, 1), sy.j1_inh[0].view(1, 1, LJ), sy.j1_inh[1].view(1, 1, LJ))
    J = (m * chi).sum(dim=(1, 2))
    g = torch.einsum('wikx,wik->wix', gchi, m.expand(Wk, N, LJ))
    h = (lchi * m).sum(-1)
    # Mt[i, j]: the matrix that multiplies chi(r_j) in electron i's pair term
    Muu, Mdd, Mud = sy.j3[0], sy.j3[1], sy.j3[2]
    Mt = torch.empty(N, N, LJ, LJ, dtype=DT)
    for i in range(N):
        for j in range(N):
            if up[i] and up[j]:
                Mt[i, j] = Muu
            elif not up[i] and not up[j]:
                Mt[i, j] = Mdd
            elif up[i]:
                Mt[i, j] = Mud
            else:
                Mt[i, j] = Mud.T
    B = torch.einsum('ijkl,wjl->wijk', Mt, chi)               # [Wk, i, j, LJ]: Mt[i,j] chi_j
    off = (~torch.eye(N, dtype=torch.bool)).to(DT).view(1, N, N, 1)
    K = (B * off).sum(2)                                      # [Wk, N, LJ]
    iu = torch.triu_indices(N, N, 1)
    J = J + (chi[:, iu[0]] * B[:, iu[0], iu[1]]).sum(dim=(1, 2))
    g = g + torch.einsum('wikx,wik->wix', gchi, K)
    h = h + (lchi * K).sum(-1)
    return J, g, h


def potential(sy: OSystem, r, R=None):
    """All-electron Coulomb energy: e-e repulsion, e-n attraction, n-n repulsion."""
    R = sy.R if R is None else R
    Wk, N, _ = r.shape
    iu = torch.triu_indices(N, N, 1)
    dee = r[:, iu[0]] - r[:, iu[1]]
    rij = torch.sqrt((dee * dee).sum(-1))
    V = (1.0 / rij).sum(-1)
    den = r.unsqueeze(2) - R.unsqueeze(0).unsqueeze(0)
    ria = torch.sqrt((den * den).sum(-1))
    V = V - (sy.Z / ria).sum(dim=(1, 2))
    A = R.shape[0]
    if A > 1:
        ia = torch.triu_indices(A, A, 1)
        dnn = R[ia[0]] - R[ia[1]]
        Rab = torch.sqrt((dnn * dnn).sum(-1))
        V = V + (sy.Z[ia[0]] * sy.Z[ia[1]] / Rab).sum()
    return V


# ---------------------------------------------------------------------------
# geminal matrix and determinant (agp_expansion, eq:wfAGPs, eq:wfAGPunpaired)
# ---------------------------------------------------------------------------

def geminal(sy: OSystem, Phi, lam=None):
    """G~ = [ Phi_up Lambda Phi_dn^T | Phi_up U ]  ->  [Wk, n_up, n_up]."""
    lam = sy.lam if lam is None else lam
    pu, pd = Phi[:, :sy.n_up], Phi[:, sy.n_up:]
    W = pu @ lam @ pd.transpose(1, 2)
    if sy.unpaired.shape[1]:
        W = torch.cat([W, pu @ sy.unpaired], dim=2)
    return W


def log_psi(sy: OSystem, r, R=None, zeta=None, lam=None, j1_b=None, j2=None):
    """log|Psi| [Wk] and sign(Psi) [Wk] (sign of the determinant)."""
    if sy.pairing:
        from oracle import pfaffian
        return pfaffian.log_psi(sy, r, R, zeta, lam, j1_b, j2)
    Phi, _, _ = agp_basis(sy, r, R, zeta)
    W = geminal(sy, Phi, lam)
    sign, logdet = torch.linalg.slogdet(W)
    J, _, _ = jastrow(sy, r, R, j1_b, j2)
    return logdet + J, sign


def evaluate(sy: OSystem, r, R=None, zeta=None, lam=None, j1_b=None, j2=None,
             with_intermediates=False) -> Dict[str, torch.Tensor]:
    """Full evaluation for walkers r [Wk, N, 3].

    Determinant derivatives follow from the cofactor expansion: the entries of
    G~ that depend on electron i form one row (up) or one column (down), so
      grad_i det / det = sum_j (d G~_ij / d r_i) (G~^{-1})_ji
      lap_i det / det  = sum_j (lap_i G~_ij)     (G~^{-1})_ji
    and lap Psi / Psi = lap det/det + 2 grad det/det . grad J + lap J + |grad J|^2.
    status: 0 ok, 1 singular (det = 0), 2 non-finite result.
    """
    if sy.pairing:
        from oracle import pfaffian
        return pfaffian.evaluate(sy, r, with_intermediates)
    lam = sy.lam if lam is None else lam
    nu, nd = sy.n_up, sy.n_dn
    Phi, G, H = agp_basis(sy, r, R, zeta)
    W = geminal(sy, Phi, lam)
    sign, logdet = torch.linalg.slogdet(W)
    singular = sign == 0
    Wsafe = torch.where(singular.view(-1, 1, 1), torch.eye(nu, dtype=DT).expand_as(W), W)
    A = torch.linalg.inv(Wsafe)                               # [Wk, nu(cols of G~), nu]
    pu, pd = Phi[:, :nu], Phi[:, nu:]
    gu, gd = G[:, :nu], G[:, nu:]
    hu, hd = H[:, :nu], H[:, nu:]
    # rows of G~ differentiated by their up electron
    grow = torch.einsum('wimx,mn,wjn->wijx', gu, lam, pd)
    hrow = torch.einsum('wim,mn,wjn->wij', hu, lam, pd)
    if sy.unpaired.shape[1]:
        grow = torch.cat([grow, torch.einsum('wimx,mk->wikx', gu, sy.unpaired)], dim=2)
        hrow = torch.cat([hrow, hu @ sy.unpaired], dim=2)
    Dup = torch.einsum('wijx,wji->wix', grow, A)
    Lup = torch.einsum('wij,wji->wi', hrow, A)
    # columns of G~ differentiated by their down electron
    gcol = torch.einsum('wim,mn,wjnx->wijx', pu, lam, gd)
    hcol = torch.einsum('wim,mn,wjn->wij', pu, lam, hd)
    Ddn = torch.einsum('wijx,wji->wjx', gcol, A[:, :nd])
    Ldn = torch.einsum('wij,wji->wj', hcol, A[:, :nd])
    D = torch.cat([Dup, Ddn], dim=1)
    Lp = torch.cat([Lup, Ldn], dim=1)
    J, gJ, hJ = jastrow(sy, r, R, None if j1_b is None else j1_b, j2)
    V = potential(sy, r, R)
    e_kin = -0.5 * (Lp + 2.0 * (D * gJ).sum(-1) + hJ + (gJ * gJ).sum(-1)).sum(-1)
    e_loc = e_kin + V
    drift = D + gJ
    logabs = logdet + J
    status = torch.zeros(r.shape[0], dtype=torch.int32)
    finite = torch.isfinite(logabs) & torch.isfinite(e_loc) & torch.isfinite(drift).all(-1).all(-1)
    status = torch.where(~finite, torch.full_like(status, 2), status)
    status = torch.where(singular, torch.full_like(status, 1), status)
    out = dict(logabs=torch.where(singular, torch.full_like(logabs, -math.inf), logabs),
               sign=sign, drift=drift, e_kin=e_kin, e_loc=e_loc, V=V, J=J,
               status=status)
    if with_intermediates:
        out.update(Phi=Phi, gradPhi=G, lapPhi=H, W=W, A=A, D=D, Ldet=Lp,
                   gradJ=gJ, lapJ=hJ, logdet=logdet)
    return out


# ---------------------------------------------------------------------------
# single-electron moves: the ratio Psi(x')/Psi(x) by its definition
# ---------------------------------------------------------------------------

def move_ratio(sy: OSystem, r, e, r_new):
    """Psi(x')/Psi(x) [Wk] where x' moves electron e of each walker to r_new [Wk, 3].
    Both wave functions are evaluated from scratch."""
    la, sa = log_psi(sy, r)
    r2 = r.clone()
    r2[:, e] = r_new
    lb, sb = log_psi(sy, r2)
    return sa * sb * torch.exp(lb - la)


def run_chain(sy: OSystem, r0, disp, unif, e_start=0, n_steps=None):
    """Metropolis chain with single-electron moves (VMC section).

    Step t moves electron (e_start + t) mod N of every walker by disp[t] and
    accepts iff unif[t] < ratio^2 (strict).  The ratio is the definition
    Psi(x')/Psi(x) from full re-evaluation.
    Returns final positions, per-step ratios [n_steps, Wk], accept flags.
    """
    r = r0.clone()
    N = sy.n_elec
    n_steps = disp.shape[0] if n_steps is None else n_steps
    la, sa = log_psi(sy, r)
    ratios, accs = [], []
    for t in range(n_steps):
        e = (e_start + t) % N
        r2 = r.clone()
        r2[:, e] = r[:, e] + disp[t]
        lb, sb = log_psi(sy, r2)
        ratio = sa * sb * torch.exp(lb - la)
        acc = unif[t] < ratio * ratio
        r = torch.where(acc.view(-1, 1, 1), r2, r)
        la = torch.where(acc, lb, la)
        sa = torch.where(acc, sb, sa)
        ratios.append(ratio)
        accs.append(acc)
    return r, torch.stack(ratios), torch.stack(accs)


# ---------------------------------------------------------------------------
# derivatives (Derivatives of energy section): O_k = d ln Psi / d alpha_k and
# d e_L / d alpha_k, here by reverse-mode autodiff of the plain definition.
# ---------------------------------------------------------------------------

GRAD_KEYS = ("R", "zeta", "lam", "jas", "r")


def _params(sy: OSystem, r):
    R = sy.R.detach().clone().requires_grad_(True)
    zeta = sy.zeta.detach().clone().requires_grad_(True)
    lam = sy.lam.detach().clone().requires_grad_(True)
    jas = torch.cat([sy.j1_b, sy.j2]).detach().clone().requires_grad_(True)
    rr = r.detach().clone().requires_grad_(True)
    return dict(R=R, zeta=zeta, lam=lam, jas=jas, r=rr)


def _eval_params(sy: OSystem, p):
    A = sy.R.shape[0]
    return evaluate(sy, p["r"], R=p["R"], zeta=p["zeta"], lam=p["lam"],
                    j1_b=p["jas"][:A], j2=p["jas"][A:])


def forces_vjp(sy: OSystem, r, gbar_logpsi, gbar_eloc):
    """Gradients of sum_w (gbar_logpsi[w] log|Psi_w| + gbar_eloc[w] e_L,w)
    with respect to R [A,3], zeta [L], Lambda [L,L] (unconstrained entries),
    the Jastrow vector [A + n_j2] and r [Wk,N,3]."""
    p = _params(sy, r)
    out = _eval_params(sy, p)
    F = (gbar_logpsi * out["logabs"]).sum() + (gbar_eloc * out["e_loc"]).sum()
    g = torch.autograd.grad(F, [p[k] for k in GRAD_KEYS], allow_unused=True)
    return {k: (torch.zeros_like(p[k]) if gi is None else gi) for k, gi in zip(GRAD_KEYS, g)}


def forces_per_walker(sy: OSystem, r):
    """Per-walker gradients of log|Psi| and of e_L (the walker's own r only).
    Returns dict name -> (d logpsi [Wk, ...], d e_loc [Wk, ...])."""
    Wk = r.shape[0]
    res = {k: ([], []) for k in GRAD_KEYS}
    for w in range(Wk):
        sub = r[w:w + 1]
        for which in (0, 1):
            gl = torch.tensor([1.0 if which == 0 else 0.0], dtype=DT)
            ge = torch.tensor([1.0 if which == 1 else 0.0], dtype=DT)
            g = forces_vjp(sy, sub, gl, ge)
            for k in GRAD_KEYS:
                res[k][which].append(g[k][0] if k == "r" else g[k])
    return {k: (torch.stack(v[0]), torch.stack(v[1])) for k, v in res.items()}
