"""CPU oracle for the Pfaffian wave function (test infrastructure only).

THIS MODULE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.

Plain FP64 statements of the Pfaffian wave function section:

  * Pf(G) of a skew-symmetric matrix (eq:Pfdef); here by the recursive
    expansion along the first row (small n, the definition) and by the
    Parlett-Reid reduction (any n): congruence transformations with unit lower
    triangular matrices (determinant 1) and row/column exchanges (each changes
    the sign) reduce G to 2x2 blocks, whose upper entries multiply to Pf(G)
  * the pairing matrix G_ij = g(i, j) with g = f_S |0,0> + f_T |1,0> +
    f_uu |1,+1> + f_dd |1,-1> (eq:g), each f expanded over the orbitals
    (agp_expansion): for electrons of spins s_i, s_j
        G_ij = phi(r_i)^T A^{s_i s_j} phi(r_j),
    A^{uu}, A^{dd} skew-symmetric (triplet +1 / -1), A^{ud} = A_S + A_T (the
    unlike-spin singlet plus triplet-zero coefficients, the spin factors
    absorbed), A^{du} = -(A^{ud})^T
  * k unpaired orbitals as k fictitious electrons (eq:pfodd and the
    paragraph after it): G~ = [[G, Phi], [-Phi^T, 0]] with
    Phi_il = phi(r_i) . U^{s_i}[:, l], N + k even
  * Psi = Pf(G~) exp(J); e_L by the same cofactor identity as for the
    determinant: the entries of G~ that depend on r_i are row i and column i,
    Pf is linear in them, and d log Pf = 1/2 tr(G~^{-1} dG~) with G~^{-1}
    skew-symmetric gives
        grad_i Pf / Pf = sum_j (grad_i G~_ij) (G~^{-1})_ji,
        lap_i  Pf / Pf = sum_j (lap_i  G~_ij) (G~^{-1})_ji.
"""
from __future__ import annotations

import math
from typing import Dict

import torch

DT = torch.float64


# ---------------------------------------------------------------------------
# Pfaffian of a skew-symmetric matrix
# ---------------------------------------------------------------------------

def pfaffian_expansion(G: torch.Tensor) -> torch.Tensor:
    """Pf(G) of one n x n skew-symmetric matrix by the expansion along the
    first row, Pf(G) = sum_{j>0} (-1)^(j+1) G_0j Pf(G without rows/cols 0, j)
    (the definition eq:Pfdef regrouped; exponential cost, small n only)."""
    n = G.shape[0]
    if n == 0:
        return torch.tensor(1.0, dtype=DT)
    if n % 2:
        return torch.tensor(0.0, dtype=DT)
    total = torch.tensor(0.0, dtype=DT)
    for j in range(1, n):
        keep = [c for c in range(1, n) if c != j]
        sub = G[keep][:, keep]
        total = total + (-1.0) ** (j + 1) * G[0, j] * pfaffian_expansion(sub)
    return total


def pfaffian_parlett_reid(G: torch.Tensor):
    """(sign, log|Pf|) of one skew-symmetric matrix by the Parlett-Reid
    reduction with partial pivoting.  For k = 0, 2, 4, ...: exchange column
    and row k+1 with the one holding the largest |A[k, j]|, j > k (a sign
    change); with a = A[k, k+1] and tau_j = A[k, j] / a (j >= k+2) the
    congruence by I - tau e_{k+1}^T clears row and column k beyond k+1 and
    leaves Pf unchanged; Pf(A) = a Pf(A[k+2:, k+2:]) after the update
        A[i, j] <- A[i, j] - tau_i A[k+1, j] + tau_j A[k+1, i]   (i, j >= k+2)."""
    A = G.clone()
    n = A.shape[0]
    if n % 2:
        return torch.tensor(0.0, dtype=DT), torch.tensor(-math.inf, dtype=DT)
    sign = 1.0
    logabs = 0.0
    for k in range(0, n - 1, 2):
        p = k + 1 + int(torch.argmax(A[k, k + 1:].abs()))
        if p != k + 1:
            A[[k + 1, p]] = A[[p, k + 1]]
            A[:, [k + 1, p]] = A[:, [p, k + 1]]
            sign = -sign
        a = A[k, k + 1].item()
        if a == 0.0:
            return torch.tensor(0.0, dtype=DT), torch.tensor(-math.inf, dtype=DT)
        sign *= 1.0 if a > 0 else -1.0
        logabs += math.log(abs(a))
        if k + 2 < n:
            tau = A[k, k + 2:] / a
            row = A[k + 1, k + 2:].clone()
            A[k + 2:, k + 2:] += -torch.outer(tau, row) + torch.outer(row, tau)
    return torch.tensor(sign, dtype=DT), torch.tensor(logabs, dtype=DT)


def pfaffian_batch(G: torch.Tensor):
    """(sign [B], log|Pf| [B]) of a batch [B, n, n]."""
    out = [pfaffian_parlett_reid(G[b]) for b in range(G.shape[0])]
    return torch.stack([o[0] for o in out]), torch.stack([o[1] for o in out])


# ---------------------------------------------------------------------------
# pairing matrix and wave function
# ---------------------------------------------------------------------------

def _blocks(sy):
    """A^{s s'} for the four spin pairs."""
    Aud = sy.lam
    return sy.pf_uu, Aud, -Aud.T, sy.pf_dd


def _pair_products(sy, left, right):
    """X[w, i, j, ...] = left_i^T A^{s_i s_j} right_j over all electron pairs,
    by spin blocks (left [Wk, N, L] or [Wk, N, L, 3], right [Wk, N, L])."""
    nu = sy.n_up
    Auu, Aud, Adu, Add = _blocks(sy)
    blocks = {(0, 0): Auu, (0, 1): Aud, (1, 0): Adu, (1, 1): Add}
    vec = left.dim() == 4
    rows = []
    for si, I in ((0, slice(0, nu)), (1, slice(nu, None))):
        cols = []
        for sj, J in ((0, slice(0, nu)), (1, slice(nu, None))):
            A = blocks[(si, sj)]
            if vec:
                cols.append(torch.einsum('wilx,lm,wjm->wijx', left[:, I], A, right[:, J]))
            else:
                cols.append(torch.einsum('wil,lm,wjm->wij', left[:, I], A, right[:, J]))
        rows.append(torch.cat(cols, dim=2))
    return torch.cat(rows, dim=1)


def unpaired_rows(sy):
    """U^{s_i} per electron: [N, L, k]."""
    N, nu = sy.n_elec, sy.n_up
    Uu = sy.unpaired
    Ud = sy.unpaired_dn if sy.unpaired_dn is not None else torch.zeros_like(Uu)
    return torch.stack([Uu if i < nu else Ud for i in range(N)])


def pairing_matrix(sy, Phi):
    """G~ [Wk, N+k, N+k] from orbital values Phi [Wk, N, L]."""
    Wk, N, _ = Phi.shape
    G = _pair_products(sy, Phi, Phi)
    G = G * (~torch.eye(N, dtype=torch.bool)).to(DT)
    U = unpaired_rows(sy)
    k = U.shape[2]
    if k == 0:
        return G
    Ph = torch.einsum('wil,ilk->wik', Phi, U)                   # [Wk, N, k]
    top = torch.cat([G, Ph], dim=2)
    bot = torch.cat([-Ph.transpose(1, 2), torch.zeros(Wk, k, k, dtype=DT)], dim=2)
    return torch.cat([top, bot], dim=1)


def log_psi(sy, r, R=None, zeta=None, lam=None, j1_b=None, j2=None):
    from oracle import jagp as O
    Phi, _, _ = O.agp_basis(sy, r, R, zeta)
    sign, logpf = pfaffian_batch(pairing_matrix(sy, Phi))
    J, _, _ = O.jastrow(sy, r, R, j1_b, j2)
    return logpf + J, sign


def evaluate(sy, r, with_intermediates=False) -> Dict[str, torch.Tensor]:
    """log|Psi|, sign, drift, E_kin, E_loc and status [Wk] (as jagp.evaluate)."""
    from oracle import jagp as O
    N = sy.n_elec
    Phi, Gp, Hp = O.agp_basis(sy, r)
    Gt = pairing_matrix(sy, Phi)
    n = Gt.shape[1]
    sign, logpf = pfaffian_batch(Gt)
    singular = sign == 0
    Gs = torch.where(singular.view(-1, 1, 1), torch.eye(n, dtype=DT).expand_as(Gt), Gt)
    Ginv = torch.linalg.inv(Gs)
    U = unpaired_rows(sy)
    # derivatives of row i of G~ with respect to r_i
    dG = _pair_products(sy, Gp, Phi)                            # [Wk, N, N, 3]
    hG = _pair_products(sy, Hp, Phi)
    off = (~torch.eye(N, dtype=torch.bool)).to(DT)
    dG = dG * off.view(1, N, N, 1)
    hG = hG * off.view(1, N, N)
    if U.shape[2]:
        dG = torch.cat([dG, torch.einsum('wilx,ilk->wikx', Gp, U)], dim=2)
        hG = torch.cat([hG, torch.einsum('wil,ilk->wik', Hp, U)], dim=2)
    GiT = Ginv[:, :, :N]                                        # (G~^-1)_{j i}, j < n, i < N
    D = torch.einsum('wijx,wji->wix', dG, GiT)
    Lp = torch.einsum('wij,wji->wi', hG, GiT)
    J, gJ, hJ = O.jastrow(sy, r)
    V = O.potential(sy, r)
    e_kin = -0.5 * (Lp + 2.0 * (D * gJ).sum(-1) + hJ + (gJ * gJ).sum(-1)).sum(-1)
    e_loc = e_kin + V
    drift = D + gJ
    logabs = logpf + J
    status = torch.zeros(r.shape[0], dtype=torch.int32)
    finite = torch.isfinite(logabs) & torch.isfinite(e_loc) & torch.isfinite(drift).all(-1).all(-1)
    status = torch.where(~finite, torch.full_like(status, 2), status)
    status = torch.where(singular, torch.full_like(status, 1), status)
    out = dict(logabs=torch.where(singular, torch.full_like(logabs, -math.inf), logabs), sign=sign,
               drift=drift, e_kin=e_kin, e_loc=e_loc, V=V, J=J, status=status)
    if with_intermediates:
        out.update(G=Gt, Ginv=Ginv, D=D, Ldet=Lp, logpf=logpf)
    return out
