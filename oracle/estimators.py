"""CPU oracle for the force and optimisation estimators (test infrastructure
only).

THIS MODULE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.

Plain FP64 definitions from the Atomic forces and Stochastic reconfiguration
sections of the paper:

  * space warp: omega_a(r) = kappa(|r - R_a|) / sum_b kappa(|r - R_b|),
    kappa(r) = 1/r^4; total derivatives per walker
      d e_L/dR_a          = de_L/dR_a + sum_i omega_a(r_i) de_L/dr_i
      d ln(J^1/2 Psi)/dR_a = dlnPsi/dR_a + sum_i [omega_a(r_i) dlnPsi/dr_i
                                                  + 1/2 grad omega_a(r_i)]
  * finite-variance reweighting: R = (S sum_ij |G^-1_ij|^2)^(-theta),
    S = min_i sum_j |G_ij|^2 (G the geminal matrix W, or the Pfaffian's
    pairing matrix), R^eps = max(R, eps),
    weight = (R / R^eps)^2
  * stochastic reconfiguration: S_kl = <(O_k - Obar_k)(O_l - Obar_l)>,
    f_k = -2 <e_L (O_k - Obar_k)>, diagonal s_kk (1 + eps), step S'^-1 f
    (averages optionally weighted, sum w x / sum w).
"""
from __future__ import annotations

import torch

from oracle import jagp as O

DT = torch.float64


def warp_weights(sy: O.OSystem, r, R=None):
    """omega [Wk, N, A] and grad_r omega [Wk, N, A, 3] with kappa = 1/r^4."""
    R = sy.R if R is None else R
    d = r.unsqueeze(2) - R.view(1, 1, -1, 3)                 # [Wk, N, A, 3]
    r2 = (d * d).sum(-1)
    kap = 1.0 / (r2 * r2)
    gkap = -4.0 * d / (r2 * r2 * r2).unsqueeze(-1)           # grad of (r^2)^-2
    K = kap.sum(-1, keepdim=True)
    gK = gkap.sum(2, keepdim=True)
    om = kap / K
    gom = gkap / K.unsqueeze(-1) - kap.unsqueeze(-1) * gK / (K * K).unsqueeze(-1)
    return om, gom


def swct_total(sy: O.OSystem, r, dR, dr, jacobian=False):
    """Total derivatives [Wk, A, 3] from the partials dR [Wk, A, 3] and
    dr [Wk, N, 3]; jacobian adds 1/2 sum_i grad omega_a(r_i)."""
    om, gom = warp_weights(sy, r)
    out = dR + torch.einsum('wia,wix->wax', om, dr)
    if jacobian:
        out = out + 0.5 * gom.sum(1)
    return out


def reweight(sy: O.OSystem, r, theta, eps):
    """R [Wk] and weight [Wk] from the geminal matrix of the configuration."""
    Phi, _, _ = O.agp_basis(sy, r)
    if sy.pairing:
        # the pairing matrix of the Pfaffian, fictitious rows included
        from oracle import pfaffian as PF
        W = PF.pairing_matrix(sy, Phi)
    else:
        W = O.geminal(sy, Phi)
    A = torch.linalg.inv(W)
    S = (W * W).sum(-1).min(-1).values
    R = (S * (A * A).sum(dim=(1, 2))) ** (-theta)
    Reps = torch.clamp(R, min=eps)
    return R, (R / Reps) ** 2


def sr_step(Ok, e_loc, eps, weights=None):
    """Stochastic-reconfiguration step: delta [P], force f [P], S [P, P].
    Ok [M, P] logarithmic derivatives, e_loc [M]."""
    M = Ok.shape[0]
    w = torch.ones(M, dtype=DT) if weights is None else weights
    wn = w / w.sum()
    Obar = (wn.unsqueeze(1) * Ok).sum(0)
    Dc = Ok - Obar
    S = (wn.view(M, 1, 1) * Dc.unsqueeze(2) * Dc.unsqueeze(1)).sum(0)
    f = -2.0 * (wn.unsqueeze(1) * e_loc.unsqueeze(1) * Dc).sum(0)
    Sp = S + eps * torch.diag(torch.diagonal(S))
    delta = torch.linalg.solve(Sp, f)
    return delta, f, S
