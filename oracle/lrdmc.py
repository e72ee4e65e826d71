"""CPU oracle for the lattice-regularised diffusion Monte Carlo step (test
infrastructure only).

THIS MODULE IS TEST INFRASTRUCTURE.  Only the tests, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.

It follows the Lattice regularized Monte Carlo section of the paper, for the
guiding function Psi_G = Psi (the JAGP of oracle.jagp):

  * the kinetic term is the finite-difference Laplacian with hop length a:
    Delta^a_i f = (1/a^2) sum_{k in x,y,z} [f(r_i + a e_k) + f(r_i - a e_k) - 2 f],
    so H^a = -1/2 sum_i Delta^a_i + V^a connects x with the 6N configurations
    x' in which one electron has hopped by +-a along one axis, with the
    off-diagonal element -1/(2 a^2)                        (the (6N+1) candidates)
  * V^a = V + 1/2 sum_i (Delta^a_i - Delta_i) Psi_G / Psi_G   (lrdmc_potential)
  * the fixed-node Hamiltonian H^{FN,gamma} with s_{x',x} = Psi_G(x') H_{x',x} / Psi_G(x)
    and the spin-flip term V_sf = sum_{x': s > 0} H_{x',x} Psi_G(x') / Psi_G(x):
    diagonal H_xx + (1 + gamma) V_sf, off-diagonal H_{x',x} where s < 0 and
    -gamma H_{x',x} where s > 0
  * the importance-sampled Green's function G~_{x',x} = (lambda - H^FN)_{x',x}
    Psi_G(x') / Psi_G(x) (is-green-function) and its column sum b~_x
    (lrdmc_mod_weight); the local energy e~_L = sum_{x'} H_{x',x} Psi_G(x')/Psi_G(x)
    (lrdmc_mod_local_energy)
  * the continuous-time treatment of diagonal moves: the walker stays for
    tau_xi = -log(1 - xi) / b_x, b_x here being the rate of leaving x (the sum
    of the off-diagonal G~ elements, to which the per-step probability of a
    non-diagonal move tends times lambda as lambda grows), its weight is
    multiplied by exp(-tau_xi e_L), and the hop x -> x' is drawn with
    probability G~_{x',x} / b_x, until the projection time tau is used up.
  * double grid: hop length a near nuclei and a' in the valence region, the
    boundary set by the Thomas-Fermi length 0.8853 Z^{-1/3} bohr (a reading:
    the paper names the ingredients, not the switching rule).

Every ratio Psi(x')/Psi(x) is the definition: two evaluations from scratch.
Hop order (used by the hop index and the selection): electron-major, then
+x, -x, +y, -y, +z, -z.
"""
from __future__ import annotations

import math
from typing import Dict

import torch

from oracle import jagp as O

DT = torch.float64
TF_COEF = 0.8853          # Thomas-Fermi screening length 0.8853 Z^{-1/3} (bohr)
# (sign, axis) of the six hops of one electron
DIRS = ((1.0, 0), (-1.0, 0), (1.0, 1), (-1.0, 1), (1.0, 2), (-1.0, 2))


def mesh(sy: O.OSystem, r, a, a_valence=0.0, tf_scale=1.0):
    """Hop length of every electron [Wk, N].  Single grid (a_valence <= 0): a.
    Double grid: a for an electron closer than tf_scale Thomas-Fermi lengths to
    some nucleus, a_valence otherwise."""
    Wk, N, _ = r.shape
    if a_valence <= 0.0:
        return torch.full((Wk, N), float(a), dtype=DT)
    d = r.unsqueeze(2) - sy.R.view(1, 1, -1, 3)
    dist = torch.sqrt((d * d).sum(-1))                       # [Wk, N, A]
    tf = TF_COEF * sy.Z.pow(-1.0 / 3.0)                      # [A]
    near = (dist < tf_scale * tf).any(-1)
    return torch.where(near, torch.full_like(dist[..., 0], float(a)),
                       torch.full_like(dist[..., 0], float(a_valence)))


def hop_configs(r, a_i):
    """The 6N hopped configurations [Wk, N, 6, N, 3]: copy k of electron i has
    electron i moved by sign * a_i along axis."""
    Wk, N, _ = r.shape
    out = r.view(Wk, 1, 1, N, 3).repeat(1, N, 6, 1, 1)
    for i in range(N):
        for k, (sg, ax) in enumerate(DIRS):
            out[:, i, k, i, ax] = r[:, i, ax] + sg * a_i[:, i]
    return out


def lattice_ratios(sy: O.OSystem, r, a_i, chunk=64):
    """Psi(x')/Psi(x) [Wk, N, 6] for every lattice hop, by full re-evaluation."""
    Wk, N, _ = r.shape
    la, sa = O.log_psi(sy, r)
    xs = hop_configs(r, a_i).reshape(Wk * N * 6, N, 3)
    lb, sb = [], []
    for s in range(0, xs.shape[0], chunk):
        l_, s_ = O.log_psi(sy, xs[s:s + chunk])
        lb.append(l_)
        sb.append(s_)
    lb = torch.cat(lb).view(Wk, N, 6)
    sb = torch.cat(sb).view(Wk, N, 6)
    return sa.view(Wk, 1, 1) * sb * torch.exp(lb - la.view(Wk, 1, 1))


def green_column(sy: O.OSystem, r, a_i, gamma, ratios=None, ev=None) -> Dict[str, torch.Tensor]:
    """The column x of the lattice Hamiltonians and of the fixed-node
    importance-sampled Green's function (without lambda), per walker.

    Returns
      ratios   [Wk, N, 6]  Psi(x')/Psi(x)
      H_off    [Wk, N, 6]  H^a_{x',x} = -1/(2 a_i^2)
      lap_a    [Wk]        sum_i Delta^a_i Psi / Psi
      V, e_kin, e_loc [Wk] from the continuous evaluation
      V_a      [Wk]        V^a (lrdmc_potential)
      H_diag   [Wk]        H^a_{x,x} = 3 sum_i 1/a_i^2 + V^a
      V_sf     [Wk]        spin-flip term
      HFN_off  [Wk, N, 6]  off-diagonal H^{FN,gamma}
      HFN_diag [Wk]        H_xx + (1 + gamma) V_sf
      G_off    [Wk, N, 6]  off-diagonal G~^{FN} = -HFN_off * ratio
      escape   [Wk]        sum of G_off (rate of leaving x)
      e_L_fn   [Wk]        sum_{x'} H^{FN}_{x',x} Psi(x')/Psi(x), x' = x included
    """
    if ev is None:
        ev = O.evaluate(sy, r)
    if ratios is None:
        ratios = lattice_ratios(sy, r, a_i)
    inv_a2 = 1.0 / (a_i * a_i)                                  # [Wk, N]
    H_off = (-0.5 * inv_a2).unsqueeze(-1).expand_as(ratios)
    # Delta^a_i Psi / Psi = (1/a^2) sum_k (Psi(x'_k)/Psi(x) - 1)   (the -2f of
    # each axis shared between its two hops)
    lap_a = (inv_a2.unsqueeze(-1) * (ratios - 1.0)).sum(dim=(1, 2))
    lap_cont = -2.0 * ev["e_kin"]                               # sum_i Delta_i Psi / Psi
    V = ev["V"]
    V_a = V + 0.5 * (lap_a - lap_cont)
    H_diag = 3.0 * inv_a2.sum(-1) + V_a
    s = ratios * H_off                                          # s_{x',x}
    pos = s > 0
    V_sf = torch.where(pos, H_off * ratios, torch.zeros_like(s)).sum(dim=(1, 2))
    HFN_off = torch.where(pos, -gamma * H_off, H_off)
    HFN_diag = H_diag + (1.0 + gamma) * V_sf
    G_off = -HFN_off * ratios
    escape = G_off.sum(dim=(1, 2))
    e_L_fn = HFN_diag + (HFN_off * ratios).sum(dim=(1, 2))
    return dict(ratios=ratios, H_off=H_off, lap_a=lap_a, V=V, e_kin=ev["e_kin"],
                e_loc=ev["e_loc"], V_a=V_a, H_diag=H_diag, V_sf=V_sf, HFN_off=HFN_off,
                HFN_diag=HFN_diag, G_off=G_off, escape=escape, e_L_fn=e_L_fn)


def discrete_column(col, lam):
    """Discrete-time G~^{FN} column for a given lambda: diagonal lambda - H^FN_xx,
    off-diagonal G_off, and its sum b~_x (lrdmc_mod_weight)."""
    diag = lam - col["HFN_diag"]
    b = diag + col["G_off"].sum(dim=(1, 2))
    return diag, b


def advance(r, a_i, col, xi, weight, tau_left, singular=None):
    """One continuous-time step of every walker.

    xi [Wk, 2]: xi[:, 0] draws the time spent in x, xi[:, 1] the hop.
    A walker with tau_left <= 0 (or a singular guiding function) is left as it
    is (hop -1).  Otherwise tau_xi = -log(1 - xi0) / escape; if tau_xi >= tau_left
    the walker stays, its weight is multiplied by exp(-tau_left e_L) and
    tau_left becomes 0 (hop -1); else the weight is multiplied by
    exp(-tau_xi e_L), tau_left decreases by tau_xi and the hop is the first k
    (in hop order) whose cumulative G_off exceeds xi1 * escape.
    Returns new positions, weight, tau_left and hop index 6 i + k (-1: none).
    """
    Wk, N, _ = r.shape
    r_next = r.clone()
    w_next = weight.clone()
    t_next = tau_left.clone()
    hop = torch.full((Wk,), -1, dtype=torch.int64)
    e_L = col["e_loc"]
    for w in range(Wk):
        if tau_left[w] <= 0.0 or (singular is not None and bool(singular[w])):
            continue
        b = col["escape"][w]
        tau_xi = -math.log1p(-float(xi[w, 0])) / float(b) if b > 0 else math.inf
        if tau_xi >= float(tau_left[w]):
            w_next[w] = weight[w] * math.exp(-float(tau_left[w]) * float(e_L[w]))
            t_next[w] = 0.0
            continue
        w_next[w] = weight[w] * math.exp(-tau_xi * float(e_L[w]))
        t_next[w] = tau_left[w] - tau_xi
        g = col["G_off"][w].reshape(-1)
        cum = torch.cumsum(g, 0)
        target = float(xi[w, 1]) * float(b)
        k = int(torch.searchsorted(cum, torch.tensor([target], dtype=DT), right=True)[0])
        if k >= g.numel():               # rounding at the top end: the last possible hop
            k = int(torch.nonzero(g > 0)[-1])
        i, d = divmod(k, 6)
        sg, ax = DIRS[d]
        r_next[w, i, ax] = r[w, i, ax] + sg * a_i[w, i]
        hop[w] = k
    return r_next, w_next, t_next, hop
