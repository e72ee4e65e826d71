// Lattice-regularised diffusion Monte Carlo step on the JAGP guiding function
// (Lattice regularized Monte Carlo section).
//
// The lattice kinetic term connects a configuration x with the 6N
// configurations x' in which one electron i has hopped by +-a_i along x, y or z
// (the (6N+1)-candidate column of the lattice Hamiltonian).  The ratios
// Psi(x')/Psi(x) need no inverse update: moving electron i changes one row
// (up) or column (down) of W, so the determinant ratio is psi(r')^T Yt[i] with
// the cofactor row Yt[i] that the evaluation already holds for the local
// energy (Yt_up = W^{-T} P_dn, Yt_dn = W^{-1} P_up), times exp of the Jastrow
// change.  From those ratios:
//   lap_a   = sum_i Delta^{a_i}_i Psi / Psi = sum_{i,k} (ratio_ik - 1) / a_i^2
//   V^a - V = (lap_a - sum_i Delta_i Psi / Psi) / 2 = (lap_a + 2 E_kin) / 2   (lrdmc_potential)
//   V_sf    = sum over hops with ratio < 0 of |ratio| / (2 a_i^2)              (spin-flip term)
//   G~FN    = ratio / (2 a_i^2) for ratio > 0, gamma |ratio| / (2 a_i^2) else  (fixed node, is-green-function)
//   escape  = sum of the off-diagonal G~FN (rate of leaving x)
//   H^FN_xx = 3 sum_i 1/a_i^2 + V^a + (1 + gamma) V_sf
// and the fixed-node local energy equals the continuous e_L for every gamma.
// The continuous-time step draws the time spent in x, tau_xi = -log(1-xi)/escape,
// multiplies the weight by exp(-tau_xi e_L) and hops with probability
// G~FN_{x',x} / escape, until the projection time left is used up.
#include "lrdmc.h"

namespace qmc {

// Hop length of an electron at (x, y, z): a within tf_scale Thomas-Fermi
// lengths of some nucleus, a_val elsewhere (double grid); a everywhere when
// a_val <= 0.  Every lane of the wave takes part.
__device__ __forceinline__ double hop_length(const SysDev& s, const LrdmcParams& p, double x, double y,
                                             double z) {
  if (!(p.a_val > 0.0)) return p.a;
  int near = 0;
  for (int n = threadIdx.x & 63; n < s.n_nuc; n += 64) {
    const double dx = x - s.R[3 * n], dy = y - s.R[3 * n + 1], dz = z - s.R[3 * n + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    near |= d < p.tf_scale * (kTfCoef * pow(s.Z[n], -1.0 / 3.0)) ? 1 : 0;
  }
  return __any(near) ? p.a : p.a_val;
}

// Coordinate `ax` of hop k (k = 2 ax + (0: +a, 1: -a)) added to (x, y, z).
template <int K>
__device__ __forceinline__ void hop_point(double x, double y, double z, double a, double& px, double& py,
                                          double& pz) {
  constexpr int ax = K >> 1;
  const double d = (K & 1) ? -a : a;
  px = ax == 0 ? x + d : x;
  py = ax == 1 ? y + d : y;
  pz = ax == 2 ? z + d : z;
}

// One wave per (walker, electron): the six hop ratios of electron i.
__global__ __launch_bounds__(256) void lrdmc_ratio_kernel(SysDev s, WalkDev w, LrdmcDev l, LrdmcParams p) {
  const int wk = blockIdx.x, lane = threadIdx.x & 63;
  const int i = blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= s.N) return;                       // whole waves only; no block barrier below
  const double* r = w.r + (long)wk * s.N * 3;
  const double xi = r[3 * i], yi = r[3 * i + 1], zi = r[3 * i + 2];
  const double a = hop_length(s, p, xi, yi, zi);
  double px[kHops], py[kHops], pz[kHops];
  hop_point<0>(xi, yi, zi, a, px[0], py[0], pz[0]);
  hop_point<1>(xi, yi, zi, a, px[1], py[1], pz[1]);
  hop_point<2>(xi, yi, zi, a, px[2], py[2], pz[2]);
  hop_point<3>(xi, yi, zi, a, px[3], py[3], pz[3]);
  hop_point<4>(xi, yi, zi, a, px[4], py[4], pz[4]);
  hop_point<5>(xi, yi, zi, a, px[5], py[5], pz[5]);

  // determinant ratios psi(r'_k) . Yt[i]
  double c[kHops] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const double* Y = w.Yt + ((long)wk * s.N + i) * s.Lp;
  // contracted orbitals: sum_c y_c phi_c(r') = sum_mu (sum_c C[mu][c] y_c) psi_mu(r')
  const int nb = s.nprim();
  for (int mu = lane; mu < nb; mu += 64) {
    const double4 f = s.bfn[mu];
    const int kind = s.kind[mu];
    const double y_mu = s.Lq ? prim_weight(s, mu, Y) : Y[mu];
#pragma unroll
    for (int k = 0; k < kHops; ++k) {
      const double dx = px[k] - f.x, dy = py[k] - f.y, dz = pz[k] - f.z;
      c[k] += angular_value(kind_ang(kind), dx, dy, dz) * radial_e(kind, f.w, dx * dx + dy * dy + dz * dz) * y_mu;
    }
  }

  // Jastrow change J(x'_k) - J(x)
  double dj[kHops] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (s.j1_form) {
    for (int n = lane; n < s.n_nuc; n += 64) {
      const double Rx = s.R[3 * n], Ry = s.R[3 * n + 1], Rz = s.R[3 * n + 2], Z = s.Z[n], b = s.j1_b[n];
      double f0, f1, f2;
      {
        const double dx = xi - Rx, dy = yi - Ry, dz = zi - Rz;
        j1_radial(s.j1_form, Z, b, sqrt(dx * dx + dy * dy + dz * dz), f0, f1, f2);
      }
#pragma unroll
      for (int k = 0; k < kHops; ++k) {
        const double dx = px[k] - Rx, dy = py[k] - Ry, dz = pz[k] - Rz;
        double g0, g1, g2;
        j1_radial(s.j1_form, Z, b, sqrt(dx * dx + dy * dy + dz * dz), g0, g1, g2);
        dj[k] += g0 - f0;
      }
    }
  }
  if (s.j2_form) {
    const bool up_i = i < s.nu;
    for (int j = lane; j < s.N; j += 64) {
      if (j == i) continue;
      const bool same = up_i == (j < s.nu);
      const double xj = r[3 * j], yj = r[3 * j + 1], zj = r[3 * j + 2];
      double v0, v1, v2;
      {
        const double dx = xi - xj, dy = yi - yj, dz = zi - zj;
        j2_radial(s.j2_form, s.j2d, same, sqrt(dx * dx + dy * dy + dz * dz), v0, v1, v2);
      }
#pragma unroll
      for (int k = 0; k < kHops; ++k) {
        const double dx = px[k] - xj, dy = py[k] - yj, dz = pz[k] - zj;
        double u0, u1, u2;
        j2_radial(s.j2_form, s.j2d, same, sqrt(dx * dx + dy * dy + dz * dz), u0, u1, u2);
        dj[k] += u0 - v0;
      }
    }
  }
  if (s.LJ) {   // Jastrow-basis change (chi(r'_k) - chi(r_i)) . (G_s - h_i + m_s)
    const int LJ = s.LJ, sp = i < s.nu ? 0 : 1;
    const double* ci = w.chi + ((long)wk * s.N + i) * LJ;
    const double* hi = w.hv + ((long)wk * s.N + i) * LJ;
    const double* G = w.G3 + ((long)wk * 2 + sp) * LJ;
    const double* m = s.jm + (long)sp * LJ;
    for (int q = lane; q < LJ; q += 64) {
      const double g = G[q] - hi[q] + m[q], c0 = ci[q];
#pragma unroll
      for (int k = 0; k < kHops; ++k) dj[k] += (basis_value_tab(s.jbfn, s.jkind, q, px[k], py[k], pz[k]) - c0) * g;
    }
  }
#pragma unroll
  for (int k = 0; k < kHops; ++k) {
    c[k] = wave_sum(c[k]);
    dj[k] = wave_sum(dj[k]);
  }
  if (lane == 0) {
    double* o = l.ratio + ((long)wk * s.N + i) * kHops;
#pragma unroll
    for (int k = 0; k < kHops; ++k) o[k] = c[k] * exp(dj[k]);
    l.ah[(long)wk * s.N + i] = a;
  }
}

__device__ double lr_block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += red[k];
  __syncthreads();
  return t;
}

// Off-diagonal fixed-node Green's function element of hop k (without the
// diagonal lambda): -H^FN_{x',x} Psi(x')/Psi(x).
__device__ __forceinline__ double green_off(double q, double a, double gamma) {
  const double h = 0.5 * (1.0 / (a * a));
  if (q > 0.0) return h * q;
  if (q < 0.0) return -((gamma * h) * q);
  return 0.0;
}

// One workgroup per walker: the per-walker terms of the Green's function column.
__global__ __launch_bounds__(256) void lrdmc_terms_kernel(SysDev s, WalkDev w, LrdmcDev l, LrdmcParams p) {
  __shared__ double red[4];
  const int wk = blockIdx.x;
  const int n6 = kHops * s.N;
  const double* q = l.ratio + (long)wk * n6;
  const double* ah = l.ah + (long)wk * s.N;
  double lap = 0.0, vsf = 0.0, pos = 0.0, ia2 = 0.0;
  for (int k = threadIdx.x; k < n6; k += blockDim.x) {
    const double a = ah[k / kHops];
    const double inv = 1.0 / (a * a);
    const double qk = q[k];
    lap += inv * (qk - 1.0);
    const double hq = (0.5 * inv) * qk;
    if (qk > 0.0) pos += hq;
    else if (qk < 0.0) vsf -= hq;
  }
  for (int i = threadIdx.x; i < s.N; i += blockDim.x) ia2 += 1.0 / (ah[i] * ah[i]);
  lap = lr_block_sum(lap, red);
  vsf = lr_block_sum(vsf, red);
  pos = lr_block_sum(pos, red);
  ia2 = lr_block_sum(ia2, red);
  if (threadIdx.x == 0) {
    const double ekin = l.ekin[wk], eloc = l.eloc[wk];
    const double shift = 0.5 * (lap + 2.0 * ekin);
    double* t = l.terms + (long)wk * kLrTerms;
    t[kLrEloc] = eloc;
    t[kLrEkin] = ekin;
    t[kLrLapA] = lap;
    t[kLrVaShift] = shift;
    t[kLrVsf] = vsf;
    t[kLrEscape] = pos + p.gamma * vsf;
    t[kLrHfnDiag] = 3.0 * ia2 + (eloc - ekin) + shift + (1.0 + p.gamma) * vsf;
  }
}

hipError_t launch_lrdmc_hops(const SysDev& s, const WalkDev& w, const LrdmcDev& l, const LrdmcParams& p,
                             hipStream_t st) {
  hipLaunchKernelGGL(lrdmc_ratio_kernel, dim3(w.Wk, (s.N + 3) / 4), dim3(256), 0, st, s, w, l, p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(lrdmc_terms_kernel, dim3(w.Wk), dim3(256), 0, st, s, w, l, p);
  return hipGetLastError();
}

// One workgroup per walker: the continuous-time step.  Hops are scanned in
// the order electron-major, then +x, -x, +y, -y, +z, -z; each thread owns a
// contiguous chunk, the chunk sums are scanned by one thread, and the first
// hop whose running sum exceeds xi1 * escape is taken (the smallest index any
// thread finds).
__global__ __launch_bounds__(256) void lrdmc_advance_kernel(SysDev s, WalkDev w, LrdmcDev l, LrdmcParams p,
                                                           const double* __restrict__ xi,
                                                           double* __restrict__ weight,
                                                           double* __restrict__ tau_left,
                                                           double* __restrict__ r_next,
                                                           int32_t* __restrict__ hop) {
  __shared__ double part[256];
  __shared__ int sel, last_pos;
  const int wk = blockIdx.x, tid = threadIdx.x;
  const int N = s.N, n6 = kHops * N;
  const double* r = w.r + (long)wk * N * 3;
  double* rn = r_next + (long)wk * N * 3;
  for (int k = tid; k < 3 * N; k += blockDim.x) rn[k] = r[k];
  const double tl = tau_left[wk];
  const double* t = l.terms + (long)wk * kLrTerms;
  const double esc = t[kLrEscape], eloc = t[kLrEloc];
  const bool skip = !(tl > 0.0) || w.singular[wk] != 0;
  const double tx = esc > 0.0 ? -log1p(-xi[2 * wk]) / esc : __builtin_inf();
  if (skip || tx >= tl) {                      // the same for every thread of the block
    if (tid == 0) {
      if (!skip) {
        weight[wk] *= exp(-tl * eloc);
        tau_left[wk] = 0.0;
      }
      if (hop) hop[wk] = -1;
    }
    return;
  }
  const double target = xi[2 * wk + 1] * esc;
  const double* q = l.ratio + (long)wk * n6;
  const double* ah = l.ah + (long)wk * N;
  const int chunk = (n6 + (int)blockDim.x - 1) / (int)blockDim.x;
  const int k0 = min(tid * chunk, n6), k1 = min(k0 + chunk, n6);
  double sum = 0.0;
  int lp = -1;
  for (int k = k0; k < k1; ++k) {
    const double g = green_off(q[k], ah[k / kHops], p.gamma);
    sum += g;
    if (g > 0.0) lp = k;
  }
  part[tid] = sum;
  if (tid == 0) { sel = 0x7fffffff; last_pos = -1; }
  __syncthreads();
  if (tid == 0) {
    double run = 0.0;
    for (int u = 0; u < (int)blockDim.x; ++u) {
      const double v = part[u];
      part[u] = run;
      run += v;
    }
  }
  if (lp >= 0) atomicMax(&last_pos, lp);
  __syncthreads();
  double run = part[tid];
  for (int k = k0; k < k1; ++k) {
    run += green_off(q[k], ah[k / kHops], p.gamma);
    if (run > target) {
      atomicMin(&sel, k);
      break;
    }
  }
  __syncthreads();
  if (tid == 0) {
    const int k = sel != 0x7fffffff ? sel : last_pos;
    weight[wk] *= exp(-tx * eloc);
    tau_left[wk] = tl - tx;
    if (hop) hop[wk] = k;
    if (k >= 0) {
      const int i = k / kHops, d = k % kHops;
      const int ax = d >> 1;
      const double a = ah[i];
      rn[3 * i + ax] = r[3 * i + ax] + ((d & 1) ? -a : a);
    }
  }
}

hipError_t launch_lrdmc_advance(const SysDev& s, const WalkDev& w, const LrdmcDev& l, const LrdmcParams& p,
                                const double* xi, double* weight, double* tau_left, double* r_next,
                                int32_t* hop, hipStream_t st) {
  hipLaunchKernelGGL(lrdmc_advance_kernel, dim3(w.Wk), dim3(256), 0, st, s, w, l, p, xi, weight, tau_left,
                     r_next, hop);
  return hipGetLastError();
}

}  // namespace qmc
