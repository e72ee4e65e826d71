// Device bodies of the single-electron move kernels, shared by the one-system
// launches (move.hip) and the persistent multi-system launches (multi.hip) so
// that both run the same arithmetic in the same order.  See move.hip for the
// method.
#pragma once

#include "internal.h"

namespace qmc {

__device__ double block_sum_mv(double v, double* red) {
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

// out[i] = sum_j M[i*ld + j] x[j] for i < m (m <= kWbMax), x in LDS, out in LDS.
// Rows are spread over groups of G lanes (G = blockDim / m rounded up to a power
// of two >= 4, at most 64), so the loads of every row are issued together rather
// than one row per wave at a time; each group reduces by a fixed xor-shuffle
// tree.  Called by every thread of the workgroup; the caller synchronises.
__device__ __forceinline__ void rows_dot_lds(const double* __restrict__ M, long ld, int m, int n,
                                             const double* x, double* out) {
  int mp = 4;
  while (mp < m) mp <<= 1;
  int G = (int)blockDim.x / mp;
  if (G > 64) G = 64;
  const int i = threadIdx.x / G, sub = threadIdx.x % G;
  double p = 0.0;
  if (i < m)
    for (int j = sub; j < n; j += G) p += M[(long)i * ld + j] * x[j];
  for (int o = G >> 1; o > 0; o >>= 1) p += __shfl_xor(p, o, 64);
  if (i < m && sub == 0) out[i] = p;
}

// Jastrow terms of electron e at position p, summed over this thread's share
// of nuclei and electrons: value and gradient.
__device__ void jastrow_one(const SysDev& s, const double* r, int e, double px, double py, double pz,
                            bool want_grad, double& val, double& gx, double& gy, double& gz) {
  val = 0.0; gx = gy = gz = 0.0;
  if (s.j1_form) {
    for (int a = threadIdx.x; a < s.n_nuc; a += blockDim.x) {
      const double dx = px - s.R[3 * a], dy = py - s.R[3 * a + 1], dz = pz - s.R[3 * a + 2];
      const double ria = sqrt(dx * dx + dy * dy + dz * dz);
      double f, f1, f2;
      j1_radial(s.j1_form, s.Z[a], s.j1_b[a], ria, f, f1, f2);
      val += f;
      if (want_grad) { const double q = f1 / ria; gx += q * dx; gy += q * dy; gz += q * dz; }
    }
  }
  if (s.j2_form) {
    const bool up_e = e < s.nu;
    for (int j = threadIdx.x; j < s.N; j += blockDim.x) {
      if (j == e) continue;
      const double dx = px - r[3 * j], dy = py - r[3 * j + 1], dz = pz - r[3 * j + 2];
      const double rij = sqrt(dx * dx + dy * dy + dz * dz);
      double v, v1, v2;
      j2_radial(s.j2_form, s.j2d, up_e == (j < s.nu), rij, v, v1, v2);
      val += v;
      if (want_grad) { const double q = v1 / rij; gx += q * dx; gy += q * dy; gz += q * dz; }
    }
  }
}

// The current inverse's column e (up move) or row e (down move) from the
// refresh inverse A0 and the delayed updates (one workgroup per walker):
//   v0 = A0[:, e] or A0[e, :],  t_i = d_i . v0,  z = S^{-1} t,  c = v0 - sum_i z_i v_i.
// v0, t, z and c are kept for the accept step.
__device__ void inverse_line_body(const SysDev& s, const WalkDev& w, int wk, int e) {
  __shared__ double sv0[kBigMaxN];
  __shared__ double st[kWbMax];
  __shared__ double sz[kWbMax];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = s.nu, kb = w.kb;
  const bool up = e < s.nu;
  const int ie = up ? e : e - s.nu;
  const double* A0 = w.A + (long)wk * n * n;
  double* v0 = w.v0 + (long)wk * n;
  double* cv = w.cvec + (long)wk * n;
  const int m = w.wm[wk];
  for (int j = tid; j < n; j += blockDim.x) {
    const double v = up ? A0[(long)j * n + ie] : A0[(long)ie * n + j];
    sv0[j] = v;
    v0[j] = v;
  }
  __syncthreads();
  if (m == 0) {
    for (int j = tid; j < n; j += blockDim.x) cv[j] = sv0[j];
    return;   // uniform
  }
  const double* D = w.wd + (long)wk * kb * n;
  const double* V = w.wv + (long)wk * kb * n;
  const double* Si = w.wS + (long)wk * kb * kb;
  double* tz = w.tz + (long)wk * 2 * kb;
  rows_dot_lds(D, n, m, n, sv0, st);          // t = D^T v0
  __syncthreads();
  rows_dot_lds(Si, kb, m, m, st, sz);         // z = S^{-1} t
  __syncthreads();
  for (int i = tid; i < m; i += blockDim.x) {
    tz[i] = st[i];
    tz[kb + i] = sz[i];
  }
  for (int j = tid; j < n; j += blockDim.x) {
    double c = sv0[j];
    for (int i = 0; i < m; ++i) c -= sz[i] * V[(long)i * n + j];
    cv[j] = c;
  }
}

// Step 1 of a proposal, one workgroup per walker: the new position, the basis
// values psi(r') (zero-padded to Lp, and their gradients when a drift is
// requested) and the Jastrow change J(x') - J(x) (and grad J at r').
// r_new: this walker's new position [3], or disp: its displacement [3].
// psi(r') (zero-padded to Lp; with their gradients when DRIFT) into this
// walker's psi_new / gpsi_new: the basis functions, or the contracted orbitals
// (primitives at r' into the walker's slice of qbuf, then phi_c = sum_t C_t
// psi_{idx_t}).  Called by every thread of the workgroup.
template <bool DRIFT>
__device__ void orbitals_at(const SysDev& s, const WalkDev& w, int wk, double px, double py, double pz) {
  const int tid = threadIdx.x;
  double* psi = w.psi_new + (long)wk * s.Lp;
  double* gpsi = w.gpsi_new + (long)wk * 3 * s.Lp;
  if (s.Lq) {
    const int Lq = s.Lq;
    double* qb = w.qbuf + (long)wk * 4 * Lq;
    for (int mu = tid; mu < Lq; mu += blockDim.x) {
      if (DRIFT) {
        double v, gx, gy, gz, lp;
        basis_vgl(s, mu, px, py, pz, v, gx, gy, gz, lp);
        qb[mu] = v; qb[Lq + mu] = gx; qb[2 * Lq + mu] = gy; qb[3 * Lq + mu] = gz;
      } else {
        qb[mu] = basis_value(s, mu, px, py, pz);
      }
    }
    __syncthreads();
    for (int c = tid; c < s.Lp; c += blockDim.x) {
      double v = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      if (c < s.L)
        for (int k = s.con_ptr[c]; k < s.con_ptr[c + 1]; ++k) {
          const double cf = s.con_coef[k];
          const int mu = s.con_idx[k];
          v += cf * qb[mu];
          if (DRIFT) { gx += cf * qb[Lq + mu]; gy += cf * qb[2 * Lq + mu]; gz += cf * qb[3 * Lq + mu]; }
        }
      psi[c] = v;
      if (DRIFT) { gpsi[c] = gx; gpsi[s.Lp + c] = gy; gpsi[2 * s.Lp + c] = gz; }
    }
    return;
  }
  for (int mu = tid; mu < s.Lp; mu += blockDim.x) {
    if (mu >= s.L) {
      psi[mu] = 0.0;
      if (DRIFT) { gpsi[mu] = 0.0; gpsi[s.Lp + mu] = 0.0; gpsi[2 * s.Lp + mu] = 0.0; }
    } else if (DRIFT) {
      double v, gx, gy, gz, lp;
      basis_vgl(s, mu, px, py, pz, v, gx, gy, gz, lp);
      psi[mu] = v; gpsi[mu] = gx; gpsi[s.Lp + mu] = gy; gpsi[2 * s.Lp + mu] = gz;
    } else {
      psi[mu] = basis_value(s, mu, px, py, pz);
    }
  }
}

// This thread's share of J(x') - J(x) for electron e moved to p (and of grad J
// at p when DRIFT): one- and two-body terms, and with a Jastrow basis
// (chi(r') - chi(r_e)) . (G_s - h_e + m_s), writing chi(r') into chi_new.
template <bool DRIFT>
__device__ void jastrow_change(const SysDev& s, const WalkDev& w, int wk, int e, double px, double py, double pz,
                               double& dj, double& gxn, double& gyn, double& gzn) {
  const int tid = threadIdx.x;
  const double* r = w.r + (long)wk * s.N * 3;
  double jn, jo, d0, d1, d2;
  jastrow_one(s, r, e, px, py, pz, DRIFT, jn, gxn, gyn, gzn);
  jastrow_one(s, r, e, r[3 * e], r[3 * e + 1], r[3 * e + 2], false, jo, d0, d1, d2);
  dj = jn - jo;
  if (s.LJ) {
    const int sp = e < s.nu ? 0 : 1, LJ = s.LJ;
    const double* ce = w.chi + ((long)wk * s.N + e) * LJ;
    const double* he = w.hv + ((long)wk * s.N + e) * LJ;
    const double* G = w.G3 + ((long)wk * 2 + sp) * LJ;
    const double* m = s.jm + (long)sp * LJ;
    double* cn = w.chi_new + (long)wk * LJ;
    for (int k = tid; k < LJ; k += blockDim.x) {
      const double g = G[k] - he[k] + m[k];
      double v;
      if (DRIFT) {
        double vx, vy, vz, vl;
        basis_vgl_tab(s.jbfn, s.jkind, k, px, py, pz, v, vx, vy, vz, vl);
        gxn += vx * g; gyn += vy * g; gzn += vz * g;
      } else {
        v = basis_value_tab(s.jbfn, s.jkind, k, px, py, pz);
      }
      cn[k] = v;
      dj += (v - ce[k]) * g;
    }
  }
}

// Screened proposals (QMC_REFINED): the basis functions at r' whose column of
// the streamed P rows can change the ratio.  Over the rows j of the other spin,
//   |sum_j c_j P_j[mu] psi_mu(r')| <= |psi_mu(r')| cmax_mu sum_j |c_j|,
// cmax_mu = max_j |P_j[mu]|, c the current inverse column (row) of the moved
// electron.  Functions with |psi_mu| cmax_mu |c|_1 <= kScreenTol / L are
// skipped, so all skipped ones together change the ratio by at most
// kScreenTol (and each new W entry by at most kScreenTol / |c|_1).  The kept
// ones are listed in increasing mu with their values.  Called by every thread
// of the workgroup after psi_new and cvec of electron e are written.
__device__ void screen_list_body(const SysDev& s, const WalkDev& w, int wk, int e) {
  __shared__ double red[8];
  __shared__ int wcount[4];
  __shared__ int total;
  __syncthreads();
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool up = e < s.nu;
  const double* cv = w.cvec + (long)wk * s.nu;
  double c1 = 0.0;
  for (int j = tid; j < s.nu; j += blockDim.x) c1 += fabs(cv[j]);
  c1 = block_sum_mv(c1, red);
  const double thr = (c1 > 0.0) ? kScreenTol / ((double)s.L * c1) : 0.0;
  const double* cm = w.cmax + ((long)wk * 2 + (up ? 1 : 0)) * s.Lp;   // the rows the proposal streams
  const double* psi = w.psi_new + (long)wk * s.Lp;
  int* mk = w.muk + (long)wk * s.Lp;
  double* pk = w.psk + (long)wk * s.Lp;
  if (tid == 0) total = 0;
  __syncthreads();
  for (int base = 0; base < s.L; base += blockDim.x) {
    const int mu = base + tid;
    double v = 0.0;
    bool keep = false;
    if (mu < s.L) {
      v = psi[mu];
      keep = fabs(v) * cm[mu] > thr;
    }
    const unsigned long long b = __ballot(keep);
    if (lane == 0) wcount[wave] = __popcll(b);
    __syncthreads();
    int off = total;
    for (int k = 0; k < wave; ++k) off += wcount[k];
    if (keep) {
      const int at = off + __popcll(b & ((1ull << lane) - 1ull));
      mk[at] = mu;
      pk[at] = v;
    }
    __syncthreads();
    if (tid == 0) {
      int t = total;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += wcount[k];
      total = t;
    }
    __syncthreads();
  }
  if (tid == 0) w.nkeep[wk] = total;
}

template <bool DRIFT>
__device__ void prep_body(const SysDev& s, const WalkDev& w, int wk, int e, const double* __restrict__ r_new,
                          const double* __restrict__ disp) {
  __shared__ double red[8];
  __shared__ double rn[3];
  const int tid = threadIdx.x;
  const double* r = w.r + (long)wk * s.N * 3;
  if (tid < 3) {
    rn[tid] = disp ? r[3 * e + tid] + disp[tid] : r_new[tid];
    w.r_new[3 * wk + tid] = rn[tid];
  }
  __syncthreads();
  const double px = rn[0], py = rn[1], pz = rn[2];
  orbitals_at<DRIFT>(s, w, wk, px, py, pz);
  double dj, gxn, gyn, gzn;
  jastrow_change<DRIFT>(s, w, wk, e, px, py, pz, dj, gxn, gyn, gzn);
  const double dJ = block_sum_mv(dj, red);
  if (DRIFT) {
    gxn = block_sum_mv(gxn, red); gyn = block_sum_mv(gyn, red); gzn = block_sum_mv(gzn, red);
  }
  if (tid == 0) {
    w.dJ[wk] = dJ;
    if (DRIFT) { w.gJ_new[3 * wk] = gxn; w.gJ_new[3 * wk + 1] = gyn; w.gJ_new[3 * wk + 2] = gzn; }
  }
  inverse_line_body(s, w, wk, e);
  if (s.screened()) screen_list_body(s, w, wk, e);
}

template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef double2 type; static constexpr int n = 2; };
template <> struct Vec16<float> { typedef float4 type; static constexpr int n = 4; };
template <> struct Vec16<bf16s> { typedef uint4 type; static constexpr int n = 8; };

__device__ __forceinline__ double vget(const double2& v, int i) { return i == 0 ? v.x : v.y; }
__device__ __forceinline__ double vget(const float4& v, int i) {
  return (double)(i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w)));
}
// eight BF16 values: element i is half i % 2 of word i / 2 (exact widening)
__device__ __forceinline__ double vget(const uint4& v, int i) {
  const uint32_t w = (i >> 1) == 0 ? v.x : ((i >> 1) == 1 ? v.y : ((i >> 1) == 2 ? v.z : v.w));
  return (double)__uint_as_float((i & 1) ? (w & 0xffff0000u) : (w << 16));
}

// 16-byte load marked non-temporal (the P rows are read once per proposal).
template <typename V>
__device__ __forceinline__ V load16_nt(const void* p) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 x = __builtin_nontemporal_load(reinterpret_cast<const u4*>(p));
  V v;
  __builtin_memcpy(&v, &x, 16);
  return v;
}

// Combine the per-wave (lane 0) partial ratios of one block into rdet_part.
__device__ __forceinline__ void block_partial(double part, double gx, double gy, double gz, bool drift,
                                              const WalkDev& w, int wk, int S, int sb) {
  __shared__ double red[16];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    red[wave] = part;
    if (drift) { red[4 + wave] = gx; red[8 + wave] = gy; red[12 + wave] = gz; }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
    for (int k = 0; k < nw; ++k) {
      t += red[k];
      if (drift) { tx += red[4 + k]; ty += red[8 + k]; tz += red[12 + k]; }
    }
    w.rdet_part[(long)wk * S + sb] = t;
    if (drift) {
      double* g = w.gdet_part + ((long)wk * S + sb) * 3;
      g[0] = tx; g[1] = ty; g[2] = tz;
    }
  }
}

// Step 2, streaming: the workgroup computes the new W entries of rows
// [sb*R, (sb+1)*R) of the opposite spin of walker wk and their contribution to
// the determinant ratio (partial sum sb of S).  Wave v takes rows j0+v, j0+v+nw,
// ... two at a time (both rows' loads in flight before either reduction);
// psi(r') chunks sit in registers and each row is read with NC independent
// 16-byte loads per lane (NC = ceil(Lp / (64 * 16 / sizeof(T))); chunks past Lp
// contribute exact zeros).  The entries of the current inverse's column (up) or
// row (down) that weight the rows are loaded once at the start, lane k holding
// the one of the wave's k-th row.  FP64 rows are loaded non-temporally: on
// MI355X that streams them at 80 % of the HBM peak instead of 71 %, while it
// slows the FP32 rows (34 -> 50 us per launch), which keep ordinary loads.
template <typename T, int NC>
__device__ void rows_body(const SysDev& s, const WalkDev& w, int wk, int sb, int S, int e, int R) {
  typedef typename Vec16<T>::type V;
  constexpr int VN = Vec16<T>::n;
  constexpr int STEP = 64 * VN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const bool up = e < s.nu;
  const int row0 = up ? s.nu : 0;
  const int nrow = s.nu;   // W is n_up x n_up: a row has n_dn paired and nk unpaired columns
  const T* Pw = (const T*)w.P + ((long)wk * s.N + row0) * s.Lp;
  // row j of the streamed side: walker rows, then (up moves) the unpaired orbitals
  auto rowp = [&](int j) -> const T* {
    return (up && j >= s.nd) ? (const T*)s.UphS + (long)(j - s.nd) * s.Lp : Pw + (long)j * s.Lp;
  };
  const double* cv = w.cvec + (long)wk * s.nu;
  double* wn_g = w.w_new + (long)wk * s.nu;
  const double* psi = w.psi_new + (long)wk * s.Lp;
  const int j0 = sb * R;
  const int j1 = min(j0 + R, nrow);
  double a_own = 0.0;
  {
    const int j = j0 + wave + lane * nw;
    if (j < j1) a_own = cv[j];
  }
  double ps[NC][VN];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int i0 = c * STEP + lane * VN;
#pragma unroll
    for (int v = 0; v < VN; ++v) ps[c][v] = (i0 < s.Lp) ? psi[i0 + v] : 0.0;
  }
  double part = 0.0;
  int k = 0;
  for (int j = j0 + wave; j < j1; j += 2 * nw, k += 2) {
    const int jb = j + nw;
    const bool two = jb < j1;   // uniform over the wave
    const T* pa = rowp(j);
    const T* pb = two ? rowp(jb) : pa;   // never formed past the block
    V va[NC], vb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int i0 = c * STEP + lane * VN;
      if constexpr (sizeof(T) == 8) {
        va[c] = (i0 < s.Lp) ? load16_nt<V>(pa + i0) : V{};
        vb[c] = (two && i0 < s.Lp) ? load16_nt<V>(pb + i0) : V{};
      } else {
        va[c] = (i0 < s.Lp) ? *reinterpret_cast<const V*>(pa + i0) : V{};
        vb[c] = (two && i0 < s.Lp) ? *reinterpret_cast<const V*>(pb + i0) : V{};
      }
    }
    double xa = 0.0, xb = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        xa += vget(va[c], v) * ps[c][v];
        xb += vget(vb[c], v) * ps[c][v];
      }
    xa = wave_sum(xa);
    xb = wave_sum(xb);
    const double aa = __shfl(a_own, k, 64), ab = __shfl(a_own, k + 1, 64);
    if (lane == 0) {
      wn_g[j] = xa;
      part += xa * aa;
      if (two) {
        wn_g[jb] = xb;
        part += xb * ab;
      }
    }
  }
  block_partial(part, 0.0, 0.0, 0.0, false, w, wk, S, sb);
}

// Generic streaming kernel (any Lp; optional gradients for the drift at r').
template <typename T, bool DRIFT>
__device__ void rows_generic_body(const SysDev& s, const WalkDev& w, int wk, int sb, int S, int e, int R) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const bool up = e < s.nu;
  const int row0 = up ? s.nu : 0;
  const int nrow = s.nu;   // W is n_up x n_up (see rows_body)
  const T* Pw = (const T*)w.P + ((long)wk * s.N + row0) * s.Lp;
  const double* cv = w.cvec + (long)wk * s.nu;
  double* wn_g = w.w_new + (long)wk * s.nu;
  const double* psi = w.psi_new + (long)wk * s.Lp;
  const double* gpsi = w.gpsi_new + (long)wk * 3 * s.Lp;
  const int j0 = sb * R;
  const int j1 = min(j0 + R, nrow);
  double part = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int j = j0 + wave; j < j1; j += nw) {
    const T* prow = (up && j >= s.nd) ? (const T*)s.UphS + (long)(j - s.nd) * s.Lp : Pw + (long)j * s.Lp;
    double a0 = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int mu = lane; mu < s.Lp; mu += 64) {
      const double p = (double)prow[mu];
      a0 += p * psi[mu];
      if (DRIFT) { ax += p * gpsi[mu]; ay += p * gpsi[s.Lp + mu]; az += p * gpsi[2 * s.Lp + mu]; }
    }
    a0 = wave_sum(a0);
    if (DRIFT) { ax = wave_sum(ax); ay = wave_sum(ay); az = wave_sum(az); }
    if (lane == 0) {
      wn_g[j] = a0;
      const double a = cv[j];
      part += a0 * a;
      if (DRIFT) { gx += ax * a; gy += ay * a; gz += az * a; }
    }
  }
  block_partial(part, gx, gy, gz, DRIFT, w, wk, S, sb);
}

// ---------------------------------------------------------------------------
// Accept: decide (device Metropolis, u < ratio^2, when u is given) and record
// the accepted move as a delayed update (one workgroup per walker).  With
// delta = w' - (old row / column of W), v0, t, z and c from the proposal:
//   r_j = delta . v_j (j < m),  gamma = 1 + delta . v0 - r . z  (= 1 + delta . c,
//   the determinant ratio),  y = S^{-T} r,
//   S^{-1} <- [[S^{-1} + z y^T / gamma, -z / gamma], [-y^T / gamma, 1 / gamma]],
//   v_m = v0, d_m = delta, m <- m + 1   (the bordered inverse of S).
// The inverse itself is not touched; W's row / column, the basis row, the
// position and the tracked log|Psi|, sign and Jastrow sum are.
// S > 0: the ratio is first summed from the proposal's S partial sums.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void accept_apply(const SysDev& s, const WalkDev& w, int wk, int e, double R, int m,
                             int32_t* __restrict__ cnt);

// Jastrow-basis state after electron e (spin s) moved: with dchi = chi(r') - chi(r_e),
// [G_u; G_d] += M3[:, s block] dchi, h_e = M^{ss} chi(r'), chi_e = chi(r').
// Called by every thread of the workgroup (block-uniform).
__device__ void jastrow3_accept(const SysDev& s, const WalkDev& w, int wk, int e) {
  const int LJ = s.LJ, sp = e < s.nu ? 0 : 1;
  double* ce = w.chi + ((long)wk * s.N + e) * LJ;
  const double* cn = w.chi_new + (long)wk * LJ;
  double* G = w.G3 + (long)wk * 2 * LJ;
  double* he = w.hv + ((long)wk * s.N + e) * LJ;
  for (int o = threadIdx.x; o < 3 * LJ; o += blockDim.x) {
    if (o < 2 * LJ) {
      const double* row = s.M3 + (long)o * 2 * LJ + (long)sp * LJ;
      double g = 0.0;
      for (int k = 0; k < LJ; ++k) g += row[k] * (cn[k] - ce[k]);
      G[o] += g;
    } else {
      const int j = o - 2 * LJ;
      const double* row = s.M3 + ((long)sp * LJ + j) * 2 * LJ + (long)sp * LJ;
      double h = 0.0;
      for (int k = 0; k < LJ; ++k) h += row[k] * cn[k];
      he[j] = h;
    }
  }
  __syncthreads();   // every read of chi_e is done
  for (int k = threadIdx.x; k < LJ; k += blockDim.x) ce[k] = cn[k];
}

// acc_in: this walker's host decision (mode 0), or u: its uniform (mode 1).
// cnt: this walker's accept counter (may be null).
template <typename T>
__device__ void accept_body(const SysDev& s, const WalkDev& w, int wk, int e, int mode,
                            const uint8_t* __restrict__ acc_in, double u, int32_t* __restrict__ cnt, int S) {
  const int tid = threadIdx.x;
  double R, ratio;
  if (S > 0) {
    R = 0.0;
    for (int k = 0; k < S; ++k) R += w.rdet_part[(long)wk * S + k];
    ratio = R * exp(w.dJ[wk]);
  } else {
    R = w.rdet[wk];
    ratio = w.ratio[wk];
  }
  const int kb = w.kb, m = w.wm[wk];
  // a full buffer cannot occur (the host refreshes first); if it did, the move
  // is rejected rather than written past the buffer
  const bool acc = m < kb && ((mode == 1) ? (u < ratio * ratio) : (acc_in[0] != 0));
  if (tid == 0) {
    if (S > 0) { w.rdet[wk] = R; w.ratio[wk] = ratio; }
    w.acc[wk] = acc ? 1 : 0;
  }
  if (acc) accept_apply<T>(s, w, wk, e, R, m, cnt);   // uniform over the block
}

template <typename T>
__device__ void accept_apply(const SysDev& s, const WalkDev& w, int wk, int e, double R, int m,
                             int32_t* __restrict__ cnt) {
  __shared__ double sd[kBigMaxN];
  __shared__ double sr[kWbMax];
  __shared__ double sy[kWbMax];
  __shared__ double red[16];
  __shared__ double gam_s;
  const int n = s.nu;             // W is n_up x n_up
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int kb = w.kb;
  const bool up = e < s.nu;
  const int ie = up ? e : e - s.nu;
  double* Ww = w.W + (long)wk * n * n;
  const double* wn = w.w_new + (long)wk * n;
  const double* v0 = w.v0 + (long)wk * n;
  double* D = w.wd + (long)wk * kb * n;
  double* V = w.wv + (long)wk * kb * n;
  double* Si = w.wS + (long)wk * kb * kb;
  const double* tz = w.tz + (long)wk * 2 * kb;
  // delta, then W's row / column and the new buffer entries
  double p0 = 0.0;
  for (int j = tid; j < n; j += blockDim.x) {
    const long off = up ? (long)ie * n + j : (long)j * n + ie;
    const double d = wn[j] - Ww[off];
    sd[j] = d;
    p0 += d * v0[j];
    D[(long)m * n + j] = d;
    V[(long)m * n + j] = v0[j];
  }
  // delta . v0 (block sum in fixed order)
  p0 = wave_sum(p0);
  if (lane == 0) red[wave] = p0;
  __syncthreads();
  rows_dot_lds(V, n, m, n, sd, sr);           // r_i = delta . v_i
  __syncthreads();
  if (tid == 0) {
    double dv = 0.0;
    for (int k = 0; k < nw; ++k) dv += red[k];
    double rz = 0.0;
    for (int i = 0; i < m; ++i) rz += sr[i] * tz[kb + i];
    gam_s = 1.0 + dv - rz;
  }
  for (int k = tid; k < m; k += blockDim.x) {
    double y = 0.0;
    for (int i = 0; i < m; ++i) y += Si[i * kb + k] * sr[i];
    sy[k] = y;
  }
  __syncthreads();
  const double ig = 1.0 / gam_s;
  for (int idx = tid; idx < (m + 1) * (m + 1); idx += blockDim.x) {
    const int i = idx / (m + 1), k = idx % (m + 1);
    double v;
    if (i < m && k < m) v = Si[i * kb + k] + tz[kb + i] * sy[k] * ig;
    else if (i < m) v = -tz[kb + i] * ig;
    else if (k < m) v = -sy[k] * ig;
    else v = ig;
    Si[i * kb + k] = v;
  }
  for (int j = tid; j < n; j += blockDim.x) {
    if (up) Ww[(long)ie * n + j] = wn[j];
    else Ww[(long)j * n + ie] = wn[j];
  }
  T* prow = (T*)w.phi + ((long)wk * s.N + e) * s.Lp;
  const double* pn = w.psi_new + (long)wk * s.Lp;
  for (int mu = tid; mu < s.L; mu += blockDim.x) prow[mu] = (T)pn[mu];
  if (s.LJ) jastrow3_accept(s, w, wk, e);
  if (tid == 0) {
    w.wm[wk] = m + 1;
    double* re = w.r + ((long)wk * s.N + e) * 3;
    re[0] = w.r_new[3 * wk]; re[1] = w.r_new[3 * wk + 1]; re[2] = w.r_new[3 * wk + 2];
    const double dJ = w.dJ[wk];
    w.logabs[wk] += log(fabs(R)) + dJ;
    if (R < 0.0) w.sign[wk] = -w.sign[wk];
    w.J[wk] += dJ;
    if (cnt) cnt[0] += 1;
  }
}

// ---------------------------------------------------------------------------
// Metropolis accept of electron e fused with the set-up of the next proposal
// (electron e2 != e, displacement disp2), one workgroup per walker.  The basis
// values at r' = r[e2] + disp2 do not depend on the accept (it changes only
// r[e]); they are computed first, into LDS, so that their arithmetic overlaps
// the accept's memory round trips.  After a barrier (the accept has consumed
// psi_new, r_new, dJ, v0 and z) the set-up continues exactly as prep_body:
// psi_new, r_new, the Jastrow change with the updated positions and the
// current inverse's column / row of e2 from the updated buffer.
// ---------------------------------------------------------------------------
template <typename T>
__device__ void accept_prep_body(const SysDev& s, const WalkDev& w, int wk, int e, double u,
                                 int32_t* __restrict__ cnt, int S, int e2, const double* __restrict__ disp2) {
  __shared__ double sps[kFuseMaxLp];
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const double* r = w.r + (long)wk * s.N * 3;
  const double px = r[3 * e2] + disp2[0], py = r[3 * e2 + 1] + disp2[1], pz = r[3 * e2 + 2] + disp2[2];
  for (int mu = tid; mu < s.L; mu += blockDim.x) sps[mu] = basis_value(s, mu, px, py, pz);
  accept_body<T>(s, w, wk, e, 1, nullptr, u, cnt, S);
  __syncthreads();
  double* psi = w.psi_new + (long)wk * s.Lp;
  for (int mu = tid; mu < s.Lp; mu += blockDim.x) psi[mu] = mu < s.L ? sps[mu] : 0.0;
  if (tid < 3) w.r_new[3 * wk + tid] = tid == 0 ? px : (tid == 1 ? py : pz);
  double jn, gxn, gyn, gzn, jo, d0, d1, d2;
  jastrow_one(s, r, e2, px, py, pz, false, jn, gxn, gyn, gzn);
  jastrow_one(s, r, e2, r[3 * e2], r[3 * e2 + 1], r[3 * e2 + 2], false, jo, d0, d1, d2);
  const double dJ = block_sum_mv(jn - jo, red);
  if (tid == 0) w.dJ[wk] = dJ;
  inverse_line_body(s, w, wk, e2);
  if (s.screened()) screen_list_body(s, w, wk, e2);
}

}  // namespace qmc
