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
      j2_radial(s.j2_form, s.j2, up_e == (j < s.nu), rij, v, v1, v2);
      val += v;
      if (want_grad) { const double q = v1 / rij; gx += q * dx; gy += q * dy; gz += q * dz; }
    }
  }
}

// Step 1 of a proposal, one workgroup per walker: the new position, the basis
// values psi(r') (zero-padded to Lp, and their gradients when a drift is
// requested) and the Jastrow change J(x') - J(x) (and grad J at r').
// r_new: this walker's new position [3], or disp: its displacement [3].
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
  double* psi = w.psi_new + (long)wk * s.Lp;
  double* gpsi = w.gpsi_new + (long)wk * 3 * s.Lp;
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
  double jn, gxn, gyn, gzn, jo, d0, d1, d2;
  jastrow_one(s, r, e, px, py, pz, DRIFT, jn, gxn, gyn, gzn);
  jastrow_one(s, r, e, r[3 * e], r[3 * e + 1], r[3 * e + 2], false, jo, d0, d1, d2);
  const double dJ = block_sum_mv(jn - jo, red);
  if (DRIFT) {
    gxn = block_sum_mv(gxn, red); gyn = block_sum_mv(gyn, red); gzn = block_sum_mv(gzn, red);
  }
  if (tid == 0) {
    w.dJ[wk] = dJ;
    if (DRIFT) { w.gJ_new[3 * wk] = gxn; w.gJ_new[3 * wk + 1] = gyn; w.gJ_new[3 * wk + 2] = gzn; }
  }
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
// contribute exact zeros).  The W^{-1} entries that weight the rows are loaded
// once at the start, lane k holding the one of the wave's k-th row.
template <typename T, int NC>
__device__ void rows_body(const SysDev& s, const WalkDev& w, int wk, int sb, int S, int e, int R) {
  typedef typename Vec16<T>::type V;
  constexpr int VN = Vec16<T>::n;
  constexpr int STEP = 64 * VN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const bool up = e < s.nu;
  const int row0 = up ? s.nu : 0;
  const int nrow = up ? s.nd : s.nu;
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  const T* Pw = (const T*)w.P + ((long)wk * s.N + row0) * s.Lp;
  const double* Aw = w.A + (long)wk * s.nd * s.nu;
  double* wn_g = w.w_new + (long)wk * nmax;
  const double* psi = w.psi_new + (long)wk * s.Lp;
  const int j0 = sb * R;
  const int j1 = min(j0 + R, nrow);
  double a_own = 0.0;
  {
    const int j = j0 + wave + lane * nw;
    if (j < j1) a_own = up ? Aw[(long)j * s.nu + e] : Aw[(long)(e - s.nu) * s.nu + j];
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
    const T* pa = Pw + (long)j * s.Lp;
    const T* pb = two ? Pw + (long)jb * s.Lp : pa;   // never formed past the block
    V va[NC], vb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int i0 = c * STEP + lane * VN;
      va[c] = (i0 < s.Lp) ? *reinterpret_cast<const V*>(pa + i0) : V{};
      vb[c] = (two && i0 < s.Lp) ? *reinterpret_cast<const V*>(pb + i0) : V{};
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
  const int nrow = up ? s.nd : s.nu;
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  const T* Pw = (const T*)w.P + ((long)wk * s.N + row0) * s.Lp;
  const double* Aw = w.A + (long)wk * s.nd * s.nu;
  double* wn_g = w.w_new + (long)wk * nmax;
  const double* psi = w.psi_new + (long)wk * s.Lp;
  const double* gpsi = w.gpsi_new + (long)wk * 3 * s.Lp;
  const int j0 = sb * R;
  const int j1 = min(j0 + R, nrow);
  double part = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int j = j0 + wave; j < j1; j += nw) {
    const T* prow = Pw + (long)j * s.Lp;
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
      const double a = up ? Aw[(long)j * s.nu + e] : Aw[(long)(e - s.nu) * s.nu + j];
      part += a0 * a;
      if (DRIFT) { gx += ax * a; gy += ay * a; gz += az * a; }
    }
  }
  block_partial(part, gx, gy, gz, DRIFT, w, wk, S, sb);
}

// Sums 16 per-lane values over the 64 lanes of a wave with 17 shuffles in six
// dependent rounds: each of the first four rounds keeps half of the live values
// and trades the other half with the partner lane.  Lanes 4m..4m+3 return the
// total of x[m].
#define QMC_MS_STAGE(H, O)                                      \
  {                                                             \
    const bool hi = (lane & (O)) != 0;                          \
    _Pragma("unroll") for (int k = 0; k < (H); ++k) {           \
      const double send = hi ? x[k] : x[k + (H)];               \
      const double keep = hi ? x[k + (H)] : x[k];               \
      x[k] = keep + __shfl_xor(send, (O), 64);                  \
    }                                                           \
  }
__device__ __forceinline__ double wave_multi_sum16(double (&x)[16], int lane) {
  QMC_MS_STAGE(8, 32)
  QMC_MS_STAGE(4, 16)
  QMC_MS_STAGE(2, 8)
  QMC_MS_STAGE(1, 4)
  double t = x[0];
  t += __shfl_xor(t, 2, 64);
  t += __shfl_xor(t, 1, 64);
  return t;
}
#undef QMC_MS_STAGE

// ---------------------------------------------------------------------------
// Accept: decide (device Metropolis, u < ratio^2, when unif is given) and
// apply the rank-1 Sherman-Morrison update of A = W^{-1} in FP64:
//   up e   (row e of W replaced by w'):    A <- A - A[:,e] (delta^T A) / R
//   down e (column e of W replaced by w'): A <- A - (A delta) A[e,:] / R
// with delta = w' - (old row/column) and R = det W'/det W.  Thread t holds
// column c = t % n of rows g, g+G, ... (g = t / n, G = blockDim / n) in
// registers: A is read once and written once.  Column sums (up moves) combine
// the G groups' partials through LDS; row sums (down moves) are read row-wise
// (served from cache, the rows having just been read) and reduced 16 rows per
// wave at a time.  Every thread takes the acceptance decision itself from the
// same values, so no barrier precedes the loads of A.
// S > 0: the ratio is first summed from the proposal's S partial sums.
// ---------------------------------------------------------------------------
// acc_in: this walker's host decision (mode 0), or u: its uniform (mode 1).
// cnt: this walker's accept counter (may be null).
// UP = (e < n_up), fixed per instantiation so that each direction gets its own
// register allocation.
template <typename T, int QMAX, bool UP>
__device__ void accept_body(const SysDev& s, const WalkDev& w, int wk, int e, int mode,
                            const uint8_t* __restrict__ acc_in, double u, int32_t* __restrict__ cnt, int S) {
  __shared__ double delta[kLuMaxN];
  __shared__ double save[kLuMaxN];
  __shared__ double coef[kLuMaxN];
  __shared__ double part[256];
  const int n = s.nu;             // square: n_up == n_dn
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  double R, ratio;
  if (S > 0) {
    R = 0.0;
    for (int k = 0; k < S; ++k) R += w.rdet_part[(long)wk * S + k];
    ratio = R * exp(w.dJ[wk]);
  } else {
    R = w.rdet[wk];
    ratio = w.ratio[wk];
  }
  const bool acc = (mode == 1) ? (u < ratio * ratio) : (acc_in[0] != 0);
  if (tid == 0) {
    if (S > 0) { w.rdet[wk] = R; w.ratio[wk] = ratio; }
    w.acc[wk] = acc ? 1 : 0;
  }
  if (!acc) return;   // uniform over the block
  const double invR = 1.0 / R;
  constexpr bool up = UP;
  const int ed = e - s.nu;
  double* Aw = w.A + (long)wk * n * n;
  double* Ww = w.W + (long)wk * n * n;
  const double* wn = w.w_new + (long)wk * n;
  const int G = blockDim.x / n, c = tid % n, g = tid / n;
  const bool own = g < G;
  double a[QMAX];
  // up moves: the column slices load while delta and the bookkeeping proceed;
  // down moves load them after the row sums (cache hits, fewer live registers)
  if constexpr (UP) {
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = g + G * q;
      a[q] = (own && j < n) ? Aw[(long)j * n + c] : 0.0;
    }
  }
  for (int j = tid; j < n; j += blockDim.x)
    delta[j] = up ? wn[j] - Ww[(long)e * n + j] : wn[j] - Ww[(long)j * n + ed];
  // bookkeeping that does not depend on the update
  {
    T* prow = (T*)w.phi + ((long)wk * s.N + e) * s.Lp;
    const double* pn = w.psi_new + (long)wk * s.Lp;
    for (int mu = tid; mu < s.L; mu += blockDim.x) prow[mu] = (T)pn[mu];
    if (tid == 0) {
      double* re = w.r + ((long)wk * s.N + e) * 3;
      re[0] = w.r_new[3 * wk]; re[1] = w.r_new[3 * wk + 1]; re[2] = w.r_new[3 * wk + 2];
    }
    if (tid == (blockDim.x > 64 ? 64 : 0)) {
      const double dJ = w.dJ[wk];
      w.logabs[wk] += log(fabs(R)) + dJ;
      if (R < 0.0) w.sign[wk] = -w.sign[wk];
      w.J[wk] += dJ;
      if (cnt) cnt[0] += 1;
    }
  }
  __syncthreads();
  if constexpr (UP) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = g + G * q;
      if (own && j < n) t += delta[j] * a[q];
    }
    if (own) part[g * n + c] = t;
    if (own && c == e) {
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int j = g + G * q;
        if (j < n) save[j] = a[q];
      }
    }
    __syncthreads();
    if (own) {
      double uc = 0.0;
      for (int q = 0; q < G; ++q) uc += part[q * n + c];
      const double ck = uc * invR;
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int j = g + G * q;
        if (j < n) Aw[(long)j * n + c] = a[q] - save[j] * ck;
      }
    }
    for (int j = tid; j < n; j += blockDim.x) Ww[(long)e * n + j] = wn[j];
  } else {
    // rows j = wave + nw * m, 16 values of m per pass (n <= 32 nw)
    for (int m0 = 0; wave + nw * m0 < n; m0 += 16) {
      double x[16];
#pragma unroll
      for (int m = 0; m < 16; ++m) {
        const int j = wave + nw * (m0 + m);
        double t = 0.0;
        if (j < n)
          for (int i = lane; i < n; i += 64) t += Aw[(long)j * n + i] * delta[i];
        x[m] = t;
      }
      const double tot = wave_multi_sum16(x, lane);
      const int j = wave + nw * (m0 + (lane >> 2));
      if ((lane & 3) == 0 && j < n) coef[j] = tot * invR;
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = g + G * q;
      a[q] = (own && j < n) ? Aw[(long)j * n + c] : 0.0;
    }
    if (own && g == ed % G) {
      const int qe = ed / G;
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < QMAX; ++q) if (q == qe) v = a[q];
      save[c] = v;
    }
    __syncthreads();
    if (own) {
      const double sc = save[c];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int j = g + G * q;
        if (j < n) Aw[(long)j * n + c] = a[q] - coef[j] * sc;
      }
    }
    for (int i = tid; i < n; i += blockDim.x) Ww[(long)i * n + ed] = wn[i];
  }
}

}  // namespace qmc
