// Single-electron moves (the ratio Psi(x')/Psi(x) and the update after an
// accepted move).  A move of electron e changes one row of W (e spin up) or
// one column (e spin down) and nothing else, since neither the basis nor the
// Jastrow has backflow (Wave functions section).  With P = Phi Lambda kept per
// walker, the new row/column is a single dot product per entry:
//   up e:    w'_j = sum_mu psi_mu(r') P_dn[j][mu]          (P_dn = Phi_dn Lambda^T)
//   down e:  w'_i = sum_nu P_up[i][nu] psi_nu(r')          (P_up = Phi_up Lambda)
// and by the matrix-determinant lemma
//   up e:    det W'/det W = sum_j w'_j A[j][e]
//   down e:  det W'/det W = sum_i A[e][i] w'_i
// accumulated in FP64 whatever the storage precision of P.  The Jastrow
// factor contributes exp(J(x') - J(x)) over the N_at + N - 1 terms that
// involve the moved electron.
//
// The proposal streams the N/2 x L block of P of the other spin for every
// walker: it is bound by HBM bandwidth.  A small per-walker kernel first
// computes psi(r') and the Jastrow change; the streaming kernel then splits
// each walker's rows over several workgroups (s.prop_rows() rows each) so that
// many blocks are in flight, and every block writes a partial determinant
// ratio, which the accept kernel (device Metropolis) or the finalize kernel
// (host-driven moves) sums in a fixed order.
#include <hip/hip_ext.h>

#include "move_dev.h"
#include <algorithm>

namespace qmc {

constexpr int kStageQL = (kFuseMaxLp + 255) / 256;   // per-thread slots over Lp <= kFuseMaxLp
__host__ __device__ inline size_t pad1k(size_t b) { return (b + 1023) & ~(size_t)1023; }
typedef double dbl2 __attribute__((ext_vector_type(2)));

template <bool DRIFT>
__global__ void __launch_bounds__(256)
propose_prep_kernel(SysDev s, WalkDev w, int e, const double* __restrict__ r_new_in,
                    const double* __restrict__ disp) {
  const int wk = blockIdx.x;
  prep_body<DRIFT>(s, w, wk, e, r_new_in ? r_new_in + 3 * (long)wk : nullptr,
                   disp ? disp + 3 * (long)wk : nullptr);
}

// 1-D grid of S * Wk blocks; block (wk, sb) handles rows [sb*R, (sb+1)*R) of
// walker wk, R = s.prop_rows().  Workgroups are handed to the eight XCDs in
// turn (block b to XCD b mod 8), each with its own L2: when Wk is a multiple of
// 8 the S blocks of one walker are given ids with one residue mod 8, so psi(r')
// and the inverse column they all read come from HBM once per walker, not once
// per XCD.
__device__ __forceinline__ void rows_block(int b, int S, int Wk, int& wk, int& sb) {
  if ((Wk & 7) == 0) {
    const int q = b >> 3;
    wk = (b & 7) + 8 * (q / S);
    sb = q % S;
  } else {
    wk = b / S;
    sb = b % S;
  }
}

template <typename T, int NC>
__global__ void __launch_bounds__(256) propose_rows_kernel(SysDev s, WalkDev w, int e, int S) {
  int wk, sb;
  rows_block(blockIdx.x, S, w.Wk, wk, sb);
  rows_body<T, NC>(s, w, wk, sb, S, e, s.prop_rows());
}

template <typename T, bool DRIFT>
__global__ void __launch_bounds__(256) propose_rows_generic_kernel(SysDev s, WalkDev w, int e, int S) {
  int wk, sb;
  rows_block(blockIdx.x, S, w.Wk, wk, sb);
  rows_generic_body<T, DRIFT>(s, w, wk, sb, S, e, s.prop_rows());
}

template <typename T>
__global__ void __launch_bounds__(256)
accept_kernel(SysDev s, WalkDev w, int e, const uint8_t* __restrict__ acc_in,
              const double* __restrict__ unif, int32_t* __restrict__ accept_count, int S) {
  const int wk = blockIdx.x;
  accept_body<T>(s, w, wk, e, unif ? 1 : 0, acc_in ? acc_in + wk : nullptr, unif ? unif[wk] : 0.0,
                 accept_count ? accept_count + wk : nullptr, S);
}

template <typename T>
__global__ void __launch_bounds__(256)
accept_prep_kernel(SysDev s, WalkDev w, int e, const double* __restrict__ unif, int32_t* __restrict__ accept_count,
                   int S, int e2, const double* __restrict__ disp2) {
  const int wk = blockIdx.x;
  accept_prep_body<T>(s, w, wk, e, unif[wk], accept_count ? accept_count + wk : nullptr, S, e2,
                      disp2 + 3 * (long)wk);
}

// Sum the partial ratios (fixed order) for host-driven proposals.
__global__ void propose_finalize_kernel(WalkDev w, int S, double* __restrict__ ratio_o,
                                        double* __restrict__ drift_o) {
  const int wk = blockIdx.x * blockDim.x + threadIdx.x;
  if (wk >= w.Wk) return;
  double R = 0.0;
  for (int k = 0; k < S; ++k) R += w.rdet_part[(long)wk * S + k];
  const double ratio = R * exp(w.dJ[wk]);
  w.rdet[wk] = R;
  w.ratio[wk] = ratio;
  if (ratio_o) ratio_o[wk] = ratio;
  if (drift_o) {
    // grad log|det| of the moved electron at r' uses the updated inverse, whose
    // column (row) e equals the old one divided by the determinant ratio
    double g[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < S; ++k)
      for (int c = 0; c < 3; ++c) g[c] += w.gdet_part[((long)wk * S + k) * 3 + c];
    for (int c = 0; c < 3; ++c) drift_o[3 * wk + c] = g[c] / R + w.gJ_new[3 * wk + c];
  }
}

int propose_splits(const SysDev& s) {
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  const int R = s.prop_rows();
  return (nmax + R - 1) / R;
}

hipError_t launch_propose_prep(const SysDev& s, const WalkDev& w, int e, const double* r_new,
                               const double* disp, bool drift, hipStream_t st) {
  if (drift)
    hipLaunchKernelGGL(propose_prep_kernel<true>, dim3(w.Wk), dim3(256), 0, st, s, w, e, r_new, disp);
  else
    hipLaunchKernelGGL(propose_prep_kernel<false>, dim3(w.Wk), dim3(256), 0, st, s, w, e, r_new, disp);
  return hipGetLastError();
}

// ev_start / ev_stop (may be null): events recorded by the streaming kernel's
// own dispatch (hipExtLaunchKernelGGL), so that they time that kernel alone.
hipError_t launch_propose_rows(const SysDev& s, const WalkDev& w, int e, double* ratio,
                               double* drift_new, bool finalize, hipStream_t st, hipEvent_t ev_start,
                               hipEvent_t ev_stop) {
  const bool drift = drift_new != nullptr;
  if (s.prop_rows() < kPropRowsMin) return hipErrorInvalidValue;   // rdet_part would overflow
  const int S = propose_splits(s);
  const dim3 grid((unsigned)(S * w.Wk));
  const int store = s.store();
  hipError_t err;
  const int vn = store == 0 ? 2 : (store == 1 ? 4 : 8);   // elements per 16-byte load
  const int chunks = (s.Lp + 64 * vn - 1) / (64 * vn);
#define QMC_GEN(D)                                                                                         \
  if (store == 2) hipExtLaunchKernelGGL((propose_rows_generic_kernel<bf16s, D>), grid, dim3(256), 0, st, ev_start, ev_stop, 0, s, w, e, S); \
  else if (store == 1) hipExtLaunchKernelGGL((propose_rows_generic_kernel<float, D>), grid, dim3(256), 0, st, ev_start, ev_stop, 0, s, w, e, S); \
  else hipExtLaunchKernelGGL((propose_rows_generic_kernel<double, D>), grid, dim3(256), 0, st, ev_start, ev_stop, 0, s, w, e, S);
  if (drift) {
    QMC_GEN(true)
  } else if (chunks <= 8) {
#define QMC_ROWS(T, NC) \
    case NC: hipExtLaunchKernelGGL((propose_rows_kernel<T, NC>), grid, dim3(256), 0, st, ev_start, ev_stop, 0, s, w, e, S); break;
    if (store == 2) {
      switch (chunks) { QMC_ROWS(bf16s, 1) QMC_ROWS(bf16s, 2) QMC_ROWS(bf16s, 3) QMC_ROWS(bf16s, 4)
                        QMC_ROWS(bf16s, 5) QMC_ROWS(bf16s, 6) QMC_ROWS(bf16s, 7) QMC_ROWS(bf16s, 8) }
    } else if (store == 1) {
      switch (chunks) { QMC_ROWS(float, 1) QMC_ROWS(float, 2) QMC_ROWS(float, 3) QMC_ROWS(float, 4)
                        QMC_ROWS(float, 5) QMC_ROWS(float, 6) QMC_ROWS(float, 7) QMC_ROWS(float, 8) }
    } else {
      switch (chunks) { QMC_ROWS(double, 1) QMC_ROWS(double, 2) QMC_ROWS(double, 3) QMC_ROWS(double, 4)
                        QMC_ROWS(double, 5) QMC_ROWS(double, 6) QMC_ROWS(double, 7) QMC_ROWS(double, 8) }
    }
#undef QMC_ROWS
  } else {
    QMC_GEN(false)
  }
#undef QMC_GEN
  err = hipGetLastError();
  if (err != hipSuccess || !finalize) return err;
  hipLaunchKernelGGL(propose_finalize_kernel, dim3((w.Wk + 255) / 256), dim3(256), 0, st, w, S, ratio,
                     drift_new);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Screened proposals (QMC_REFINED).  The new W row (column) of walker wk is
//   w'_j = sum over the kept mu of psi_mu(r') PT[wk][mu][i0 + j],
// one contiguous column of the other spin's rows per kept basis function (the
// skipped ones change the ratio by at most kScreenTol, see screen_list_body).
// One workgroup per walker: wave v takes kept functions v, v + 4, ..., four at
// a time, lane l the rows l, l + 64, ...; the waves' partial rows are added in
// a fixed order through LDS, then the ratio sum_j w'_j c_j.  The ratio goes to
// the first of the walker's S partial slots (the others are zeroed), which the
// accept and finalize kernels sum as usual.
// ---------------------------------------------------------------------------
template <int NB>
__global__ void __launch_bounds__(256) propose_screened_kernel(SysDev s, WalkDev w, int e, int S) {
  __shared__ double part[4][64 * NB];
  __shared__ double red[8];
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool up = e < s.nu;
  const int i0 = up ? s.nu : 0;
  const int n = up ? s.nd : s.nu;
  const double* base = w.PT + (long)wk * s.Lp * s.N + i0;
  const int cnt = w.nkeep[wk];
  const int* mk = w.muk + (long)wk * s.Lp;
  const double* pk = w.psk + (long)wk * s.Lp;
  double acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = 0.0;
  int k = wave;
  for (; k + 12 < cnt; k += 16) {   // four functions in flight per wave
    int mu[4];
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { mu[q] = mk[k + 4 * q]; v[q] = pk[k + 4 * q]; }
    double x[4][NB];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = lane + 64 * b;
        x[q][b] = j < n ? __builtin_nontemporal_load(base + (long)mu[q] * s.N + j) : 0.0;
      }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] += v[q] * x[q][b];
  }
  for (; k < cnt; k += 4) {
    const int mu = mk[k];
    const double v = pk[k];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = lane + 64 * b;
      if (j < n) acc[b] += v * base[(long)mu * s.N + j];
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) part[wave][lane + 64 * b] = acc[b];
  __syncthreads();
  const double* cv = w.cvec + (long)wk * s.nu;
  double* wn = w.w_new + (long)wk * s.nu;
  double rp = 0.0;
  for (int j = tid; j < n; j += blockDim.x) {
    const double x = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
    wn[j] = x;
    rp += x * cv[j];
  }
  const double R = block_sum_mv(rp, red);
  for (int q = tid; q < S; q += blockDim.x) w.rdet_part[(long)wk * S + q] = q == 0 ? R : 0.0;
}

// Blocked form of the same sum, for an even row count n: the kept functions
// are taken FB at a time (FB n a multiple of 128, IPB = FB n / 128 <= 8), and
// a wave reads a block's FB columns (FB n doubles) with IPB 16-byte loads of
// all 64 lanes: lane l of load i holds the two rows j, j + 1 of function f
// with 2 (64 i + l) = f n + j, fixed over the blocks.  The kept list and the
// inverse line come first (one round), then every wave issues about eight
// loads at once (8 / IPB blocks), some 32 KiB in flight per walker.  The
// per-lane sums go to LDS and row j adds its FB x 4 partial sums in a fixed
// order (waves outer, functions inner).
template <int IPB>
__global__ void __launch_bounds__(256) propose_screened_blk_kernel(SysDev s, WalkDev w, int e, int S, int FB) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double red[8];
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool up = e < s.nu;
  const int i0 = up ? s.nu : 0;
  const int n = up ? s.nd : s.nu;
  const int Lp = s.Lp;
  const double* base = w.PT + (long)wk * Lp * s.N + i0;
  int* lmu = (int*)lds;
  double* lv = (double*)(lds + pad1k(sizeof(int) * (size_t)Lp));
  dbl2* part = (dbl2*)((char*)lv + pad1k(sizeof(double) * (size_t)Lp));
  // the kept list (the whole Lp-long arrays: no wait on the count), c
  const int* mk = w.muk + (long)wk * Lp;
  const double* pk = w.psk + (long)wk * Lp;
  int xm[kStageQL];
  double xv[kStageQL];
#pragma unroll
  for (int k = 0; k < kStageQL; ++k) {
    const int q = tid + 256 * k, qc = q < Lp ? q : 0;
    xm[k] = mk[qc];
    xv[k] = pk[qc];
  }
  const int cnt = w.nkeep[wk];
  const double cj = w.cvec[(long)wk * s.nu + (tid < n ? tid : 0)];
#pragma unroll
  for (int k = 0; k < kStageQL; ++k) {
    const int q = tid + 256 * k;
    if (q < Lp) { lmu[q] = xm[k]; lv[q] = xv[k]; }
  }
  __syncthreads();
  // this lane's (function, row) of each of its IPB loads
  int fi[IPB], ji[IPB];
#pragma unroll
  for (int i = 0; i < IPB; ++i) {
    const int el = 2 * (64 * i + lane);
    fi[i] = el / n;
    ji[i] = el - fi[i] * n;
  }
  dbl2 acc[IPB];
#pragma unroll
  for (int i = 0; i < IPB; ++i) acc[i] = dbl2{0.0, 0.0};
  const int nblk = (cnt + FB - 1) / FB;
  constexpr int UB = 8 / IPB > 1 ? 8 / IPB : 1;   // blocks per wave in flight (8 loads)
  for (int b0 = wave; b0 < nblk; b0 += 4 * UB) {
    dbl2 x[UB][IPB];
    double vv[UB][IPB];
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int i = 0; i < IPB; ++i) {
        const int kk = (b0 + 4 * u) * FB + fi[i];
        const bool ok = kk < cnt;
        const int mu = lmu[ok ? kk : 0];
        vv[u][i] = ok ? lv[kk] : 0.0;
        x[u][i] = __builtin_nontemporal_load((const dbl2*)(base + (long)mu * s.N + ji[i]));
      }
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int i = 0; i < IPB; ++i) {
        acc[i].x += vv[u][i] * x[u][i].x;
        acc[i].y += vv[u][i] * x[u][i].y;
      }
  }
#pragma unroll
  for (int i = 0; i < IPB; ++i) part[wave * 64 * IPB + 64 * i + lane] = acc[i];
  __syncthreads();
  const double* pd = (const double*)part;
  double* wn = w.w_new + (long)wk * s.nu;
  double rp = 0.0;
  if (tid < n) {
    double t = 0.0;
    for (int v = 0; v < 4; ++v)
      for (int f = 0; f < FB; ++f) t += pd[v * 128 * IPB + f * n + tid];
    wn[tid] = t;
    rp = t * cj;
  }
  const double R = block_sum_mv(rp, red);
  for (int q = tid; q < S; q += blockDim.x) w.rdet_part[(long)wk * S + q] = q == 0 ? R : 0.0;
}

// Column maxima of the P halves (bit 0: up rows, bit 1: down rows):
// cmax[w][h][mu] = max over the rows i of half h of |P[w][i][mu]|.
// One workgroup per (walker, half), columns in chunks of 512: wave v takes the
// rows v, v + 4, ..., each lane the columns lane + 64 c of the chunk (all
// eight loaded per row together), and the four waves' maxima meet in LDS (a
// maximum does not depend on the order).
__global__ void __launch_bounds__(256) screen_colmax_kernel(SysDev s, WalkDev w, int halves) {
  constexpr int CM = 8;
  __shared__ double part[4][64 * CM];
  const int wk = blockIdx.x, h = blockIdx.y;
  if (!((halves >> h) & 1)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = h == 0 ? 0 : s.nu, n = h == 0 ? s.nu : s.nd, Lp = s.Lp;
  const double* P = (const double*)w.P + ((long)wk * s.N + i0) * Lp;
  double* out = w.cmax + ((long)wk * 2 + h) * Lp;
  for (int c0 = 0; c0 < Lp; c0 += 64 * CM) {
    double m[CM];
#pragma unroll
    for (int c = 0; c < CM; ++c) m[c] = 0.0;
    for (int i = wave; i < n; i += 4) {
      const double* row = P + (long)i * Lp + c0;
      double v[CM];
#pragma unroll
      for (int c = 0; c < CM; ++c) {
        const int mu = lane + 64 * c;
        v[c] = c0 + mu < Lp ? __builtin_nontemporal_load(row + mu) : 0.0;
      }
#pragma unroll
      for (int c = 0; c < CM; ++c) m[c] = fmax(m[c], fabs(v[c]));
    }
    __syncthreads();   // the previous chunk's maxima are written out
#pragma unroll
    for (int c = 0; c < CM; ++c) part[wave][lane + 64 * c] = m[c];
    __syncthreads();
    for (int mu = tid; mu < 64 * CM && c0 + mu < Lp; mu += blockDim.x)
      out[c0 + mu] = fmax(fmax(part[0][mu], part[1][mu]), fmax(part[2][mu], part[3][mu]));
  }
}

__global__ void int_to_double_kernel(const int* __restrict__ src, double* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = (double)src[i];
}

hipError_t launch_export_kept(const WalkDev& w, double* dst, hipStream_t st) {
  if (!w.nkeep) return hipErrorInvalidValue;
  hipLaunchKernelGGL(int_to_double_kernel, dim3((w.Wk + 255) / 256), dim3(256), 0, st, w.nkeep, dst, w.Wk);
  return hipGetLastError();
}

hipError_t launch_screen_colmax(const SysDev& s, const WalkDev& w, int halves, hipStream_t st) {
  if (!w.cmax) return hipErrorInvalidValue;
  hipLaunchKernelGGL(screen_colmax_kernel, dim3(w.Wk, 2), dim3(256), 0, st, s, w, halves);
  return hipGetLastError();
}

hipError_t launch_propose_screened(const SysDev& s, const WalkDev& w, int e, double* ratio, bool finalize,
                                   hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (!w.PT || !w.muk) return hipErrorInvalidValue;
  const int n = e < s.nu ? s.nd : s.nu;
  const int S = propose_splits(s);
  const dim3 grid(w.Wk), blk(256);
  // blocked kernel: n even, FB = 128 / gcd(n, 128) functions per block, IPB
  // = FB n / 128 loads per lane and block, at most 8; n <= 256 (one row per
  // thread in the final sums), Lp <= kFuseMaxLp (the kept list in LDS)
  int g = 128;
  while (n % g) g >>= 1;
  const int FB = 128 / g, IPB = FB * n / 128;
  if (n % 2 == 0 && n <= 256 && IPB <= 8 && s.Lp <= kFuseMaxLp && (uintptr_t)w.PT % 16 == 0 && s.N % 2 == 0 &&
      (e < s.nu ? s.nu : 0) % 2 == 0) {
    const size_t lds = pad1k(sizeof(int) * (size_t)s.Lp) + pad1k(sizeof(double) * (size_t)s.Lp) +
                       sizeof(dbl2) * 4 * 64 * (size_t)IPB;
#define QMC_SBLK(I) case I: hipExtLaunchKernelGGL(propose_screened_blk_kernel<I>, grid, blk, lds, st, ev_start, ev_stop, 0, s, w, e, S, FB); break;
    switch (IPB) { QMC_SBLK(1) QMC_SBLK(2) QMC_SBLK(3) QMC_SBLK(4) QMC_SBLK(5) QMC_SBLK(6) QMC_SBLK(7) QMC_SBLK(8) }
#undef QMC_SBLK
  } else if (n <= 64) hipExtLaunchKernelGGL(propose_screened_kernel<1>, grid, blk, 0, st, ev_start, ev_stop, 0, s, w, e, S);
  else if (n <= 128) hipExtLaunchKernelGGL(propose_screened_kernel<2>, grid, blk, 0, st, ev_start, ev_stop, 0, s, w, e, S);
  else if (n <= 256) hipExtLaunchKernelGGL(propose_screened_kernel<4>, grid, blk, 0, st, ev_start, ev_stop, 0, s, w, e, S);
  else if (n <= 512) hipExtLaunchKernelGGL(propose_screened_kernel<8>, grid, blk, 0, st, ev_start, ev_stop, 0, s, w, e, S);
  else if (n <= 1024) hipExtLaunchKernelGGL(propose_screened_kernel<16>, grid, blk, 0, st, ev_start, ev_stop, 0, s, w, e, S);
  else return hipErrorNotSupported;
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || !finalize) return err;
  hipLaunchKernelGGL(propose_finalize_kernel, dim3((w.Wk + 255) / 256), dim3(256), 0, st, w, S, ratio,
                     (double*)nullptr);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Metropolis accept of e fused with the set-up of e2, staged through LDS.
// The same arithmetic in the same order as accept_prep_body (so chains are
// bitwise those of the unstaged kernel and of the multi-system launches), but
// every input the workgroup reads is requested at once at the start: the
// delayed-update buffers V and D (rows below mc), S^{-1} and the positions go
// global -> LDS by direct copies (no registers held), while the basis records
// of psi(r'), the nuclei of the one-body Jastrow, the new and old W line, v0
// and z of the pending proposal, A0's line of e2, psi(r') of the pending
// proposal and the column maxima of the screened proposals go to registers.
// psi(r') of e2 is computed while the copies are in flight.  The unstaged
// kernel walks a chain of some fifteen dependent global round trips per
// walker; this one, one.
// mc bounds the buffered moves: at the accept of an attempt, wm <= the
// attempts since the last refresh (both restart together, wm grows by at
// most one per attempt), which the host passes.  A walker with more (not
// reachable through the move calls) reads the buffers from global memory.
// LDS: V, D [(mc+1) n], S^{-1} [(mc+1) kb], r [3 N] (each padded to 1 KiB,
// the copy granule), psi(r') of e2 [Lp], three n-vectors, five kb-vectors.
// ---------------------------------------------------------------------------
constexpr int kStageMaxN = 128;    // n <= 128 (one W entry per thread)
constexpr int kStageMaxNe = 256;   // electrons
constexpr int kStageMaxNuc = 256;  // nuclei (one per thread)
constexpr int kStageMaxSplits = (kStageMaxN + kPropRowsMin - 1) / kPropRowsMin;   // partial ratios
constexpr size_t kStageMaxLds = 63 * 1024;   // dynamic LDS (the static arrays take the rest of 64 KiB)

struct StageLayout {
  size_t V, D, S, vec, total;   // byte offsets of the regions and the size
};
__host__ __device__ inline StageLayout stage_layout(int n, int kb, int mc) {
  StageLayout o;
  o.V = 0;
  o.D = o.V + pad1k(sizeof(double) * (size_t)(mc + 1) * n);
  o.S = o.D + pad1k(sizeof(double) * (size_t)(mc + 1) * n);
  o.vec = o.S + pad1k(sizeof(double) * (size_t)(mc + 1) * kb);
  o.total = o.vec + sizeof(double) * (3 * (size_t)n + 5 * (size_t)kb);
  return o;
}

// bytes (a multiple of 8) from global src to LDS dst in 1 KiB granules, 16
// bytes per lane (global_load_lds): granule j by wave j mod the wave count.
// Lanes past the end re-read src's first 16 bytes into dst's padding.
__device__ __forceinline__ void lds_copy_async(void* dst, const void* src, int bytes) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const char* s = (const char*)src;
  char* d = (char*)dst;
  const int nch = (bytes + 1023) >> 10;
  for (int j = wave; j < nch; j += nw) {
    const int off = (j << 10) + 16 * lane;
    const char* p = off < bytes ? s + off : s;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)p,
                                     (__attribute__((address_space(3))) void*)(d + (j << 10)), 16, 0, 0);
  }
}

// Prefetched per-thread inputs of the staged kernel.
struct StagePre {
  double4 bf[kStageQL];   // basis records of mu = tid + 256 q
  int bk[kStageQL];
  double xp[kStageQL];    // psi(r') of the pending proposal (the accepted row)
  double xc[kStageQL];    // column maxima of the rows e2's proposal streams (screened)
  double sv[kStageQL];    // psi(r') of e2 (computed)
  double nx, ny, nz, nZ, nb;   // nucleus tid (one-body Jastrow)
  double ex, ey, ez;           // electron tid's position (two-body Jastrow)
  double wn, Wo, v0, a0, z;    // new W entry, old one, v0, A0's line of e2, z (thread = index)
};

// jastrow_one for N <= the block size: nucleus tid's record and electron
// tid's position (xj, yj, zj) in registers, the two-body parameters (j2p, the
// eight of s.j2d) in LDS.
__device__ __forceinline__ double jastrow_staged(const SysDev& s, int e, double px, double py, double pz,
                                                 const StagePre& q, double xj, double yj, double zj,
                                                 const double* j2p) {
  double val = 0.0;
  const int tid = threadIdx.x;
  if (s.j1_form) {
    if (tid < s.n_nuc) {
      const double dx = px - q.nx, dy = py - q.ny, dz = pz - q.nz;
      const double ria = sqrt(dx * dx + dy * dy + dz * dz);
      double f, f1, f2;
      j1_radial(s.j1_form, q.nZ, q.nb, ria, f, f1, f2);
      val += f;
    }
  }
  if (s.j2_form) {
    const bool up_e = e < s.nu;
    const int j = tid;
    if (j < s.N && j != e) {
      const double dx = px - xj, dy = py - yj, dz = pz - zj;
      const double rij = sqrt(dx * dx + dy * dy + dz * dz);
      double v, v1, v2;
      j2_radial(s.j2_form, j2p, up_e == (j < s.nu), rij, v, v1, v2);
      val += v;
    }
  }
  return val;
}

template <typename T, bool STAGED, int QL>
__device__ void accept_prep_staged_body(const SysDev& s, const WalkDev& w, int wk, int e, double u,
                                        int32_t* __restrict__ cnt, int cnt0, int S, int e2, double px, double py,
                                        double pz, double R, double dJ, int m, int mc, char* lds, const StagePre& q,
                                        const double* j2p, double la, double sg, double jv, double rx, double ry,
                                        double rz, double ox, double oy, double oz) {
  __shared__ double red[16];
  __shared__ double gam_s;
  __shared__ int wcnt[QL][4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = s.nu, kb = w.kb, N = s.N, L = s.L, Lp = s.Lp;
  const bool up = e < n;
  const int ie = up ? e : e - n;
  const StageLayout ly = stage_layout(n, kb, mc);
  double* Vl = (double*)(lds + ly.V);
  double* Dl = (double*)(lds + ly.D);
  double* Sl = (double*)(lds + ly.S);
  double* sd = (double*)(lds + ly.vec);
  double* sv0 = sd + n;
  double* cvl = sv0 + n;
  double* zo = cvl + n;
  double* sr = zo + kb;
  double* sy = sr + kb;
  double* st = sy + kb;
  double* sz = st + kb;
  double* Vg = w.wv + (long)wk * kb * n;
  double* Dg = w.wd + (long)wk * kb * n;
  double* Sg = w.wS + (long)wk * kb * kb;
  const double* Vr = STAGED ? Vl : Vg;
  const double* Dr = STAGED ? Dl : Dg;
  double* Sr = STAGED ? Sl : Sg;

  // the accept of e (accept_body, Metropolis mode)
  const double ratio = R * exp(dJ);
  const bool acc = m < kb && u < ratio * ratio;
  if (tid == 0) {
    w.rdet[wk] = R;
    w.ratio[wk] = ratio;
    w.acc[wk] = acc ? 1 : 0;
  }
  if (acc) {
    double p0 = 0.0;
    if (tid < n) {
      const double d = q.wn - q.Wo;
      sd[tid] = d;
      p0 += d * q.v0;
      Dg[(long)m * n + tid] = d;
      Vg[(long)m * n + tid] = q.v0;
      if (STAGED) { Dl[(long)m * n + tid] = d; Vl[(long)m * n + tid] = q.v0; }
    }
    p0 = wave_sum(p0);
    if (lane == 0) red[wave] = p0;
    __syncthreads();
    rows_dot_lds(Vr, n, m, n, sd, sr);           // r_i = delta . v_i
    __syncthreads();
    if (tid == 0) {
      double dv = 0.0;
      for (int k = 0; k < nw; ++k) dv += red[k];
      double rzs = 0.0;
      for (int i = 0; i < m; ++i) rzs += sr[i] * zo[i];
      gam_s = 1.0 + dv - rzs;
    }
    for (int k = tid; k < m; k += blockDim.x) {
      double y = 0.0;
      for (int i = 0; i < m; ++i) y += Sr[i * kb + k] * sr[i];
      sy[k] = y;
    }
    __syncthreads();
    const double ig = 1.0 / gam_s;
    for (int idx = tid; idx < (m + 1) * (m + 1); idx += blockDim.x) {
      const int i = idx / (m + 1), k = idx % (m + 1);
      double v;
      if (i < m && k < m) v = Sr[i * kb + k] + zo[i] * sy[k] * ig;
      else if (i < m) v = -zo[i] * ig;
      else if (k < m) v = -sy[k] * ig;
      else v = ig;
      Sr[i * kb + k] = v;
      if (STAGED) Sg[i * kb + k] = v;
    }
    if (tid < n) {
      double* Ww = w.W + (long)wk * n * n;
      if (up) Ww[(long)ie * n + tid] = q.wn;
      else Ww[(long)tid * n + ie] = q.wn;
    }
    T* prow = (T*)w.phi + ((long)wk * N + e) * Lp;
#pragma unroll
    for (int k = 0; k < QL; ++k) {
      const int mu = tid + 256 * k;
      if (mu < L) prow[mu] = (T)q.xp[k];
    }
    if (tid == 0) {
      w.wm[wk] = m + 1;
      double* re = w.r + ((long)wk * N + e) * 3;
      re[0] = rx; re[1] = ry; re[2] = rz;
      w.logabs[wk] = la + (log(fabs(R)) + dJ);
      if (R < 0.0) w.sign[wk] = -sg;
      w.J[wk] = jv + dJ;
      if (cnt) cnt[0] = cnt0 + 1;
    }
  }
  __syncthreads();

  // the set-up of e2: psi(r'), r', the Jastrow change (with e at its new
  // position when accepted)
  double* psi = w.psi_new + (long)wk * Lp;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = tid + 256 * k;
    if (mu < Lp) psi[mu] = mu < L ? q.sv[k] : 0.0;
  }
  if (tid < 3) w.r_new[3 * wk + tid] = tid == 0 ? px : (tid == 1 ? py : pz);
  const bool me = acc && tid == e;
  const double xj = me ? rx : q.ex, yj = me ? ry : q.ey, zj = me ? rz : q.ez;
  const double jn = jastrow_staged(s, e2, px, py, pz, q, xj, yj, zj, j2p);
  const double jo = jastrow_staged(s, e2, ox, oy, oz, q, xj, yj, zj, j2p);
  const double dJ2 = block_sum_mv(jn - jo, red);
  if (tid == 0) w.dJ[wk] = dJ2;

  // the current inverse's line of e2 (inverse_line_body)
  double* v0g = w.v0 + (long)wk * n;
  double* cv = w.cvec + (long)wk * n;
  if (tid < n) v0g[tid] = sv0[tid];
  const int m2 = acc ? m + 1 : m;
  if (m2 == 0) {
    if (tid < n) { cv[tid] = sv0[tid]; cvl[tid] = sv0[tid]; }
  } else {
    double* tz = w.tz + (long)wk * 2 * kb;
    rows_dot_lds(Dr, n, m2, n, sv0, st);        // t = D^T v0
    __syncthreads();
    rows_dot_lds(Sr, kb, m2, m2, st, sz);       // z = S^{-1} t
    __syncthreads();
    for (int i = tid; i < m2; i += blockDim.x) {
      tz[i] = st[i];
      tz[kb + i] = sz[i];
    }
    if (tid < n) {
      double c = sv0[tid];
      for (int i = 0; i < m2; ++i) c -= sz[i] * Vr[(long)i * n + tid];
      cv[tid] = c;
      cvl[tid] = c;
    }
  }
  if (!s.screened()) return;

  // screened proposals of e2 (screen_list_body)
  __syncthreads();
  double c1 = 0.0;
  for (int j = tid; j < n; j += blockDim.x) c1 += fabs(cvl[j]);
  c1 = block_sum_mv(c1, red);
  const double thr = (c1 > 0.0) ? kScreenTol / ((double)L * c1) : 0.0;
  int* mk = w.muk + (long)wk * Lp;
  double* pk = w.psk + (long)wk * Lp;
  // the kept functions in increasing mu: every slot's ballot first, one
  // barrier, then each kept lane's place from the counts before it
  unsigned long long bal[QL];
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = 256 * k + tid;
    const bool keep = mu < L && fabs(q.sv[k]) * q.xc[k] > thr;
    bal[k] = __ballot(keep);
    if (lane == 0) wcnt[k][wave] = __popcll(bal[k]);
  }
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    int before = off;   // kept in earlier slots, then earlier waves of this slot
    for (int k2 = 0; k2 < wave; ++k2) before += wcnt[k][k2];
    if ((bal[k] >> lane) & 1ull) {
      const int at = before + __popcll(bal[k] & ((1ull << lane) - 1ull));
      mk[at] = 256 * k + tid;
      pk[at] = q.sv[k];
    }
    for (int k2 = 0; k2 < nw; ++k2) off += wcnt[k][k2];
  }
  if (tid == 0) w.nkeep[wk] = off;
}

template <typename T, int QL>
__global__ void __launch_bounds__(256)
accept_prep_staged_kernel(SysDev s, WalkDev w, int e, const double* __restrict__ unif,
                          int32_t* __restrict__ accept_count, int S, int e2, const double* __restrict__ disp2,
                          int mc) {
  extern __shared__ __align__(16) char lds[];
  __shared__ double scal[kStageMaxSplits + 22];
  __shared__ int ints_s[2];
  const int wk = blockIdx.x, tid = threadIdx.x;
  const int n = s.nu, kb = w.kb, N = s.N, L = s.L, Lp = s.Lp;
  const bool up = e < n, up2 = e2 < n;
  const int ie = up ? e : e - n, ie2 = up2 ? e2 : e2 - n;
  const StageLayout ly = stage_layout(n, kb, mc);
  // bulk copies first
  lds_copy_async(lds + ly.V, w.wv + (long)wk * kb * n, 8 * mc * n);
  lds_copy_async(lds + ly.D, w.wd + (long)wk * kb * n, 8 * mc * n);
  lds_copy_async(lds + ly.S, w.wS + (long)wk * kb * kb, 8 * mc * kb);
  // per-thread loads, every address valid (indices past the ends read element 0)
  StagePre q;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = tid + 256 * k, mc0 = mu < L ? mu : 0;
    q.bf[k] = s.bfn[mc0];
    q.bk[k] = s.kind[mc0];
  }
  {
    const int a = tid < s.n_nuc ? tid : 0;
    q.nx = s.R[3 * a]; q.ny = s.R[3 * a + 1]; q.nz = s.R[3 * a + 2];
    q.nZ = s.Z[a];
    q.nb = s.j1_b[a];
    const double* rj = w.r + ((long)wk * N + (tid < N ? tid : 0)) * 3;
    q.ex = rj[0]; q.ey = rj[1]; q.ez = rj[2];
  }
  {
    const int j = tid < n ? tid : 0;
    const double* Ww = w.W + (long)wk * n * n;
    const double* A0 = w.A + (long)wk * n * n;
    q.wn = w.w_new[(long)wk * n + j];
    q.Wo = up ? Ww[(long)ie * n + j] : Ww[(long)j * n + ie];
    q.v0 = w.v0[(long)wk * n + j];
    q.a0 = up2 ? A0[(long)j * n + ie2] : A0[(long)ie2 * n + j];
    q.z = w.tz[(long)wk * 2 * kb + kb + (tid < kb ? tid : 0)];
  }
  const double* pn = w.psi_new + (long)wk * Lp;
  const double* cm = s.screened() ? w.cmax + ((long)wk * 2 + (up2 ? 1 : 0)) * Lp : pn;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = tid + 256 * k, mc0 = mu < L ? mu : 0;
    q.xp[k] = pn[mc0];
    q.xc[k] = cm[mc0];
  }
  // the walker's scalars, one per thread, through LDS: the S partial ratios
  // (threads 0..S-1), then dJ, log|Psi|, sign, J, u, the displacement of e2,
  // r' of e and r of e2 and the eight two-body parameters (wave 1), the
  // buffered-move and accept counts.  Loads first, unconditionally (every
  // address valid), stores after.
  const double pv = w.rdet_part[(long)wk * S + (tid < S ? tid : 0)];
  const int t2 = tid - 64;
  const double* sp;
  switch (t2) {
    case 0: sp = w.dJ + wk; break;
    case 1: sp = w.logabs + wk; break;
    case 2: sp = w.sign + wk; break;
    case 3: sp = w.J + wk; break;
    case 4: sp = unif + wk; break;
    case 5: case 6: case 7: sp = disp2 + 3 * (long)wk + (t2 - 5); break;
    case 8: case 9: case 10: sp = w.r_new + 3 * (long)wk + (t2 - 8); break;
    case 11: case 12: case 13: sp = w.r + ((long)wk * N + e2) * 3 + (t2 - 11); break;
    case 14: case 15: case 16: case 17: case 18: case 19: case 20: case 21: sp = s.j2d + (t2 - 14); break;
    default: sp = w.dJ + wk; break;
  }
  const double sv_ = *sp;
  const int mv = w.wm[wk];
  const int cv_ = accept_count ? accept_count[wk] : 0;
  if (tid < S) scal[tid] = pv;
  if (t2 >= 0 && t2 < 22) scal[kStageMaxSplits + t2] = sv_;
  if (tid == 128) { ints_s[0] = mv; ints_s[1] = cv_; }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies landed
  __syncthreads();
  double R = 0.0;
  for (int k = 0; k < S; ++k) R += scal[k];
  const double* sc = scal + kStageMaxSplits;
  const double dJ = sc[0], la = sc[1], sg = sc[2], jv = sc[3], u = sc[4];
  const double rx = sc[8], ry = sc[9], rz = sc[10];
  const double px = sc[11] + sc[5], py = sc[12] + sc[6], pz = sc[13] + sc[7];
  const int m = ints_s[0];
  double* sv0 = (double*)(lds + ly.vec) + n;
  double* zo = sv0 + 2 * n;
  // psi(r') of e2
#pragma unroll
  for (int k = 0; k < QL; ++k) q.sv[k] = basis_value_rec(q.bf[k], q.bk[k], px, py, pz);
  if (tid < n) sv0[tid] = q.a0;
  if (tid < kb) zo[tid] = q.z;
  __syncthreads();
  int32_t* cnt = accept_count ? accept_count + wk : nullptr;
  if (m <= mc)
    accept_prep_staged_body<T, true, QL>(s, w, wk, e, u, cnt, ints_s[1], S, e2, px, py, pz, R, dJ, m, mc, lds, q,
                                         sc + 14, la, sg, jv, rx, ry, rz, sc[11], sc[12], sc[13]);
  else
    accept_prep_staged_body<T, false, QL>(s, w, wk, e, u, cnt, ints_s[1], S, e2, px, py, pz, R, dJ, m, mc, lds, q,
                                          sc + 14, la, sg, jv, rx, ry, rz, sc[11], sc[12], sc[13]);
}

static hipError_t accept_launch(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc,
                                const double* unif, int32_t* accept_count, int S, hipStream_t st) {
  if (s.nu > kBigMaxN || !w.wv) return hipErrorNotSupported;
  const dim3 grid(w.Wk), blk(256);
  if (s.bf16()) hipLaunchKernelGGL(accept_kernel<bf16s>, grid, blk, 0, st, s, w, e, acc, unif, accept_count, S);
  else if (s.f32()) hipLaunchKernelGGL(accept_kernel<float>, grid, blk, 0, st, s, w, e, acc, unif, accept_count, S);
  else hipLaunchKernelGGL(accept_kernel<double>, grid, blk, 0, st, s, w, e, acc, unif, accept_count, S);
  return hipGetLastError();
}

hipError_t launch_accept(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc, hipStream_t st) {
  return accept_launch(s, w, e, acc, nullptr, nullptr, 0, st);
}

hipError_t launch_metropolis_accept(const SysDev& s, const WalkDev& w, int e, const double* unif,
                                    int32_t* accept_count, hipStream_t st) {
  return accept_launch(s, w, e, nullptr, unif, accept_count, propose_splits(s), st);
}

hipError_t launch_metropolis_accept_prep(const SysDev& s, const WalkDev& w, int e, const double* unif,
                                         int32_t* accept_count, int e2, const double* disp2, int since,
                                         hipStream_t st) {
  if (s.nu > kBigMaxN || !w.wv || s.Lp > kFuseMaxLp || e2 == e || s.LJ > 0) return hipErrorNotSupported;
  const int S = propose_splits(s);
  const dim3 grid(w.Wk), blk(256);
  const int mc = std::max(0, std::min(since, w.kb - 1));
  const StageLayout ly = stage_layout(s.nu, w.kb, mc);
  // the direct copies move 16-byte granules: every walker's V, D, S^{-1} and
  // positions start 16-byte aligned
  const bool aligned = ((uintptr_t)w.wv | (uintptr_t)w.wd | (uintptr_t)w.wS) % 16 == 0 &&
                       ((long)w.kb * s.nu) % 2 == 0 && w.kb % 2 == 0;
  if (s.nu <= kStageMaxN && s.N <= kStageMaxNe && s.n_nuc <= kStageMaxNuc && S > 0 && S <= kStageMaxSplits &&
      aligned &&
      ly.total <= kStageMaxLds) {
    const int QL = (s.L + 255) / 256;
#define QMC_STAGED(T, Q) hipLaunchKernelGGL((accept_prep_staged_kernel<T, Q>), grid, blk, ly.total, st, s, w, e, \
                                            unif, accept_count, S, e2, disp2, mc)
#define QMC_STAGED_QL(T)                                                                                   \
  if (QL <= 1) QMC_STAGED(T, 1);                                                                           \
  else if (QL == 2) QMC_STAGED(T, 2);                                                                      \
  else if (QL == 3) QMC_STAGED(T, 3);                                                                      \
  else QMC_STAGED(T, 4);
    if (s.bf16()) { QMC_STAGED_QL(bf16s) }
    else if (s.f32()) { QMC_STAGED_QL(float) }
    else { QMC_STAGED_QL(double) }
#undef QMC_STAGED_QL
#undef QMC_STAGED
    return hipGetLastError();
  }
  if (s.bf16())
    hipLaunchKernelGGL(accept_prep_kernel<bf16s>, grid, blk, 0, st, s, w, e, unif, accept_count, S, e2, disp2);
  else if (s.f32())
    hipLaunchKernelGGL(accept_prep_kernel<float>, grid, blk, 0, st, s, w, e, unif, accept_count, S, e2, disp2);
  else
    hipLaunchKernelGGL(accept_prep_kernel<double>, grid, blk, 0, st, s, w, e, unif, accept_count, S, e2, disp2);
  return hipGetLastError();
}

// After a refresh LU: log|Psi| = log|det W| + J, sign from the LU.
__global__ void refresh_finish_kernel(WalkDev w, int32_t* __restrict__ status) {
  const int wk = blockIdx.x * blockDim.x + threadIdx.x;
  if (wk >= w.Wk) return;
  const int sing = w.singular[wk];
  w.logabs[wk] = sing ? -__builtin_inf() : w.logdet[wk] + w.J[wk];
  w.sign[wk] = w.detsign[wk];
  w.wm[wk] = 0;
  if (status) status[wk] = sing ? 1 : 0;
}

// W^{-1} of every walker from the refresh inverse A0 and the delayed updates
// (state read-out and the drift check before a refresh).  up: A0 - V^T S^{-1} (D A0);
// down: A0 - (D A0^T)^T S^{-T} V, with V, D [m][n] the buffered rows.  Three
// passes over one workgroup per walker, through `scratch` ([Wk][2][kb][n]):
//   G = D A0 (up) or D A0^T (down)                      [m][n]
//   H = S^{-1} G (up) or S^{-T} V (down)               [m][n]
//   X = A0 - V^T H (up) or A0 - G^T H (down)            [n][n]
__global__ void __launch_bounds__(256)
materialize_inverse_kernel(SysDev s, WalkDev w, int down, double* __restrict__ scratch, double* __restrict__ dst) {
  const int wk = blockIdx.x, tid = threadIdx.x;
  const int n = s.nu, kb = w.kb, m = w.wm[wk];
  const double* A0 = w.A + (long)wk * n * n;
  const double* D = w.wd + (long)wk * kb * n;
  const double* V = w.wv + (long)wk * kb * n;
  const double* Si = w.wS + (long)wk * kb * kb;
  double* G = scratch + (long)wk * 2 * kb * n;
  double* H = G + (long)kb * n;
  double* out = dst + (long)wk * n * n;
  for (int idx = tid; idx < m * n; idx += blockDim.x) {
    const int l = idx / n, j = idx % n;
    double g = 0.0;
    if (!down) for (int i = 0; i < n; ++i) g += D[(long)l * n + i] * A0[(long)i * n + j];
    else for (int i = 0; i < n; ++i) g += D[(long)l * n + i] * A0[(long)j * n + i];
    G[idx] = g;
  }
  __syncthreads();
  for (int idx = tid; idx < m * n; idx += blockDim.x) {
    const int k = idx / n, j = idx % n;
    double h = 0.0;
    if (!down) for (int l = 0; l < m; ++l) h += Si[k * kb + l] * G[(long)l * n + j];
    else for (int l = 0; l < m; ++l) h += Si[l * kb + k] * V[(long)l * n + j];
    H[idx] = h;
  }
  __syncthreads();
  const double* Lf = down ? G : V;   // left factor, read as its transpose
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    double c = 0.0;
    for (int k = 0; k < m; ++k) c += Lf[(long)k * n + i] * H[(long)k * n + j];
    out[idx] = A0[idx] - c;
  }
}

hipError_t launch_materialize_inverse(const SysDev& s, const WalkDev& w, bool down, double* scratch, double* dst,
                                      hipStream_t st) {
  hipLaunchKernelGGL(materialize_inverse_kernel, dim3(w.Wk), dim3(256), 0, st, s, w, down ? 1 : 0, scratch, dst);
  return hipGetLastError();
}

// Residual of the inverse a refresh replaces: with P = W X (X the inverse
// before the refresh), res[w] = max_ij |P_ij - delta_ij|; a walker whose
// refresh found W non-singular (status 0) gets status 3 when the residual
// exceeds tol (or is not a number).  One workgroup per walker.
__global__ void __launch_bounds__(256)
refresh_residual_kernel(const double* __restrict__ Pm, int n, int Wk, double tol, double* __restrict__ res,
                        int32_t* __restrict__ status) {
  __shared__ double red[4];
  const int wk = blockIdx.x, tid = threadIdx.x;
  const double* p = Pm + (long)wk * n * n;
  double mx = 0.0;
  bool bad = false;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const double v = fabs(p[idx] - ((idx / n == idx % n) ? 1.0 : 0.0));
    if (!(v <= mx)) { if (v != v) bad = true; else mx = v; }
  }
  for (int o = 32; o > 0; o >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, o, 64));
    bad = bad || __shfl_xor((int)bad, o, 64);
  }
  if ((tid & 63) == 0) red[tid >> 6] = bad ? __builtin_nan("") : mx;
  __syncthreads();
  if (tid == 0) {
    double m = 0.0;
    bool nan = false;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      if (red[k] != red[k]) nan = true;
      else m = fmax(m, red[k]);
    }
    const double r = nan ? __builtin_nan("") : m;
    res[wk] = r;
    if (status && status[wk] == 0 && !(r <= tol)) status[wk] = 3;
  }
}

hipError_t launch_refresh_residual(const double* Pm, int n, int Wk, double tol, double* res, int32_t* status,
                                   hipStream_t st) {
  hipLaunchKernelGGL(refresh_residual_kernel, dim3(Wk), dim3(256), 0, st, Pm, n, Wk, tol, res, status);
  return hipGetLastError();
}

hipError_t launch_refresh_finish(const SysDev& s, const WalkDev& w, int32_t* status, hipStream_t st) {
  (void)s;
  hipLaunchKernelGGL(refresh_finish_kernel, dim3((w.Wk + 255) / 256), dim3(256), 0, st, w, status);
  return hipGetLastError();
}

}  // namespace qmc
