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

#include "move_staged.h"
#include <algorithm>

namespace qmc {

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
//   w'_j = sum over the kept mu of psi_mu(r') PT[wk][mu][i0 + j],  j < n_up,
// one contiguous column of the rows the move streams per kept basis function
// (for an up move the down electrons' rows and the unpaired orbitals; the
// skipped ones change the ratio by at most kScreenTol, see screen_list_body).
// One workgroup per walker: wave v takes kept functions v, v + 4, ..., four at
// a time, lane l the rows l, l + 64, ...; the waves' partial rows are added in
// a fixed order through LDS, then the ratio sum_j w'_j c_j.  The ratio goes to
// the first of the walker's S partial slots (the others are zeroed), which the
// accept and finalize kernels sum as usual.
// ---------------------------------------------------------------------------
template <int NB>
__global__ void __launch_bounds__(256) propose_screened_kernel(SysDev s, WalkDev w, int e, int S) {
  screened_rows_walker<NB>(s, w, blockIdx.x, e, S);
}

template <int IPB>
__global__ void __launch_bounds__(256) propose_screened_blk_kernel(SysDev s, WalkDev w, int e, int S, int FB) {
  extern __shared__ __align__(16) char lds[];
  screened_stream_walker<IPB>(s, w, blockIdx.x, e, S, FB, lds);
}

// Column maxima of the P halves (bit 0: up rows, bit 1: down rows):
// cmax[w][h][mu] = max over the rows i of half h of |P[w][i][mu]|.
// One workgroup per (walker, half), columns in passes of 128 CC: each lane
// takes the column pairs 2 lane + 128 c (16-byte loads), wave v the rows v,
// v + 4, ..., four rows at a time (4 CC independent loads in flight per
// lane), and the four waves' maxima meet in LDS (a maximum does not depend on
// the order, so any split gives the same values).
template <int CC>
__global__ void __launch_bounds__(256) screen_colmax_kernel(SysDev s, WalkDev w, int halves) {
  __shared__ double part[4][128 * CC];
  const int wk = blockIdx.x, h = blockIdx.y;
  if (!((halves >> h) & 1)) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int i0 = h == 0 ? 0 : s.nu, n = h == 0 ? s.nu : s.nd, Lp = s.Lp;   // Lp even
  const double* P = (const double*)w.P + ((long)wk * s.N + i0) * Lp;
  double* out = w.cmax + ((long)wk * 2 + h) * Lp;
  for (int c0 = 0; c0 < Lp; c0 += 128 * CC) {
    double2 m[CC];
#pragma unroll
    for (int c = 0; c < CC; ++c) m[c] = double2{0.0, 0.0};
    for (int i = wave; i < n; i += 16) {
      double2 v[4][CC];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const bool ok = i + 4 * u < n;
        const double* row = P + (long)(i + 4 * u) * Lp + c0;
#pragma unroll
        for (int c = 0; c < CC; ++c) {
          const int mu = 2 * lane + 128 * c;
          v[u][c] = ok && c0 + mu < Lp ? load16_nt<double2>(row + mu) : double2{0.0, 0.0};
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int c = 0; c < CC; ++c) {
          m[c].x = fmax(m[c].x, fabs(v[u][c].x));
          m[c].y = fmax(m[c].y, fabs(v[u][c].y));
        }
    }
    __syncthreads();   // the previous pass's maxima are written out
#pragma unroll
    for (int c = 0; c < CC; ++c) {
      part[wave][2 * lane + 128 * c] = m[c].x;
      part[wave][2 * lane + 128 * c + 1] = m[c].y;
    }
    __syncthreads();
    for (int mu = tid; mu < 128 * CC && c0 + mu < Lp; mu += blockDim.x) {
      double m = fmax(fmax(part[0][mu], part[1][mu]), fmax(part[2][mu], part[3][mu]));
      if (h == 1)   // an up move also streams the unpaired orbitals' values
        for (int l = 0; l < s.nk; ++l) m = fmax(m, fabs(s.Uph[(long)l * Lp + c0 + mu]));
      out[c0 + mu] = m;
    }
  }
}

// PT[w][mu][N + l] = U[mu][l] for every walker (constant: written once)
__global__ void __launch_bounds__(256) pt_unpaired_kernel(SysDev s, WalkDev w) {
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per = (long)s.Lp * s.nk;
  if (t >= per * w.Wk) return;
  const long wk = t / per, q = t % per, mu = q / s.nk, l = q % s.nk;
  w.PT[(wk * s.Lp + mu) * s.pt_ld() + s.N + l] = s.Uph[l * s.Lp + mu];
}

hipError_t launch_pt_unpaired(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (s.nk == 0) return hipSuccess;
  if (!w.PT || !s.Uph) return hipErrorInvalidValue;
  const long n = (long)s.Lp * s.nk * w.Wk;
  hipLaunchKernelGGL(pt_unpaired_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, w);
  return hipGetLastError();
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
  if (s.Lp % 2) return hipErrorInvalidValue;
  const dim3 grid(w.Wk, 2), blk(256);
  switch (std::min(8, (s.Lp + 127) / 128)) {
    case 1: hipLaunchKernelGGL(screen_colmax_kernel<1>, grid, blk, 0, st, s, w, halves); break;
    case 2: hipLaunchKernelGGL(screen_colmax_kernel<2>, grid, blk, 0, st, s, w, halves); break;
    case 3: hipLaunchKernelGGL(screen_colmax_kernel<3>, grid, blk, 0, st, s, w, halves); break;
    case 4: hipLaunchKernelGGL(screen_colmax_kernel<4>, grid, blk, 0, st, s, w, halves); break;
    case 5: hipLaunchKernelGGL(screen_colmax_kernel<5>, grid, blk, 0, st, s, w, halves); break;
    case 6: hipLaunchKernelGGL(screen_colmax_kernel<6>, grid, blk, 0, st, s, w, halves); break;
    case 7: hipLaunchKernelGGL(screen_colmax_kernel<7>, grid, blk, 0, st, s, w, halves); break;
    default: hipLaunchKernelGGL(screen_colmax_kernel<8>, grid, blk, 0, st, s, w, halves); break;
  }
  return hipGetLastError();
}

size_t screened_stream_lds(const SysDev& s, const WalkDev& w, int e) {
  int IPB = 0, FB = 0;
  size_t lds = 0;
  return screened_blk_config(s, w, e, IPB, FB, lds) ? lds : 0;
}

hipError_t launch_propose_screened(const SysDev& s, const WalkDev& w, int e, double* ratio, bool finalize,
                                   hipStream_t st, hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (!w.PT || !w.muk) return hipErrorInvalidValue;
  const int n = e < s.nu ? s.nd + s.nk : s.nu;   // rows streamed (= n_up)
  const int S = propose_splits(s);
  const dim3 grid(w.Wk), blk(256);
  int IPB, FB;
  size_t lds;
  if (screened_blk_config(s, w, e, IPB, FB, lds)) {
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

template <typename T, int QL>
__global__ void __launch_bounds__(256)
accept_prep_staged_kernel(SysDev s, WalkDev w, int e, const double* __restrict__ unif,
                          int32_t* __restrict__ accept_count, int S, int e2, const double* __restrict__ disp2,
                          int mc) {
  extern __shared__ __align__(16) char lds[];
  accept_prep_staged_phase<T, QL>(s, w, blockIdx.x, e, unif, accept_count, S, e2, disp2, mc, mc, lds);
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
