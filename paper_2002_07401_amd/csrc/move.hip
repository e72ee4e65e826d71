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
#include "move_dev.h"
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

// grid (S, Wk): block (sb, wk) handles rows [sb*R, (sb+1)*R) of walker wk, R = s.prop_rows().
template <typename T, int NC>
__global__ void __launch_bounds__(256) propose_rows_kernel(SysDev s, WalkDev w, int e) {
  rows_body<T, NC>(s, w, blockIdx.y, blockIdx.x, gridDim.x, e, s.prop_rows());
}

template <typename T, bool DRIFT>
__global__ void __launch_bounds__(256) propose_rows_generic_kernel(SysDev s, WalkDev w, int e) {
  rows_generic_body<T, DRIFT>(s, w, blockIdx.y, blockIdx.x, gridDim.x, e, s.prop_rows());
}

template <typename T, int QMAX, bool UP>
__global__ void __launch_bounds__(256)
accept_kernel(SysDev s, WalkDev w, int e, const uint8_t* __restrict__ acc_in,
              const double* __restrict__ unif, int32_t* __restrict__ accept_count, int S) {
  const int wk = blockIdx.x;
  accept_body<T, QMAX, UP>(s, w, wk, e, unif ? 1 : 0, acc_in ? acc_in + wk : nullptr, unif ? unif[wk] : 0.0,
                           accept_count ? accept_count + wk : nullptr, S);
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

hipError_t launch_propose_rows(const SysDev& s, const WalkDev& w, int e, double* ratio,
                               double* drift_new, bool finalize, hipStream_t st) {
  const bool drift = drift_new != nullptr;
  const int S = propose_splits(s);
  const dim3 grid(S, w.Wk);
  const int store = s.store();
  hipError_t err;
  const int vn = store == 0 ? 2 : (store == 1 ? 4 : 8);   // elements per 16-byte load
  const int chunks = (s.Lp + 64 * vn - 1) / (64 * vn);
#define QMC_GEN(D)                                                                                         \
  if (store == 2) hipLaunchKernelGGL((propose_rows_generic_kernel<bf16s, D>), grid, dim3(256), 0, st, s, w, e); \
  else if (store == 1) hipLaunchKernelGGL((propose_rows_generic_kernel<float, D>), grid, dim3(256), 0, st, s, w, e); \
  else hipLaunchKernelGGL((propose_rows_generic_kernel<double, D>), grid, dim3(256), 0, st, s, w, e);
  if (drift) {
    QMC_GEN(true)
  } else if (chunks <= 8) {
#define QMC_ROWS(T, NC) \
    case NC: hipLaunchKernelGGL((propose_rows_kernel<T, NC>), grid, dim3(256), 0, st, s, w, e); break;
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

template <typename T>
static hipError_t accept_launch_t(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc,
                                  const double* unif, int32_t* accept_count, int S, hipStream_t st) {
  const int n = s.nu;
  const int G = 256 / n, Q = (n + G - 1) / G;
#define QMC_ACC(QM)                                                                                      \
  if (e < s.nu)                                                                                          \
    hipLaunchKernelGGL((accept_kernel<T, QM, true>), dim3(w.Wk), dim3(256), 0, st, s, w, e, acc, unif,     \
                       accept_count, S);                                                                 \
  else                                                                                                   \
    hipLaunchKernelGGL((accept_kernel<T, QM, false>), dim3(w.Wk), dim3(256), 0, st, s, w, e, acc, unif,    \
                       accept_count, S)
  if (Q <= 4) { QMC_ACC(4); }
  else if (Q <= 8) { QMC_ACC(8); }
  else if (Q <= 16) { QMC_ACC(16); }
  else if (Q <= 32) { QMC_ACC(32); }
  else { QMC_ACC(64); }
#undef QMC_ACC
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sherman-Morrison for kLuMaxN < n <= kBigMaxN, in two passes over A.
// Pass 1 (grid (ceil(n/64), Wk)): decision, delta, and 64 entries per block of
//   up:   coef[c] = (delta^T A)[c] / R,  save = A[:, e]   (block 0)
//   down: coef[j] = (A delta)[j] / R,    save = A[e, :]   (block 0)
// Pass 2: A -= save coef^T (up) or coef save^T (down), the W row/column, the
// basis row and the bookkeeping (block 0).  Same arithmetic as accept_body.
// ---------------------------------------------------------------------------
template <bool UP>
__global__ void __launch_bounds__(256)
accept_big_coef_kernel(SysDev s, WalkDev w, int e, const uint8_t* __restrict__ acc_in,
                       const double* __restrict__ unif, int S) {
  __shared__ double delta[kBigMaxN];
  __shared__ double part[4][64];
  const int wk = blockIdx.y, x0 = blockIdx.x * 64;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double R, ratio;
  if (S > 0) {
    R = 0.0;
    for (int k = 0; k < S; ++k) R += w.rdet_part[(long)wk * S + k];
    ratio = R * exp(w.dJ[wk]);
  } else {
    R = w.rdet[wk];
    ratio = w.ratio[wk];
  }
  const bool acc = unif ? (unif[wk] < ratio * ratio) : (acc_in[wk] != 0);
  if (blockIdx.x == 0 && tid == 0) {
    if (S > 0) { w.rdet[wk] = R; w.ratio[wk] = ratio; }
    w.acc[wk] = acc ? 1 : 0;
  }
  if (!acc) return;
  const int n = s.nu, ed = e - s.nu;
  const double invR = 1.0 / R;
  const double* Aw = w.A + (long)wk * n * n;
  const double* Ww = w.W + (long)wk * n * n;
  const double* wn = w.w_new + (long)wk * n;
  double* coef = w.smv + (long)wk * 2 * n;
  double* save = coef + n;
  for (int j = tid; j < n; j += 256) delta[j] = UP ? wn[j] - Ww[(long)e * n + j] : wn[j] - Ww[(long)j * n + ed];
  if (blockIdx.x == 0)
    for (int j = tid; j < n; j += 256) save[j] = UP ? Aw[(long)j * n + e] : Aw[(long)ed * n + j];
  __syncthreads();
  if constexpr (UP) {
    const int c = x0 + lane;
    double t = 0.0;
    if (c < n)
      for (int j = wave; j < n; j += 4) t += delta[j] * Aw[(long)j * n + c];
    part[wave][lane] = t;
    __syncthreads();
    if (tid < 64 && c < n) coef[c] = (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]) * invR;
  } else {
    double xv[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) {
      const int j = x0 + wave * 16 + m;
      double t = 0.0;
      if (j < n)
        for (int i = lane; i < n; i += 64) t += Aw[(long)j * n + i] * delta[i];
      xv[m] = t;
    }
    const double tot = wave_multi_sum16(xv, lane);
    const int j = x0 + wave * 16 + (lane >> 2);
    if ((lane & 3) == 0 && j < n) coef[j] = tot * invR;
  }
}

template <typename T, bool UP>
__global__ void __launch_bounds__(256)
accept_big_update_kernel(SysDev s, WalkDev w, int e, int32_t* __restrict__ accept_count) {
  const int wk = blockIdx.y;
  if (!w.acc[wk]) return;
  const int n = s.nu, ed = e - s.nu;
  double* Aw = w.A + (long)wk * n * n;
  const double* coef = w.smv + (long)wk * 2 * n;
  const double* save = coef + n;
  const long nn = (long)n * n;
  for (long idx = (long)blockIdx.x * 256 + threadIdx.x; idx < nn; idx += (long)gridDim.x * 256) {
    const int j = (int)(idx / n), c = (int)(idx % n);
    Aw[idx] = UP ? Aw[idx] - save[j] * coef[c] : Aw[idx] - coef[j] * save[c];
  }
  if (blockIdx.x != 0) return;
  const int tid = threadIdx.x;
  double* Ww = w.W + (long)wk * n * n;
  const double* wn = w.w_new + (long)wk * n;
  for (int j = tid; j < n; j += 256) {
    if (UP) Ww[(long)e * n + j] = wn[j];
    else Ww[(long)j * n + ed] = wn[j];
  }
  T* prow = (T*)w.phi + ((long)wk * s.N + e) * s.Lp;
  const double* pn = w.psi_new + (long)wk * s.Lp;
  for (int mu = tid; mu < s.L; mu += 256) prow[mu] = (T)pn[mu];
  if (tid == 0) {
    const double R = w.rdet[wk];
    double* re = w.r + ((long)wk * s.N + e) * 3;
    re[0] = w.r_new[3 * wk]; re[1] = w.r_new[3 * wk + 1]; re[2] = w.r_new[3 * wk + 2];
    const double dJ = w.dJ[wk];
    w.logabs[wk] += log(fabs(R)) + dJ;
    if (R < 0.0) w.sign[wk] = -w.sign[wk];
    w.J[wk] += dJ;
    if (accept_count) accept_count[wk] += 1;
  }
}

template <typename T>
static hipError_t accept_big_t(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc, const double* unif,
                               int32_t* accept_count, int S, hipStream_t st) {
  const int n = s.nu;
  if (n > kBigMaxN || !w.smv) return hipErrorNotSupported;
  const dim3 g1((n + 63) / 64, w.Wk), g2((unsigned)std::min<long>(((long)n * n + 1023) / 1024, 256), w.Wk);
  if (e < s.nu) {
    hipLaunchKernelGGL(accept_big_coef_kernel<true>, g1, dim3(256), 0, st, s, w, e, acc, unif, S);
    hipLaunchKernelGGL((accept_big_update_kernel<T, true>), g2, dim3(256), 0, st, s, w, e, accept_count);
  } else {
    hipLaunchKernelGGL(accept_big_coef_kernel<false>, g1, dim3(256), 0, st, s, w, e, acc, unif, S);
    hipLaunchKernelGGL((accept_big_update_kernel<T, false>), g2, dim3(256), 0, st, s, w, e, accept_count);
  }
  return hipGetLastError();
}

static hipError_t accept_launch(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc,
                                const double* unif, int32_t* accept_count, int S, hipStream_t st) {
  if (s.nu > kLuMaxN) {
    if (s.bf16()) return accept_big_t<bf16s>(s, w, e, acc, unif, accept_count, S, st);
    if (s.f32()) return accept_big_t<float>(s, w, e, acc, unif, accept_count, S, st);
    return accept_big_t<double>(s, w, e, acc, unif, accept_count, S, st);
  }
  if (s.bf16()) return accept_launch_t<bf16s>(s, w, e, acc, unif, accept_count, S, st);
  if (s.f32()) return accept_launch_t<float>(s, w, e, acc, unif, accept_count, S, st);
  return accept_launch_t<double>(s, w, e, acc, unif, accept_count, S, st);
}

hipError_t launch_accept(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc, hipStream_t st) {
  return accept_launch(s, w, e, acc, nullptr, nullptr, 0, st);
}

hipError_t launch_metropolis_accept(const SysDev& s, const WalkDev& w, int e, const double* unif,
                                    int32_t* accept_count, hipStream_t st) {
  return accept_launch(s, w, e, nullptr, unif, accept_count, propose_splits(s), st);
}

// After a refresh LU: log|Psi| = log|det W| + J, sign from the LU.
__global__ void refresh_finish_kernel(WalkDev w, int32_t* __restrict__ status) {
  const int wk = blockIdx.x * blockDim.x + threadIdx.x;
  if (wk >= w.Wk) return;
  const int sing = w.singular[wk];
  w.logabs[wk] = sing ? -__builtin_inf() : w.logdet[wk] + w.J[wk];
  w.sign[wk] = w.detsign[wk];
  if (status) status[wk] = sing ? 1 : 0;
}

hipError_t launch_refresh_finish(const SysDev& s, const WalkDev& w, int32_t* status, hipStream_t st) {
  (void)s;
  hipLaunchKernelGGL(refresh_finish_kernel, dim3((w.Wk + 255) / 256), dim3(256), 0, st, w, status);
  return hipGetLastError();
}

}  // namespace qmc
