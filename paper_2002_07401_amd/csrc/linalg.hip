// FP64 log-determinant, sign and inverse of the geminal matrix of every walker.
//
// det W gives the AGP determinant part (eq:wfAGPs); W^{-1} supplies the
// cofactors of the local-energy derivatives and the Sherman-Morrison moves.
// Near a nodal surface W^{-1} diverges (the inverse of the pairing matrix
// behaves like 1/Pf, finite-variance reweighting subsection), which is why this
// step stays in FP64 in every precision mode.
//
// Method: in-place Gauss-Jordan elimination with partial (row) pivoting: one
// workgroup per walker with the rows in registers for n <= kLuRowMax, else the
// blocked elimination below (panels in registers, updates in global memory).
// The pivot is the largest |entry| of the column.
//   log|det| = sum_k log|pivot_k|,  sign = prod_k sign(pivot_k) * (-1)^{#swaps}
// After elimination the row interchanges are undone as column interchanges in
// reverse order, leaving W^{-1}.  A zero pivot marks the walker singular.
#include "internal.h"

#include <type_traits>

namespace qmc {

// Row-per-thread variant (the default for n <= kLuRowMax).  The matrix is
// padded to NMAX = round_up(n, 8) with an identity block, which leaves the real
// block's elimination unchanged (padding rows are zero in real columns, real
// rows zero in padding columns).  Thread i keeps row i in registers as a
// rotating window: before step k, a[j] holds column (k + j) mod NMAX, so the
// pivot column is always a[0] and the update a[j] <- a[j+1] - g rk[j+1] shifts
// by one; after NMAX steps the window is back in place.
//
// Rows are never swapped: step k pivots on (p_k, k), p_k the unused row with
// the largest |T[p][k]| (compared on the top 44 mantissa bits, lowest row on
// ties).  A pivot row is left unscaled (its column-k entry set to 1) and
// divided by its own pivot once at the end; every later update is linear in
// the row, so this equals scaling at the pivot step.  In-place Gauss-Jordan on
// the pivots (p_k, k) leaves
//   W^{-1}[k][p_k'] = T[p_k][k'],   det W = sgn(p) prod_k pivot_k,
// sgn(p) the parity of k -> p_k.
struct GjRowShared {
  double rk[2][2][kLuRowMax];        // per parity, per wave: that wave's best row
  unsigned long long key[2][2];      // per parity, per wave: its pivot key
  int prow[kLuRowMax];
  int kof[kLuRowMax];
  double red_d[4];
  int red_i[4];
};

// Maximum of a 64-bit key over the wave, in every lane: within each row of 16
// lanes by register-to-register DPP moves (quad_perm [1,0,3,2], [2,3,0,1],
// row_ror:4, row_ror:8: every lane ends with its row's maximum), then over the
// four rows' lanes 0, 16, 32, 48 through scalar reads.  A maximum does not
// depend on the order, so this equals the butterfly over the whole wave; it
// needs no LDS round trip per stage (a Gauss-Jordan step was 7 % faster).
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp_u64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_mov_dpp((int)(unsigned)v, CTRL, 0xF, 0xF, false);
  const unsigned hi = __builtin_amdgcn_mov_dpp((int)(unsigned)(v >> 32), CTRL, 0xF, 0xF, false);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  unsigned long long u = dpp_u64<0xB1>(v);
  v = u > v ? u : v;
  u = dpp_u64<0x4E>(v);
  v = u > v ? u : v;
  u = dpp_u64<0x124>(v);
  v = u > v ? u : v;
  u = dpp_u64<0x128>(v);
  v = u > v ? u : v;
  unsigned long long m = 0ull;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const unsigned lo = __builtin_amdgcn_readlane((int)(unsigned)v, 16 * r);
    const unsigned hi = __builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 16 * r);
    const unsigned long long x = ((unsigned long long)hi << 32) | lo;
    m = x > m ? x : m;
  }
  return m;
}

template <int NMAX>
__device__ __forceinline__ void gj_row_body(const double* __restrict__ W, double* __restrict__ A, double* __restrict__ logdet,
                            double* __restrict__ detsign, int* __restrict__ singular, int n, GjRowShared& sm) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = (min((int)blockDim.x, NMAX) + 63) >> 6;   // waves holding rows
  const bool live = tid < NMAX, real = tid < n;
  double a[NMAX];
  if (real) {
    const double* row = W + (long)tid * n;
    if ((n & 1) == 0) {
#pragma unroll
      for (int j = 0; j < NMAX; j += 2) {
        if (j < n) {
          const double2 v = *reinterpret_cast<const double2*>(row + j);
          a[j] = v.x; a[j + 1] = v.y;
        } else {
          a[j] = 0.0; a[j + 1] = 0.0;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < NMAX; ++j) a[j] = j < n ? row[j] : 0.0;
    }
  } else {
#pragma unroll
    for (int j = 0; j < NMAX; ++j) a[j] = (j == tid) ? 1.0 : 0.0;
  }

  bool used = !live;
  double own_piv = 1.0;
  int own_k = tid;
  int sing = 0;
  for (int k = 0; k < NMAX; ++k) {
    const int b = k & 1;
    const double f = a[0];
    // Only real rows may pivot in the first n steps (whatever the values), so
    // real rows take steps 0..n-1 and every store below stays inside A.
    const bool elig = !used && (real || k >= n);
    const unsigned long long key =
        elig ? ((__double_as_longlong(fabs(f)) & ~0xFFull) | (unsigned long long)(255 - tid)) : 0ull;
    const unsigned long long wk = wave_max_u64(key);
    if (wave < nw) {
      if (key == wk && wk != 0ull) {
        double* dst = sm.rk[b][wave];
#pragma unroll
        for (int j = 0; j < NMAX; ++j) dst[j] = a[j];
      }
      if (lane == 0) sm.key[b][wave] = wk;
    }
    __syncthreads();
    unsigned long long best = sm.key[b][0];
    int ws = 0;
    if (nw > 1 && sm.key[b][1] > best) { best = sm.key[b][1]; ws = 1; }
    const double* rk = sm.rk[b][ws];
    const double piv = rk[0];
    if (!(piv != 0.0)) { sing = 1; break; }   // uniform across the block
    const int p = 255 - (int)(best & 0xFFull);
    const bool isp = tid == p;
    if (isp) { used = true; own_piv = piv; own_k = k; sm.prow[k] = tid; }
    const double g = isp ? 0.0 : f * (1.0 / piv);
#pragma unroll
    for (int j = 0; j < NMAX - 1; ++j) a[j] = fma(-g, rk[j + 1], a[j + 1]);
    a[NMAX - 1] = isp ? 1.0 : -g;
  }

  if (sing) {
    const double nanv = __longlong_as_double(0x7ff8000000000000LL);
    for (int idx = tid; idx < n * n; idx += blockDim.x) A[idx] = nanv;
    if (tid == 0) { *logdet = -__builtin_inf(); *detsign = 0.0; *singular = 1; }
    return;
  }
  if (live) sm.kof[tid] = own_k;
  __syncthreads();
  // log|det| = sum log|pivot|; sign from the pivots' signs and the parity of
  // the pivot permutation (inversions among real rows; padding rows are
  // pivoted last, in order).
  double ls = real ? log(fabs(own_piv)) : 0.0;
  int odd = 0;
  if (real) {
    odd = own_piv < 0.0;
    for (int i2 = tid + 1; i2 < n; ++i2) odd += sm.kof[i2] < own_k;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ls += __shfl_xor(ls, o, 64);
    odd += __shfl_xor(odd, o, 64);
  }
  if (lane == 0 && wave < 4) { sm.red_d[wave] = ls; sm.red_i[wave] = odd; }
  if (real) {
    const double inv = 1.0 / own_piv;
    double* out = A + (long)own_k * n;
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j < n) out[sm.prow[j]] = a[j] * inv;
  }
  __syncthreads();
  if (tid == 0) {
    double lsum = 0.0;
    int par = 0;
    for (int q = 0; q < nw; ++q) { lsum += sm.red_d[q]; par += sm.red_i[q]; }
    *logdet = lsum;
    *detsign = (par & 1) ? -1.0 : 1.0;
    *singular = 0;
  }
}

template <int NMAX>
__global__ void __launch_bounds__(128)
gj_inverse_row_kernel(const double* __restrict__ Wg, double* __restrict__ Ag, double* __restrict__ logdet,
                      double* __restrict__ detsign, int* __restrict__ singular, int n, long w_bs, long a_bs) {
  __shared__ GjRowShared sm;
  const long b = blockIdx.x;
  gj_row_body<NMAX>(Wg + b * w_bs, Ag + b * a_bs, logdet + b, detsign + b, singular + b, n, sm);
}

// Column-split variant for 64 < n <= 88 (NMAX = round_up(n, 8), two waves): wave w keeps columns [w H, w H + H) (H = NMAX / 2) of every row,
// lane l rows l and 64 + l.  Steps 0..H-1 pivot on wave 0's columns (its
// window of H columns rotates as in gj_row_body, the other wave's stays in
// place), steps H..2H-1 on wave 1's.  Each wave takes the pivot row's values
// in its own columns from lane p mod 64 of its own registers (readlane), so
// the row is never copied through LDS (that copy, 80 values written by one
// lane every step, was the row kernel's largest cost); only the pivot column
// crosses the waves, two values per lane.  Pivot choice, multipliers and
// updates are those of gj_row_body, so W^{-1} is bitwise the row kernel's;
// log|det| adds the same logarithms in another order.
struct GjSplitShared {
  double fcol[2][128];   // per parity: the pivot column's entries, row-indexed
  double piv[2];
  int p[2];
  int prow[kLuRowMax];
  int kof[kLuRowMax];
};

template <int NMAX>
__global__ void __launch_bounds__(128)
gj_split_kernel(const double* __restrict__ Wg, double* __restrict__ Ag, double* __restrict__ logdet,
                double* __restrict__ detsign, int* __restrict__ singular, int n, long w_bs, long a_bs) {
  static_assert(NMAX > 64 && NMAX <= 128 && NMAX % 8 == 0, "two waves, two rows per lane");
  constexpr int H = NMAX / 2;
  __shared__ GjSplitShared sm;
  const long bb = blockIdx.x;
  const double* W = Wg + bb * w_bs;
  double* A = Ag + bb * a_bs;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int r0 = lane, r1 = 64 + lane;
  const bool live1 = r1 < NMAX;
  const bool real0 = r0 < n, real1 = r1 < n;
  const int c0 = wave * H;
  double x0[H], x1[H];
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const int c = c0 + j;
    x0[j] = real0 ? (c < n ? W[(long)r0 * n + c] : 0.0) : (c == r0 ? 1.0 : 0.0);
    x1[j] = real1 ? (c < n ? W[(long)r1 * n + c] : 0.0) : (c == r1 ? 1.0 : 0.0);
  }
  bool used0 = false, used1 = !live1;
  double piv0 = 1.0, piv1 = 1.0;
  int k0 = r0, k1 = r1;
  int sing = 0;
  auto phase = [&](auto own_tag, int ph) {
    constexpr bool own = decltype(own_tag)::value;
    for (int kk = 0; kk < H; ++kk) {
      const int k = ph * H + kk, b = k & 1;
      if (own) {
        // pivot: the largest |entry| of column k among rows not yet pivoted
        // (real rows only in the first n steps), lowest row on ties
        const double f0 = x0[0], f1 = x1[0];
        const bool e0 = !used0 && (real0 || k >= n), e1 = !used1 && (real1 || k >= n);
        const unsigned long long q0 =
            e0 ? ((__double_as_longlong(fabs(f0)) & ~0xFFull) | (unsigned long long)(255 - r0)) : 0ull;
        const unsigned long long q1 =
            e1 ? ((__double_as_longlong(fabs(f1)) & ~0xFFull) | (unsigned long long)(255 - r1)) : 0ull;
        const unsigned long long wk = wave_max_u64(q0 > q1 ? q0 : q1);
        const int p = 255 - (int)(wk & 0xFFull);
        const int wl = p & 63;
        const double fp = p < 64 ? f0 : f1;   // uniform choice of register, lane wl's value below
        const double pv = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(fp), wl),
                                           __builtin_amdgcn_readlane(__double2loint(fp), wl));
        sm.fcol[b][lane] = f0;
        sm.fcol[b][64 + lane] = f1;
        if (lane == 0) {
          sm.piv[b] = wk != 0ull ? pv : 0.0;
          sm.p[b] = p;
          sm.prow[k] = p;
        }
      }
      __syncthreads();
      const double piv = sm.piv[b];
      if (!(piv != 0.0)) { sing = 1; return; }   // uniform across the block
      const int p = sm.p[b];
      const int wl = p & 63;
      const bool isp0 = r0 == p, isp1 = r1 == p;
      const double f0 = own ? x0[0] : sm.fcol[b][lane];
      const double f1 = own ? x1[0] : sm.fcol[b][64 + lane];
      if (isp0) { used0 = true; piv0 = piv; k0 = k; }
      if (isp1) { used1 = true; piv1 = piv; k1 = k; }
      const double g0 = isp0 ? 0.0 : f0 * (1.0 / piv);
      const double g1 = isp1 ? 0.0 : f1 * (1.0 / piv);
      const bool hi_row = p >= 64;
      // the pivot row's entries in this wave's columns (window order) from lane
      // wl, eight at a time, each used at once
#pragma unroll
      for (int c = 0; c < H; c += 8) {
        double pr[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = c + q + (own ? 1 : 0);
          double v = 0.0;
          if (j < H) {
            const double xs = hi_row ? x1[j] : x0[j];
            v = __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(xs), wl),
                                 __builtin_amdgcn_readlane(__double2loint(xs), wl));
          }
          pr[q] = v;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int j = c + q;
          if (own) {
            if (j < H - 1) {
              x0[j] = fma(-g0, pr[q], x0[j + 1]);
              x1[j] = fma(-g1, pr[q], x1[j + 1]);
            }
          } else if (j < H) {
            x0[j] = fma(-g0, pr[q], x0[j]);
            x1[j] = fma(-g1, pr[q], x1[j]);
          }
        }
      }
      if (own) {
        x0[H - 1] = isp0 ? 1.0 : -g0;
        x1[H - 1] = isp1 ? 1.0 : -g1;
      }
    }
  };
  if (wave == 0) {
    phase(std::true_type{}, 0);
    if (!sing) phase(std::false_type{}, 1);
  } else {
    phase(std::false_type{}, 0);
    if (!sing) phase(std::true_type{}, 1);
  }
  if (sing) {
    const double nanv = __longlong_as_double(0x7ff8000000000000LL);
    for (int idx = tid; idx < n * n; idx += blockDim.x) A[idx] = nanv;
    if (tid == 0) { logdet[bb] = -__builtin_inf(); detsign[bb] = 0.0; singular[bb] = 1; }
    return;
  }
  if (wave == 0) {
    sm.kof[r0] = k0;
    if (live1) sm.kof[r1] = k1;
  }
  __syncthreads();
  // log|det| and the sign as in gj_row_body (wave 0 holds every row once)
  double ls = 0.0;
  int odd = 0;
  if (wave == 0) {
    if (real0) {
      ls += log(fabs(piv0));
      odd += piv0 < 0.0;
      for (int i2 = r0 + 1; i2 < n; ++i2) odd += sm.kof[i2] < k0;
    }
    if (real1) {
      ls += log(fabs(piv1));
      odd += piv1 < 0.0;
      for (int i2 = r1 + 1; i2 < n; ++i2) odd += sm.kof[i2] < k1;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      ls += __shfl_xor(ls, o, 64);
      odd += __shfl_xor(odd, o, 64);
    }
  }
  if (real0) {
    const double inv = 1.0 / piv0;
    double* out = A + (long)k0 * n;
#pragma unroll
    for (int j = 0; j < H; ++j)
      if (c0 + j < n) out[sm.prow[c0 + j]] = x0[j] * inv;
  }
  if (real1) {
    const double inv = 1.0 / piv1;
    double* out = A + (long)k1 * n;
#pragma unroll
    for (int j = 0; j < H; ++j)
      if (c0 + j < n) out[sm.prow[c0 + j]] = x1[j] * inv;
  }
  if (tid == 0) {
    logdet[bb] = ls;
    detsign[bb] = (odd & 1) ? -1.0 : 1.0;
    singular[bb] = 0;
  }
}

static hipError_t launch_lu_inverse_big(const SysDev& s, const WalkDev& w, hipStream_t st);

hipError_t launch_lu_inverse(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu;
  if (n > kLuRowMax) return launch_lu_inverse_big(s, w, st);
  return launch_gj_inverse_n(w.Wk, n, w.W, w.A, w.logdet, w.detsign, w.singular, st);   // W is n_up x n_up
}

hipError_t launch_gj_inverse_n(int Wk, int n, const double* W, double* A, double* logdet, double* detsign,
                               int* singular, hipStream_t st) {
  if (n < 1 || n > kLuRowMax) return hipErrorNotSupported;
  const long wbs = (long)n * n, abs_ = wbs;
  const dim3 blk(n > 64 ? 128 : 64);
  if (n > 64 && n <= 88) {   // two waves, columns split between them (at 96, one wave per SIMD: the row kernel)
    switch ((n + 7) >> 3) {
#define QMC_LU_SPLIT(C)                                                                                 \
      case C:                                                                                           \
        hipLaunchKernelGGL(gj_split_kernel<8 * C>, dim3(Wk), blk, 0, st, W, A, logdet, detsign, singular, \
                           n, wbs, abs_);                                                               \
        break;
      QMC_LU_SPLIT(9) QMC_LU_SPLIT(10) QMC_LU_SPLIT(11)
#undef QMC_LU_SPLIT
      default: return hipErrorNotSupported;
    }
    return hipGetLastError();
  }
  switch ((n + 7) >> 3) {
#define QMC_LU_ROW(C)                                                                                   \
    case C:                                                                                             \
      hipLaunchKernelGGL(gj_inverse_row_kernel<8 * C>, dim3(Wk), blk, 0, st, W, A, logdet,              \
                         detsign, singular, n, wbs, abs_);                                              \
      break;
    QMC_LU_ROW(1) QMC_LU_ROW(2) QMC_LU_ROW(3) QMC_LU_ROW(4) QMC_LU_ROW(5) QMC_LU_ROW(6)
    QMC_LU_ROW(7) QMC_LU_ROW(8) QMC_LU_ROW(9) QMC_LU_ROW(10) QMC_LU_ROW(11) QMC_LU_ROW(12)
#undef QMC_LU_ROW
    default: return hipErrorNotSupported;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Blocked Gauss-Jordan for kLuRowMax < n <= kBigMaxN (matrix in global memory).
//
// T = [[W, 0], [0, I]] (np = n rounded up to 64; the identity block leaves the
// real block's elimination unchanged, as in the register kernel).  Panels of NB
// columns: the panel kernel runs NB in-place Gauss-Jordan steps restricted to
// the panel columns (rows in registers, the rotating window of gj_row_body,
// pivots chosen among rows not yet pivoted, real rows first), which equals
// applying the steps' elimination matrix E to the panel; E differs from the
// identity only in the columns of the panel's pivot rows P, and in-place
// Gauss-Jordan leaves exactly those columns of E in the panel.  The update
// kernel then applies E to every other column:
//   T[:, O] <- D T[:, O] + T'[:, C] T_old[P, O]      (D zeroes the rows P),
// a product with K = NB on the FP64 matrix cores.  The finish kernel writes W^{-1}[k][p_k'] = T[p_k][k']
// and log|det W| = sum log|pivot_k|, sign = sgn(p) prod sign(pivot_k).
// ---------------------------------------------------------------------------
__global__ void gj_big_init_kernel(const double* __restrict__ W, double* __restrict__ T, int* __restrict__ rowk,
                                   int* __restrict__ singular, int n, int np) {
  const long wk = blockIdx.y;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < (long)np * np) {
    const int i = (int)(idx / np), j = (int)(idx % np);
    T[wk * np * np + idx] = (i < n && j < n) ? W[wk * n * n + (long)i * n + j] : (i == j ? 1.0 : 0.0);
  }
  if (idx < np) rowk[wk * np + idx] = -1;
  if (idx == 0) singular[wk] = 0;
}

template <int NB>
__global__ void __launch_bounds__(NB == 64 ? 512 : 1024)
gj_panel_kernel(double* __restrict__ T, double* __restrict__ Tsave, int* __restrict__ rowk, int* __restrict__ prow,
                double* __restrict__ pivv, int* __restrict__ singular, int n, int np, int c0) {
  __shared__ double rk[2][16][NB];
  __shared__ unsigned long long key_s[2][16];
  __shared__ int pr_s[NB];
  const long wk = blockIdx.x;
  const int i = threadIdx.x, lane = i & 63, wave = i >> 6, nw = blockDim.x >> 6;
  if (singular[wk]) return;   // the same value for the whole block
  double* Tw = T + wk * np * np;
  int* rkw = rowk + wk * np;
  int my_k = rkw[i];
  double a[NB];
#pragma unroll
  for (int j = 0; j < NB; j += 2) {
    const double2 v = *reinterpret_cast<const double2*>(Tw + (long)i * np + c0 + j);
    a[j] = v.x; a[j + 1] = v.y;
  }
  double own_piv = 1.0;
  bool mine = false;
  int sing = 0;
  for (int kk = 0; kk < NB; ++kk) {
    const int step = c0 + kk, b = kk & 1;
    const double f = a[0];
    const bool elig = my_k < 0 && (i < n || step >= n);
    const unsigned long long key =
        elig ? ((__double_as_longlong(fabs(f)) & ~0x7FFull) | (unsigned long long)(2047 - i)) : 0ull;   // > 0
    const unsigned long long wmax = wave_max_u64(key);
    if (key == wmax && wmax != 0ull) {
#pragma unroll
      for (int j = 0; j < NB; ++j) rk[b][wave][j] = a[j];
    }
    if (lane == 0) key_s[b][wave] = wmax;
    __syncthreads();
    unsigned long long best = key_s[b][0];
    int ws = 0;
    for (int q = 1; q < nw; ++q)
      if (key_s[b][q] > best) { best = key_s[b][q]; ws = q; }
    const double* rr = rk[b][ws];
    const double piv = rr[0];
    if (!(piv != 0.0)) { sing = 1; break; }   // uniform across the block
    const int p = 2047 - (int)(best & 0x7FFull);
    const bool isp = i == p;
    if (isp) { my_k = step; own_piv = piv; mine = true; }
    if (i == 0) {
      pr_s[kk] = p;
      prow[wk * np + step] = p;
      pivv[wk * np + step] = piv;
    }
    const double g = isp ? 0.0 : f * (1.0 / piv);
#pragma unroll
    for (int j = 0; j < NB - 1; ++j) a[j] = fma(-g, rr[j + 1], a[j + 1]);
    a[NB - 1] = isp ? 1.0 : -g;
  }
  if (sing) {
    if (i == 0) singular[wk] = 1;
    return;
  }
  if (mine) {
    const double inv = 1.0 / own_piv;
#pragma unroll
    for (int j = 0; j < NB; ++j) a[j] *= inv;
  }
#pragma unroll
  for (int j = 0; j < NB; j += 2)
    *reinterpret_cast<double2*>(Tw + (long)i * np + c0 + j) = make_double2(a[j], a[j + 1]);
  rkw[i] = my_k;
  __syncthreads();
  // the panel's pivot rows outside the panel move to Tsave (the update's right
  // operand) and are cleared in T (the D of the update)
  double* Sw = Tsave + wk * NB * np;
  for (int kk = 0; kk < NB; ++kk) {
    double* src = Tw + (long)pr_s[kk] * np;
    for (int o = i; o < np; o += blockDim.x) {
      const bool in_panel = o >= c0 && o < c0 + NB;
      Sw[(long)kk * np + o] = in_panel ? 0.0 : src[o];
      if (!in_panel) src[o] = 0.0;
    }
  }
}

// T[:, O] += T[:, panel] Tsave[:, O] for the column ranges O left and right of
// the panel: batched FP64 MFMA products (the panel kernel has cleared the
// pivot rows of T[:, O]).  Walkers found singular are updated with whatever
// Tsave holds; their outputs are overwritten by the finish kernels.
static hipError_t gj_update_mfma(const WalkDev& w, int np, int c0, int NB, hipStream_t st) {
  for (int side = 0; side < 2; ++side) {
    const int o0 = side ? c0 + NB : 0, no = side ? np - c0 - NB : c0;
    if (no <= 0) continue;
    GemmArgs g = gemm_args(np, no, NB);
    g.A = w.T + c0; g.lda = np; g.a_bs = (long)np * np;
    g.B = w.Tsave + o0; g.ldb = np; g.b_bs = (long)NB * np;
    g.C = w.T + o0; g.ldc = np; g.c_bs = (long)np * np;
    g.batch = w.Wk;
    g.accumulate = 1;
    const hipError_t e = gemm_f64(g, false, false, true, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// A[k][m] = T[prow[k]][rowk[m]] for k, m < n (4 rows of A per block).
__global__ void __launch_bounds__(256)
gj_big_output_kernel(const double* __restrict__ T, const int* __restrict__ rowk, const int* __restrict__ prow,
                     const int* __restrict__ singular, double* __restrict__ A, int n, int np) {
  const long wk = blockIdx.y;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (k >= n) return;
  double* out = A + wk * n * n + (long)k * n;
  const double nanv = __longlong_as_double(0x7ff8000000000000LL);
  if (singular[wk]) {
    for (int m = lane; m < n; m += 64) out[m] = nanv;
    return;
  }
  const double* src = T + wk * np * np + (long)prow[wk * np + k] * np;
  const int* rk = rowk + wk * np;
  for (int m = lane; m < n; m += 64) out[m] = src[rk[m]];
}

// log|det W| = sum_k log|pivot_k|; sign = prod sign(pivot_k) * (-1)^{inversions of k -> p_k}.
__global__ void __launch_bounds__(1024)
gj_big_det_kernel(const int* __restrict__ rowk, const double* __restrict__ pivv, const int* __restrict__ singular,
                  double* __restrict__ logdet, double* __restrict__ detsign, int n, int np) {
  __shared__ double rd[16];
  __shared__ int ri[16];
  const long wk = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  if (singular[wk]) {
    if (tid == 0) { logdet[wk] = -__builtin_inf(); detsign[wk] = 0.0; }
    return;
  }
  const int* rk = rowk + wk * np;
  double ls = 0.0;
  int odd = 0;
  for (int k = tid; k < n; k += blockDim.x) {
    const double pv = pivv[wk * np + k];
    ls += log(fabs(pv));
    odd += pv < 0.0;
  }
  for (int i = tid; i < n; i += blockDim.x) {
    const int ki = rk[i];
    for (int i2 = i + 1; i2 < n; ++i2) odd += rk[i2] < ki;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    ls += __shfl_xor(ls, o, 64);
    odd += __shfl_xor(odd, o, 64);
  }
  if (lane == 0) { rd[wave] = ls; ri[wave] = odd; }
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    int par = 0;
    for (int q = 0; q < nw; ++q) { t += rd[q]; par += ri[q]; }
    logdet[wk] = t;
    detsign[wk] = (par & 1) ? -1.0 : 1.0;
  }
}

static hipError_t launch_lu_inverse_big(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu, np = s.np;
  if (n > kBigMaxN || np % 64 || !w.T) return hipErrorNotSupported;
  const long nn = (long)np * np;
  hipLaunchKernelGGL(gj_big_init_kernel, dim3((unsigned)((nn + 255) / 256), w.Wk), dim3(256), 0, st, w.W, w.T,
                     w.rowk, w.singular, n, np);
  const int NB = np <= 512 ? 64 : 32;
  for (int c0 = 0; c0 < np; c0 += NB) {
    if (NB == 64)
      hipLaunchKernelGGL(gj_panel_kernel<64>, dim3(w.Wk), dim3(np), 0, st, w.T, w.Tsave, w.rowk, w.prow, w.pivv,
                         w.singular, n, np, c0);
    else
      hipLaunchKernelGGL(gj_panel_kernel<32>, dim3(w.Wk), dim3(np), 0, st, w.T, w.Tsave, w.rowk, w.prow, w.pivv,
                         w.singular, n, np, c0);
    const hipError_t e = gj_update_mfma(w, np, c0, NB, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gj_big_output_kernel, dim3((n + 3) / 4, w.Wk), dim3(256), 0, st, w.T, w.rowk, w.prow,
                     w.singular, w.A, n, np);
  hipLaunchKernelGGL(gj_big_det_kernel, dim3(w.Wk), dim3(1024), 0, st, w.rowk, w.pivv, w.singular, w.logdet,
                     w.detsign, n, np);
  return hipGetLastError();
}

}  // namespace qmc
