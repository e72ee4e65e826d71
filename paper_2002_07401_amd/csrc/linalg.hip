// FP64 log-determinant, sign and inverse of the geminal matrix of every walker.
//
// det W gives the AGP determinant part (eq:wfAGPs); W^{-1} supplies the
// cofactors of the local-energy derivatives and the Sherman-Morrison moves.
// Near a nodal surface W^{-1} diverges (the inverse of the pairing matrix
// behaves like 1/Pf, finite-variance reweighting subsection), which is why this
// step stays in FP64 in every precision mode.
//
// Method: in-place Gauss-Jordan elimination with partial (row) pivoting, one
// workgroup per walker: rows in registers for n <= kLuRowMax, else the whole
// matrix resident in LDS (n <= kLuMaxN).  The pivot is the largest |entry| of
// the column.
//   log|det| = sum_k log|pivot_k|,  sign = prod_k sign(pivot_k) * (-1)^{#swaps}
// After elimination the row interchanges are undone as column interchanges in
// reverse order, leaving W^{-1}.  A zero pivot marks the walker singular.
#include "internal.h"

namespace qmc {

// One matrix per workgroup: W (n x n) -> A = W^{-1}, log|det W| and sign in
// *logdet, *detsign (singular: *singular = 1).  smem holds n (n+1) + 2n doubles.
__device__ void gj_lds_body(const double* __restrict__ W, double* __restrict__ A, double* __restrict__ logdet,
                            double* __restrict__ detsign, int* __restrict__ singular, int n, double* smem) {
  const int ld = n + 1;
  double* M = smem;                 // n x ld
  double* rk = M + (long)n * ld;    // scaled pivot row
  double* ck = rk + n;              // pivot column before the step
  __shared__ int perm[kLuMaxN];
  __shared__ int piv_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

  for (int idx = tid; idx < n * n; idx += blockDim.x) M[(idx / n) * ld + (idx % n)] = W[idx];

  // fixed thread -> (column jc, row group g) map for the elimination update
  const int G = blockDim.x / n, jc = tid % n, g = tid / n;
  double lsum = 0.0, sg = 1.0;
  int sing = 0;
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    if (wave == 0) {
      double best = -1.0;
      int bi = n;
      for (int i = k + lane; i < n; i += 64) {
        const double v = fabs(M[i * ld + k]);
        if (v > best) { best = v; bi = i; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, 64);
        const int oi = __shfl_xor(bi, o, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (lane == 0) { piv_s = bi; perm[k] = bi; }
    }
    __syncthreads();
    const int p = piv_s;
    if (p != k) {
      for (int j = tid; j < n; j += blockDim.x) {
        const double t = M[k * ld + j];
        M[k * ld + j] = M[p * ld + j];
        M[p * ld + j] = t;
      }
      sg = -sg;
    }
    __syncthreads();
    const double piv = M[k * ld + k];
    if (!(piv != 0.0)) { sing = 1; break; }   // uniform across the block
    lsum += log(fabs(piv));
    if (piv < 0.0) sg = -sg;
    const double inv = 1.0 / piv;
    for (int j = tid; j < n; j += blockDim.x) {
      rk[j] = (j == k) ? inv : M[k * ld + j] * inv;
      ck[j] = M[j * ld + k];
    }
    __syncthreads();
    if (g < G) {
      const double rj = rk[jc];
      for (int i = g; i < n; i += G) {
        double v;
        if (i == k) v = rj;
        else if (jc == k) v = -ck[i] * rk[k];
        else v = M[i * ld + jc] - ck[i] * rj;
        M[i * ld + jc] = v;
      }
    }
  }
  __syncthreads();
  if (!sing) {
    for (int k = n - 1; k >= 0; --k) {
      const int p = perm[k];
      if (p != k) {
        for (int i = tid; i < n; i += blockDim.x) {
          const double t = M[i * ld + k];
          M[i * ld + k] = M[i * ld + p];
          M[i * ld + p] = t;
        }
      }
      __syncthreads();
    }
  }
  const double nanv = __longlong_as_double(0x7ff8000000000000LL);
  for (int idx = tid; idx < n * n; idx += blockDim.x)
    A[idx] = sing ? nanv : M[(idx / n) * ld + (idx % n)];
  if (tid == 0) {
    *logdet = sing ? -__builtin_inf() : lsum;
    *detsign = sing ? 0.0 : sg;
    *singular = sing;
  }
}

__global__ void __launch_bounds__(256)
gj_inverse_kernel(const double* __restrict__ Wg, double* __restrict__ Ag, double* __restrict__ logdet,
                  double* __restrict__ detsign, int* __restrict__ singular, int n, long w_bs, long a_bs) {
  extern __shared__ double smem[];
  const long b = blockIdx.x;
  gj_lds_body(Wg + b * w_bs, Ag + b * a_bs, logdet + b, detsign + b, singular + b, n, smem);
}

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

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
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

hipError_t launch_lu_inverse_lds(const SysDev& s, const WalkDev& w, hipStream_t st);

hipError_t launch_lu_inverse(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu;
  if (n > kLuMaxN) return hipErrorNotSupported;
  if (n > kLuRowMax) return launch_lu_inverse_lds(s, w, st);
  const long wbs = (long)s.nu * s.nd, abs_ = (long)s.nd * s.nu;
  const dim3 blk(n > 64 ? 128 : 64);
  switch ((n + 7) >> 3) {
#define QMC_LU_ROW(C)                                                                                   \
    case C:                                                                                             \
      hipLaunchKernelGGL(gj_inverse_row_kernel<8 * C>, dim3(w.Wk), blk, 0, st, w.W, w.A, w.logdet,      \
                         w.detsign, w.singular, n, wbs, abs_);                                          \
      break;
    QMC_LU_ROW(1) QMC_LU_ROW(2) QMC_LU_ROW(3) QMC_LU_ROW(4) QMC_LU_ROW(5) QMC_LU_ROW(6)
    QMC_LU_ROW(7) QMC_LU_ROW(8) QMC_LU_ROW(9) QMC_LU_ROW(10) QMC_LU_ROW(11) QMC_LU_ROW(12)
#undef QMC_LU_ROW
    default: return hipErrorNotSupported;
  }
  return hipGetLastError();
}

static size_t lu_lds_bytes(int n) { return ((size_t)n * (n + 1) + 2 * (size_t)n) * sizeof(double); }

// Raises the LDS limit of the LDS variant for an n x n problem; called once at
// system creation so that no launch (possibly under graph capture) needs it.
hipError_t prepare_lu(int n) {
  if (n <= kLuRowMax || lu_lds_bytes(n) <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void*)gj_inverse_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)lu_lds_bytes(n));
}

// LDS variant with physical row swaps, for kLuRowMax < n <= kLuMaxN.
hipError_t launch_lu_inverse_lds(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu;
  if (n > kLuMaxN) return hipErrorNotSupported;
  hipLaunchKernelGGL(gj_inverse_kernel, dim3(w.Wk), dim3(256), lu_lds_bytes(n), st, w.W, w.A, w.logdet,
                     w.detsign, w.singular, n, (long)s.nu * s.nd, (long)s.nd * s.nu);
  return hipGetLastError();
}

}  // namespace qmc
