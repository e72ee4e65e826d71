// FP64 log-determinant, sign and inverse of the geminal matrix of every walker.
//
// det W gives the AGP determinant part (eq:wfAGPs); W^{-1} supplies the
// cofactors of the local-energy derivatives and the Sherman-Morrison moves.
// Near a nodal surface W^{-1} diverges (the inverse of the pairing matrix
// behaves like 1/Pf, finite-variance reweighting subsection), which is why this
// step stays in FP64 in every precision mode.
//
// Method: in-place Gauss-Jordan elimination with partial (row) pivoting, the
// whole matrix resident in LDS (n <= 128), one workgroup per walker.  The pivot
// is the largest |entry| of the column (lowest row on ties).
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

// Register-resident variant (the default).  Thread t keeps column c = t % n of
// rows g, g + G, g + 2G, ... (g = t / n, G = blockDim / n) in registers.  Rows
// are never swapped: step k pivots in place on (p_k, k), p_k the unused row
// with the largest |T[p][k]| (lowest index on ties), with the same update as
// above.  In-place Gauss-Jordan on the pivots (p_k, k) leaves
//   W^{-1}[k][p_k'] = T[p_k][k']   and   det W = sgn(p) prod_k T_k[p_k][k],
// sgn(p) the parity of the permutation k -> p_k.
template <int QMAX>
__device__ void gj_reg_body(const double* __restrict__ W, double* __restrict__ A, double* __restrict__ logdet,
                            double* __restrict__ detsign, int* __restrict__ singular, int n) {
  __shared__ double rk[kLuMaxN];
  __shared__ double ck[kLuMaxN];
  __shared__ int used[kLuMaxN];
  __shared__ int prow[kLuMaxN];
  __shared__ int invp[kLuMaxN];
  __shared__ double cand_v[256];
  __shared__ int cand_i[256];
  __shared__ double piv_s;
  __shared__ int p_s;
  const int tid = threadIdx.x;
  const int G = blockDim.x / n, c = tid % n, g = tid / n;
  const bool own = g < G;
  double a[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int i = g + G * q;
    a[q] = (own && i < n) ? W[(long)i * n + c] : 0.0;
  }
  for (int i = tid; i < n; i += blockDim.x) used[i] = 0;
  double lsum = 0.0, sg = 1.0;
  int sing = 0;
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    if (own && c == k) {
      double best = -1.0, bv = 0.0;
      int bi = n;
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int i = g + G * q;
        if (i < n && !used[i]) {
          const double v = fabs(a[q]);
          if (v > best) { best = v; bi = i; bv = a[q]; }
        }
      }
      cand_v[g] = bv;
      cand_i[g] = bi;
    }
    __syncthreads();
    if (tid == 0) {
      double best = -1.0, bv = 0.0;
      int bi = n;
      for (int q = 0; q < G; ++q) {
        const int i = cand_i[q];
        if (i >= n) continue;
        const double v = fabs(cand_v[q]);
        if (v > best || (v == best && i < bi)) { best = v; bi = i; bv = cand_v[q]; }
      }
      p_s = bi;
      piv_s = bv;
      if (bi < n) { prow[k] = bi; used[bi] = 1; invp[bi] = k; }
    }
    __syncthreads();
    const int p = p_s;
    const double piv = piv_s;
    if (p >= n || !(piv != 0.0)) { sing = 1; break; }   // uniform across the block
    lsum += log(fabs(piv));
    if (piv < 0.0) sg = -sg;
    const double inv = 1.0 / piv;
    if (own && g == p % G) {
      const int qp = p / G;
      double v = 0.0;
#pragma unroll
      for (int q = 0; q < QMAX; ++q) if (q == qp) v = a[q];
      rk[c] = (c == k) ? inv : v * inv;
    }
    if (own && c == k) {
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int i = g + G * q;
        if (i < n) ck[i] = a[q];
      }
    }
    __syncthreads();
    if (own) {
      const double rc = rk[c], rkk = rk[k];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int i = g + G * q;
        if (i < n) {
          if (i == p) a[q] = rc;
          else if (c == k) a[q] = -ck[i] * rkk;
          else a[q] -= ck[i] * rc;
        }
      }
    }
    __syncthreads();
  }
  if (!sing) {
    // parity of k -> prow[k]
    if (tid == 0) {
      int* visited = cand_i;
      for (int i = 0; i < n; ++i) visited[i] = 0;
      for (int i = 0; i < n; ++i) {
        if (visited[i]) continue;
        int len = 0, j = i;
        while (!visited[j]) { visited[j] = 1; j = prow[j]; ++len; }
        if ((len & 1) == 0) sg = -sg;
      }
      piv_s = sg;
    }
    __syncthreads();
    sg = piv_s;
    if (own) {
      const int col = prow[c];
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int i = g + G * q;
        if (i < n) A[(long)invp[i] * n + col] = a[q];
      }
    }
  } else {
    const double nanv = __longlong_as_double(0x7ff8000000000000LL);
    for (int idx = tid; idx < n * n; idx += blockDim.x) A[idx] = nanv;
  }
  if (tid == 0) {
    *logdet = sing ? -__builtin_inf() : lsum;
    *detsign = sing ? 0.0 : sg;
    *singular = sing;
  }
}

template <int QMAX>
__global__ void __launch_bounds__(256)
gj_inverse_reg_kernel(const double* __restrict__ Wg, double* __restrict__ Ag, double* __restrict__ logdet,
                      double* __restrict__ detsign, int* __restrict__ singular, int n, long w_bs, long a_bs) {
  const long b = blockIdx.x;
  gj_reg_body<QMAX>(Wg + b * w_bs, Ag + b * a_bs, logdet + b, detsign + b, singular + b, n);
}

hipError_t launch_lu_inverse_lds(const SysDev& s, const WalkDev& w, hipStream_t st);

hipError_t launch_lu_inverse(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu;
  if (n > kLuMaxN) return hipErrorNotSupported;
  const int G = 256 / n, Q = (n + G - 1) / G;
  const long wbs = (long)s.nu * s.nd, abs_ = (long)s.nd * s.nu;
  // registers pay off only while the column slices stay short (high occupancy)
  if (Q > 8) return launch_lu_inverse_lds(s, w, st);
#define QMC_LU_REG(QM)                                                                              \
  hipLaunchKernelGGL(gj_inverse_reg_kernel<QM>, dim3(w.Wk), dim3(256), 0, st, w.W, w.A, w.logdet, \
                     w.detsign, w.singular, n, wbs, abs_)
  if (Q <= 4) QMC_LU_REG(4);
  else QMC_LU_REG(8);
#undef QMC_LU_REG
  return hipGetLastError();
}

// LDS variant with physical row swaps, kept for cross-checking the register kernel.
hipError_t launch_lu_inverse_lds(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu;
  if (n > kLuMaxN) return hipErrorNotSupported;
  const size_t shm = ((size_t)n * (n + 1) + 2 * (size_t)n) * sizeof(double);
  if (shm > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute((const void*)gj_inverse_kernel,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(gj_inverse_kernel, dim3(w.Wk), dim3(256), shm, st, w.W, w.A, w.logdet,
                     w.detsign, w.singular, n, (long)s.nu * s.nd, (long)s.nd * s.nu);
  return hipGetLastError();
}

// Persistent refresh over (member, walker) items of several systems; members
// not in `mask` are skipped.  The LU variant per member is the one the
// one-system refresh uses, so the results are identical.
__global__ void __launch_bounds__(256)
multi_lu_kernel(const SysDev* __restrict__ sysv, const WalkDev* __restrict__ wkv, const int2* __restrict__ items,
                int n_items, unsigned mask) {
  extern __shared__ double smem[];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();
    const int k = items[it].x, w = items[it].y;
    if (!((mask >> k) & 1u)) continue;
    const SysDev& s = sysv[k];
    const WalkDev& wd = wkv[k];
    const int n = s.nu;
    const int G = 256 / n, Q = (n + G - 1) / G;
    const double* W = wd.W + (long)w * n * n;
    double* A = wd.A + (long)w * n * n;
    if (Q <= 8) gj_reg_body<8>(W, A, wd.logdet + w, wd.detsign + w, wd.singular + w, n);
    else gj_lds_body(W, A, wd.logdet + w, wd.detsign + w, wd.singular + w, n, smem);
    __syncthreads();
    if (threadIdx.x == 0) {
      const int sing = wd.singular[w];
      wd.logabs[w] = sing ? -__builtin_inf() : wd.logdet[w] + wd.J[w];
      wd.sign[w] = wd.detsign[w];
    }
  }
}

hipError_t prepare_multi_lu(size_t shm) {
  if (shm <= 64 * 1024) return hipSuccess;
  return hipFuncSetAttribute((const void*)multi_lu_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
}

// (prepare_multi_lu must have been called for shm beforehand: this launch may be
// inside a captured graph.)
hipError_t launch_multi_lu(const SysDev* sysv, const WalkDev* wkv, const int2* items, int n_items,
                           unsigned mask, size_t shm, int grid, hipStream_t st) {
  hipLaunchKernelGGL(multi_lu_kernel, dim3(grid), dim3(256), shm, st, sysv, wkv, items, n_items, mask);
  return hipGetLastError();
}

}  // namespace qmc
