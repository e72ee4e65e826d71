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

__global__ void __launch_bounds__(256)
gj_inverse_kernel(const double* __restrict__ Wg, double* __restrict__ Ag, double* __restrict__ logdet,
                  double* __restrict__ detsign, int* __restrict__ singular, int n, long w_bs, long a_bs) {
  extern __shared__ double smem[];
  const int ld = n + 1;
  double* M = smem;                 // n x ld
  double* rk = M + (long)n * ld;    // scaled pivot row
  double* ck = rk + n;              // pivot column before the step
  __shared__ int perm[kLuMaxN];
  __shared__ int piv_s;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* W = Wg + blockIdx.x * w_bs;
  double* A = Ag + blockIdx.x * a_bs;

  for (int idx = tid; idx < n * n; idx += blockDim.x) M[(idx / n) * ld + (idx % n)] = W[idx];

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
    for (int idx = tid; idx < n * n; idx += blockDim.x) {
      const int i = idx / n, j = idx - (idx / n) * n;
      double v;
      if (i == k) v = rk[j];
      else if (j == k) v = -ck[i] * rk[k];
      else v = M[i * ld + j] - ck[i] * rk[j];
      M[i * ld + j] = v;
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
    logdet[blockIdx.x] = sing ? -__builtin_inf() : lsum;
    detsign[blockIdx.x] = sing ? 0.0 : sg;
    singular[blockIdx.x] = sing;
  }
}

hipError_t launch_lu_inverse(const SysDev& s, const WalkDev& w, hipStream_t st) {
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

}  // namespace qmc
