// Jastrow-basis terms of the evaluation: one-body inhomogeneous and
// three/four-body factors (onebody_J_inh, threebody_jastrow) over a separate
// basis chi (Gaussian or Slater functions on the nuclei).
//
//   J1inh = sum_i m_{s_i} . chi(r_i)
//   J3/4  = sum_{i<j} chi(r_i)^T M^{s_i s_j} chi(r_j)
//         = 1/2 sum_i chi(r_i)^T (G_{s_i} - h_i)
// with X_s = sum_{j of spin s} chi(r_j), [G_u; G_d] = M3 [X_u; X_d] (M3 the
// symmetric [[M_uu, M_ud], [M_ud^T, M_dd]]) and h_i = M^{s_i s_i} chi(r_i): the
// vector multiplying chi(r_i) in electron i's pair terms is G_{s_i} - h_i.
// Electron i's terms are linear in chi(r_i), so with g_i = G_{s_i} - h_i + m_{s_i}
//   grad_i J = grad chi(r_i) . g_i,   lap_i J = lap chi(r_i) . g_i.
// Steps: chi at every electron; X and G (one workgroup per walker); h by two
// FP64 MFMA products per spin block, batched over walkers; per-electron dot
// products, which the assembly adds to the J1 + J2 terms.
#include "internal.h"

namespace qmc {

__global__ void __launch_bounds__(64) jb_values_kernel(SysDev s, const double* __restrict__ r,
                                                       double* __restrict__ chi) {
  const long row = blockIdx.x;   // w * N + i
  const double px = r[3 * row], py = r[3 * row + 1], pz = r[3 * row + 2];
  double* out = chi + row * s.LJ;
  for (int k = threadIdx.x; k < s.LJ; k += blockDim.x) out[k] = basis_value_tab(s.jbfn, s.jkind, k, px, py, pz);
}

// X_u, X_d (fixed electron order) and G = M3 X, one workgroup per walker.
__global__ void __launch_bounds__(256) j3_sum_kernel(SysDev s, WalkDev w) {
  __shared__ double X[2 * kMaxLJ];
  const int wk = blockIdx.x, LJ = s.LJ;
  const double* chi = w.chi + (long)wk * s.N * LJ;
  for (int k = threadIdx.x; k < LJ; k += blockDim.x) {
    double xu = 0.0, xd = 0.0;
    for (int i = 0; i < s.nu; ++i) xu += chi[(long)i * LJ + k];
    for (int i = s.nu; i < s.N; ++i) xd += chi[(long)i * LJ + k];
    X[k] = xu;
    X[LJ + k] = xd;
  }
  __syncthreads();
  double* G = w.G3 + (long)wk * 2 * LJ;
  for (int o = threadIdx.x; o < 2 * LJ; o += blockDim.x) {
    const double* row = s.M3 + (long)o * 2 * LJ;
    double g = 0.0;
    for (int c = 0; c < 2 * LJ; ++c) g += row[c] * X[c];
    G[o] = g;
  }
}

// Per-electron terms: one wave per (walker, electron).
__global__ void __launch_bounds__(256) j3_rowdot_kernel(SysDev s, WalkDev w, int rows) {
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int LJ = s.LJ;
  const int wk = (int)(row / s.N), i = (int)(row % s.N);
  const int sp = i < s.nu ? 0 : 1;
  const double px = w.r[3 * row], py = w.r[3 * row + 1], pz = w.r[3 * row + 2];
  const double* G = w.G3 + ((long)wk * 2 + sp) * LJ;
  const double* h = w.hv + row * LJ;
  const double* m = s.jm + (long)sp * LJ;
  double val = 0.0, gx = 0.0, gy = 0.0, gz = 0.0, gl = 0.0;
  for (int k = lane; k < LJ; k += 64) {
    double v, vx, vy, vz, vl;
    basis_vgl_tab(s.jbfn, s.jkind, k, px, py, pz, v, vx, vy, vz, vl);
    const double pair = G[k] - h[k];
    const double g = pair + m[k];
    val += v * (0.5 * pair + m[k]);
    gx += vx * g; gy += vy * g; gz += vz * g; gl += vl * g;
  }
  val = wave_sum(val); gx = wave_sum(gx); gy = wave_sum(gy); gz = wave_sum(gz); gl = wave_sum(gl);
  if (lane == 0) {
    double* o = w.j3e + row * 5;
    o[0] = val; o[1] = gx; o[2] = gy; o[3] = gz; o[4] = gl;
  }
}

hipError_t launch_jastrow3_eval(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (s.LJ <= 0) return hipSuccess;
  if (s.LJ > kMaxLJ) return hipErrorNotSupported;
  const long rows = (long)w.Wk * s.N;
  hipLaunchKernelGGL(jb_values_kernel, dim3((unsigned)rows), dim3(64), 0, st, s, w.r, w.chi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(j3_sum_kernel, dim3(w.Wk), dim3(256), 0, st, s, w);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // h_i = M^{ss} chi(r_i): rows of one spin of every walker times the diagonal
  // block of M3 (symmetric), batched over walkers
  const int LJ = s.LJ;
  for (int sp = 0; sp < 2; ++sp) {
    const int row0 = sp == 0 ? 0 : s.nu, nrow = sp == 0 ? s.nu : s.nd;
    GemmArgs g = gemm_args(nrow, LJ, LJ);
    g.A = w.chi + (long)row0 * LJ; g.lda = LJ; g.a_bs = (long)s.N * LJ;
    g.B = s.M3 + (long)sp * LJ * 2 * LJ + (long)sp * LJ; g.ldb = 2 * LJ; g.b_bs = 0;
    g.C = w.hv + (long)row0 * LJ; g.ldc = LJ; g.c_bs = (long)s.N * LJ;
    g.batch = w.Wk;
    e = gemm_f64(g, false, false, false, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(j3_rowdot_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, s, w, (int)rows);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Logarithmic derivatives of the Jastrow-basis coefficients, per walker:
//   d log Psi / d m_s      = X_s = sum_{i of spin s} chi(r_i)
//   d log Psi / d M^{ud}   = X_u X_d^T
//   d log Psi / d M^{ss}   = 1/2 (X_s X_s^T - C_s),  C_s = sum_{i of spin s} chi(r_i) chi(r_i)^T
// (M^{ss} symmetric: the gradient with respect to a symmetric matrix, each
// unordered pair once, written as a symmetric matrix so that
// dlog Psi = sum_kl D_kl dM_kl for every symmetric dM).  chi is the walkers'
// current state (evaluation, then the accepted moves).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) j3_logderiv_kernel(SysDev s, WalkDev w, double* __restrict__ dm,
                                                          double* __restrict__ dM) {
  __shared__ double X[2 * kMaxLJ];
  const int wk = blockIdx.x, LJ = s.LJ;
  const double* chi = w.chi + (long)wk * s.N * LJ;
  for (int k = threadIdx.x; k < LJ; k += blockDim.x) {
    double xu = 0.0, xd = 0.0;
    for (int i = 0; i < s.nu; ++i) xu += chi[(long)i * LJ + k];
    for (int i = s.nu; i < s.N; ++i) xd += chi[(long)i * LJ + k];
    X[k] = xu;
    X[LJ + k] = xd;
    if (dm) { dm[(long)wk * 2 * LJ + k] = xu; dm[(long)wk * 2 * LJ + LJ + k] = xd; }
  }
  __syncthreads();
  if (!dM) return;
  double* D = dM + (long)wk * 3 * LJ * LJ;
  const long LL = (long)LJ * LJ;
  for (long idx = threadIdx.x; idx < LL; idx += blockDim.x) {
    const int k = (int)(idx / LJ), l = (int)(idx % LJ);
    const double cu = s.nu > 0 ? D[idx] : 0.0, cd = s.nd > 0 ? D[LL + idx] : 0.0;   // C_s in place
    D[idx] = 0.5 * (X[k] * X[l] - cu);                           // up-up
    D[LL + idx] = 0.5 * (X[LJ + k] * X[LJ + l] - cd);            // down-down
    D[2 * LL + idx] = X[k] * X[LJ + l];                          // up-down
  }
}

hipError_t launch_jastrow3_logderiv(const SysDev& s, const WalkDev& w, double* dm, double* dM, hipStream_t st) {
  if (s.LJ <= 0 || s.LJ > kMaxLJ) return hipErrorNotSupported;
  const int LJ = s.LJ;
  if (dM) {
    // C_s = chi_s^T chi_s into the up-up and down-down slots, batched over walkers
    for (int sp = 0; sp < 2; ++sp) {
      const int row0 = sp == 0 ? 0 : s.nu, nrow = sp == 0 ? s.nu : s.nd;
      GemmArgs g = gemm_args(LJ, LJ, nrow);
      g.A = w.chi + (long)row0 * LJ; g.lda = LJ; g.a_bs = (long)s.N * LJ;
      g.B = w.chi + (long)row0 * LJ; g.ldb = LJ; g.b_bs = (long)s.N * LJ;
      g.C = dM + (long)sp * LJ * LJ; g.ldc = LJ; g.c_bs = 3L * LJ * LJ;
      g.batch = w.Wk;
      if (nrow == 0) continue;   // C_s = 0: the kernel does not read the slot
      const hipError_t e = gemm_f64(g, true, false, false, st);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(j3_logderiv_kernel, dim3(w.Wk), dim3(256), 0, st, s, w, dm, dM);
  return hipGetLastError();
}

}  // namespace qmc
