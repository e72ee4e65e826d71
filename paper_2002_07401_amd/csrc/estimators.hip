// Force and optimisation estimators on top of the adjoint's per-walker
// derivatives (Atomic forces and Stochastic reconfiguration sections).
//
// * Space warp: omega_a(r) = kappa_a / sum_b kappa_b, kappa = 1/|r - R|^4;
//   total derivatives dR_a + sum_i omega_a(r_i) dr_i (+ 1/2 sum_i grad omega_a(r_i)
//   for ln(J^1/2 Psi)), one workgroup per walker.
// * Finite-variance reweighting: R = (S sum_ij (W^-1)_ij^2)^(-theta),
//   S = min_i sum_j W_ij^2, weight = (R / max(R, eps))^2, one workgroup per walker
//   (W the geminal matrix, or the Pfaffian's pairing matrix G~).
// * Stochastic reconfiguration: (S + eps diag S) delta = f with
//   S v = O^T (w o (O v)) / sum w - Obar (Obar . v), f = -2 sum_i w_i e_i (O_i - Obar) / sum w,
//   solved by diagonally preconditioned conjugate gradients on the device
//   without forming S: per iteration u = O p (and Obar . p), O^T (w o u) by
//   column slices, S' p with partial sums of p . S'p, the x / r update with
//   partial sums of r . z and r . r, the p update.  Every reduction is a fixed-order sum
//   of per-block partials; the iteration scalars are double-buffered by parity
//   so no block reads a value another block of the same launch writes.
#include <mutex>

#include "internal.h"

namespace qmc {

// ---------------------------------------------------------------------------
// space warp
// ---------------------------------------------------------------------------
constexpr int kSwctMaxN = 1024;

__global__ void __launch_bounds__(256)
swct_kernel(SysDev s, const double* __restrict__ r, const double* __restrict__ dR, const double* __restrict__ dr,
            int jac, double* __restrict__ out) {
  __shared__ double K[kSwctMaxN][4];   // sum_b kappa_b and its gradient, per electron
  const int wk = blockIdx.x, N = s.N, A = s.n_nuc;
  const double* rw = r + (long)wk * N * 3;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double k0 = 0.0, kx = 0.0, ky = 0.0, kz = 0.0;
    for (int b = 0; b < A; ++b) {
      const double dx = rw[3 * i] - s.R[3 * b], dy = rw[3 * i + 1] - s.R[3 * b + 1], dz = rw[3 * i + 2] - s.R[3 * b + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ik = 1.0 / (r2 * r2);
      const double g = -4.0 * ik / r2;
      k0 += ik; kx += g * dx; ky += g * dy; kz += g * dz;
    }
    K[i][0] = k0; K[i][1] = kx; K[i][2] = ky; K[i][3] = kz;
  }
  __syncthreads();
  const double* drw = dr + (long)wk * N * 3;
  for (int a = threadIdx.x; a < A; a += blockDim.x) {
    double t0 = 0.0, t1 = 0.0, t2 = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
    for (int i = 0; i < N; ++i) {
      const double dx = rw[3 * i] - s.R[3 * a], dy = rw[3 * i + 1] - s.R[3 * a + 1], dz = rw[3 * i + 2] - s.R[3 * a + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      const double ka = 1.0 / (r2 * r2);
      const double om = ka / K[i][0];
      t0 += om * drw[3 * i]; t1 += om * drw[3 * i + 1]; t2 += om * drw[3 * i + 2];
      if (jac) {
        const double g = -4.0 * ka / r2, iK = 1.0 / K[i][0];
        j0 += g * dx * iK - ka * K[i][1] * iK * iK;
        j1 += g * dy * iK - ka * K[i][2] * iK * iK;
        j2 += g * dz * iK - ka * K[i][3] * iK * iK;
      }
    }
    const double* dRa = dR + ((long)wk * A + a) * 3;
    double* o = out + ((long)wk * A + a) * 3;
    o[0] = dRa[0] + t0 + 0.5 * j0;
    o[1] = dRa[1] + t1 + 0.5 * j1;
    o[2] = dRa[2] + t2 + 0.5 * j2;
  }
}

hipError_t launch_swct(const SysDev& s, int Wk, const double* r, const double* dR, const double* dr, int jac,
                       double* out, hipStream_t st) {
  if (s.N > kSwctMaxN) return hipErrorNotSupported;
  hipLaunchKernelGGL(swct_kernel, dim3(Wk), dim3(256), 0, st, s, r, dR, dr, jac, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reweighting factor
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
reweight_kernel(SysDev s, WalkDev w, double theta, double eps, double* __restrict__ Rout,
                double* __restrict__ wout) {
  __shared__ double red[4], redm[4];
  // the pairing matrix: W (n_up x n_up), or G~ of the Pfaffian with its exact inverse
  const int wk = blockIdx.x, n = s.pairing ? s.npf : s.nu, lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const double* W = w.W + (long)wk * n * n;
  const double* A = w.A + (long)wk * n * n;
  double smin = __builtin_inf(), sa = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double rs = 0.0;
    for (int j = 0; j < n; ++j) rs += W[(long)i * n + j] * W[(long)i * n + j];
    smin = fmin(smin, rs);
  }
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) sa += A[idx] * A[idx];
  sa = wave_sum(sa);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) smin = fmin(smin, __shfl_xor(smin, o, 64));
  if (lane == 0) { red[wave] = sa; redm[wave] = smin; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0, m = __builtin_inf();
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) { t += red[k]; m = fmin(m, redm[k]); }
    const double R = pow(m * t, -theta);
    const double Re = fmax(R, eps);
    Rout[wk] = R;
    if (wout) wout[wk] = (R / Re) * (R / Re);
  }
}

hipError_t launch_reweight(const SysDev& s, const WalkDev& w, double theta, double eps, double* R, double* weight,
                           hipStream_t st) {
  hipLaunchKernelGGL(reweight_kernel, dim3(w.Wk), dim3(256), 0, st, s, w, theta, eps, R, weight);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// stochastic reconfiguration
// ---------------------------------------------------------------------------
// Conjugate gradients preconditioned by the diagonal of S' (m_k = (1 + eps) s_kk,
// 1 where s_kk = 0): the regularisation is relative to the diagonal, so the
// diagonally scaled matrix has unit diagonal and a condition number bounded by
// about (P + eps) / eps whatever the scales of the parameters.
// The column sums over samples (moments, O^T (w o u)) run on a 2-D grid:
// blocks of 256 columns times `ms` slices of the samples, each slice writing
// its partial sums, which a second kernel adds in slice order.
// Workspace (doubles): Obar, d (= diag S), f, r, p, Sp [P each], u [M],
// part1, part2, part3 [nblk each], colpart [2][ms][P], scalars [16]:
//   sc[0] = sum w, sc[1] = f . f, sc[2 + (it & 1)] = r . z at iteration it,
//   sc[4] = Obar . p, sc[5] = done, sc[6] = r . r of the last update
struct SrWork {
  double *Obar, *d, *f, *r, *p, *Sp, *u, *part1, *part2, *part3, *colpart, *sc;
  long P;
  int M, nblk, ms, rows;   // rows: samples per slice
  double eps;
};

static int sr_slices(int M) {
  const int ms = (M + 127) / 128;   // about 128 samples per slice, at most 64 slices
  return ms < 1 ? 1 : (ms > 64 ? 64 : ms);
}

__device__ inline double sr_precond(const SrWork& q, long k) {
  const double m = (1.0 + q.eps) * q.d[k];
  return m > 0.0 ? m : 1.0;
}

__device__ double blk_sum256(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < 4; ++k) t += red[k];
  __syncthreads();
  return t;
}

// sum of the weights (single workgroup)
__global__ void __launch_bounds__(256) sr_wsum_kernel(SrWork q, const double* __restrict__ wts) {
  __shared__ double red[4];
  double t = 0.0;
  for (int i = threadIdx.x; i < q.M; i += blockDim.x) t += wts ? wts[i] : 1.0;
  t = blk_sum256(t, red);
  if (threadIdx.x == 0) q.sc[0] = t;
}

// Column sums over one slice of samples: pass 0: sum w O; pass 1: sum w (O - Obar)^2
// and sum w e (O - Obar); pass 2: sum w u O (u = O p).
__global__ void __launch_bounds__(256)
sr_colsum_kernel(SrWork q, const double* __restrict__ O, const double* __restrict__ el,
                 const double* __restrict__ wts, int pass) {
  if (pass == 2 && q.sc[5] != 0.0) return;   // converged (uniform)
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int sl = blockIdx.y;
  if (k >= q.P) return;
  const int i0 = sl * q.rows, i1 = min(i0 + q.rows, q.M);
  double a = 0.0, b = 0.0;
  if (pass == 0) {
    for (int i = i0; i < i1; ++i) a += (wts ? wts[i] : 1.0) * O[(long)i * q.P + k];
  } else if (pass == 1) {
    const double m = q.Obar[k];
    for (int i = i0; i < i1; ++i) {
      const double wi = wts ? wts[i] : 1.0, c = O[(long)i * q.P + k] - m;
      a += wi * c * c;
      b += wi * el[i] * c;
    }
  } else {
    for (int i = i0; i < i1; ++i) a += (wts ? wts[i] : 1.0) * q.u[i] * O[(long)i * q.P + k];
  }
  q.colpart[(long)sl * q.P + k] = a;
  if (pass == 1) q.colpart[((long)q.ms + sl) * q.P + k] = b;
}

// Obar = (sum over slices) / sum w
__global__ void __launch_bounds__(256) sr_mean_kernel(SrWork q) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= q.P) return;
  double a = 0.0;
  for (int sl = 0; sl < q.ms; ++sl) a += q.colpart[(long)sl * q.P + k];
  q.Obar[k] = a / q.sc[0];
}

// diag S and f; x = 0, r = f, p = z = f / m; partial sums of r . z and r . r
__global__ void __launch_bounds__(256) sr_moments_kernel(SrWork q, double* __restrict__ x) {
  __shared__ double red[4];
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (k < q.P) {
    const double iw = 1.0 / q.sc[0];
    double s2 = 0.0, fe = 0.0;
    for (int sl = 0; sl < q.ms; ++sl) {
      s2 += q.colpart[(long)sl * q.P + k];
      fe += q.colpart[((long)q.ms + sl) * q.P + k];
    }
    const double f = -2.0 * fe * iw;
    q.d[k] = s2 * iw; q.f[k] = f;
    const double z = f / sr_precond(q, k);
    q.r[k] = f; q.p[k] = z; x[k] = 0.0;
    rz = f * z;
    rr = f * f;
  }
  rz = blk_sum256(rz, red);
  rr = blk_sum256(rr, red);
  if (threadIdx.x == 0) { q.part2[blockIdx.x] = rz; q.part3[blockIdx.x] = rr; }
}

// r0 . z0 and f . f (single workgroup, fixed order)
__global__ void __launch_bounds__(64) sr_init_kernel(SrWork q) {
  if (threadIdx.x != 0) return;
  double rz = 0.0, rr = 0.0;
  for (int b = 0; b < q.nblk; ++b) { rz += q.part2[b]; rr += q.part3[b]; }
  q.sc[1] = rr;
  q.sc[2] = rz;
  q.sc[6] = rr;
  q.sc[5] = rr > 0.0 ? 0.0 : 1.0;
}

// u_i = O_i . p (workgroups 0..M-1) and Obar . p (workgroup M)
__global__ void __launch_bounds__(256) sr_op_kernel(SrWork q, const double* __restrict__ O) {
  __shared__ double red[4];
  if (q.sc[5] != 0.0) return;   // converged (uniform)
  const int i = blockIdx.x;
  const double* row = i < q.M ? O + (long)i * q.P : q.Obar;
  double t = 0.0;
  for (long k = threadIdx.x; k < q.P; k += blockDim.x) t += row[k] * q.p[k];
  t = blk_sum256(t, red);
  if (threadIdx.x == 0) {
    if (i < q.M) q.u[i] = t;
    else q.sc[4] = t;
  }
}

// S'p from the slice sums of O^T (w o u), and partial sums of p . S'p
__global__ void __launch_bounds__(256) sr_sp_kernel(SrWork q) {
  __shared__ double red[4];
  if (q.sc[5] != 0.0) return;
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double pp = 0.0;
  if (k < q.P) {
    double t = 0.0;
    for (int sl = 0; sl < q.ms; ++sl) t += q.colpart[(long)sl * q.P + k];
    const double sp = t / q.sc[0] - q.Obar[k] * q.sc[4] + q.eps * q.d[k] * q.p[k];
    q.Sp[k] = sp;
    pp = q.p[k] * sp;
  }
  pp = blk_sum256(pp, red);
  if (threadIdx.x == 0) q.part1[blockIdx.x] = pp;
}

// alpha = r.z / p.S'p; x += alpha p; r -= alpha S'p; partial sums of r . z and r . r
__global__ void __launch_bounds__(256) sr_update_kernel(SrWork q, double* __restrict__ x, int it) {
  __shared__ double red[4];
  __shared__ double alpha_s;
  if (q.sc[5] != 0.0) return;
  if (threadIdx.x == 0) {
    double pSp = 0.0;
    for (int b = 0; b < q.nblk; ++b) pSp += q.part1[b];
    alpha_s = pSp > 0.0 ? q.sc[2 + (it & 1)] / pSp : 0.0;
  }
  __syncthreads();
  const double alpha = alpha_s;
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double rz = 0.0, rr = 0.0;
  if (k < q.P) {
    x[k] += alpha * q.p[k];
    const double rk = q.r[k] - alpha * q.Sp[k];
    q.r[k] = rk;
    rz = rk * rk / sr_precond(q, k);
    rr = rk * rk;
  }
  rz = blk_sum256(rz, red);
  rr = blk_sum256(rr, red);
  if (threadIdx.x == 0) { q.part2[blockIdx.x] = rz; q.part3[blockIdx.x] = rr; }
}

// beta = r.z(new) / r.z(old); p = z + beta p
__global__ void __launch_bounds__(256) sr_dir_kernel(SrWork q, int it) {
  __shared__ double beta_s, rzn_s, rrn_s;
  if (q.sc[5] != 0.0) return;
  if (threadIdx.x == 0) {
    double rzn = 0.0, rrn = 0.0;
    for (int b = 0; b < q.nblk; ++b) { rzn += q.part2[b]; rrn += q.part3[b]; }
    const double rzo = q.sc[2 + (it & 1)];
    beta_s = rzo > 0.0 ? rzn / rzo : 0.0;
    rzn_s = rzn;
    rrn_s = rrn;
  }
  __syncthreads();
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < q.P) q.p[k] = q.r[k] / sr_precond(q, k) + beta_s * q.p[k];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    q.sc[2 + ((it + 1) & 1)] = rzn_s;
    q.sc[6] = rrn_s;
  }
}

// Converged when r.r <= tol^2 f.f (read after the whole direction launch)
__global__ void __launch_bounds__(64) sr_check_kernel(SrWork q, double tol) {
  if (threadIdx.x == 0 && q.sc[5] == 0.0 && q.sc[6] <= tol * tol * q.sc[1]) q.sc[5] = 1.0;
}

__global__ void __launch_bounds__(256) sr_finish_kernel(SrWork q, double* __restrict__ force,
                                                        double* __restrict__ resid) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (force && k < q.P) force[k] = q.f[k];
  if (resid && k == 0) resid[0] = q.sc[1] > 0.0 ? sqrt(q.sc[6] / q.sc[1]) : 0.0;
}

size_t sr_workspace_doubles(int M, long P) {
  const long nblk = (P + 255) / 256;
  return (size_t)(6 * P + M + 3 * nblk + 16 + 2L * sr_slices(M) * P);
}

hipError_t launch_sr_step(int M, long P, const double* O, const double* el, const double* wts, double eps,
                          int max_iter, double tol, double* delta, double* force, double* resid, double* work,
                          hipStream_t st) {
  SrWork q;
  q.P = P; q.M = M; q.nblk = (int)((P + 255) / 256); q.eps = eps;
  q.ms = sr_slices(M); q.rows = (M + q.ms - 1) / q.ms;
  double* p = work;
  q.Obar = p; p += P; q.d = p; p += P; q.f = p; p += P; q.r = p; p += P; q.p = p; p += P; q.Sp = p; p += P;
  q.u = p; p += M; q.part1 = p; p += q.nblk; q.part2 = p; p += q.nblk; q.part3 = p; p += q.nblk;
  q.colpart = p; p += 2L * q.ms * P; q.sc = p;
  const dim3 gk(q.nblk), g2(q.nblk, q.ms), blk(256);
  hipLaunchKernelGGL(sr_wsum_kernel, dim3(1), blk, 0, st, q, wts);
  hipLaunchKernelGGL(sr_colsum_kernel, g2, blk, 0, st, q, O, el, wts, 0);
  hipLaunchKernelGGL(sr_mean_kernel, gk, blk, 0, st, q);
  hipLaunchKernelGGL(sr_colsum_kernel, g2, blk, 0, st, q, O, el, wts, 1);
  hipLaunchKernelGGL(sr_moments_kernel, gk, blk, 0, st, q, delta);
  hipLaunchKernelGGL(sr_init_kernel, dim3(1), dim3(64), 0, st, q);
  for (int it = 0; it < max_iter; ++it) {
    hipLaunchKernelGGL(sr_op_kernel, dim3(M + 1), blk, 0, st, q, O);
    hipLaunchKernelGGL(sr_colsum_kernel, g2, blk, 0, st, q, O, el, wts, 2);
    hipLaunchKernelGGL(sr_sp_kernel, gk, blk, 0, st, q);
    hipLaunchKernelGGL(sr_update_kernel, gk, blk, 0, st, q, delta, it);
    hipLaunchKernelGGL(sr_dir_kernel, gk, blk, 0, st, q, it);
    hipLaunchKernelGGL(sr_check_kernel, dim3(1), dim3(64), 0, st, q, tol);
  }
  hipLaunchKernelGGL(sr_finish_kernel, gk, blk, 0, st, q, force, resid);
  return hipGetLastError();
}

}  // namespace qmc

// ---------------------------------------------------------------------------
// SR step without allocation: the workspace is a fixed device array of the
// library (one copy per GPU, alive until the process ends).  Host code never
// passes the array's name to a kernel or a copy: on the host that name is a
// stand-in, not a device address.  Its address on each device is looked up
// once, with that device current, and kept.
// ---------------------------------------------------------------------------
constexpr size_t kSrStaticDoubles = (size_t)2 << 20;   // 16 MiB of FP64
static __device__ __align__(256) double scratch[kSrStaticDoubles];
namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

extern "C" qmc_status qmc_sr_step_static(int32_t n_samples, int64_t n_params, const double* O, const double* e_loc,
                                         const double* weights, double eps, int32_t max_iter, double tol,
                                         double* delta, double* force, double* residual, hipStream_t stream) {
  using namespace qmc;
  if (!O || !e_loc || !delta) return set_error(QMC_ERR_ARG, "null argument");
  if (n_samples <= 0 || n_params <= 0 || max_iter < 0) return set_error(QMC_ERR_ARG, "bad sizes");
  if (!(eps >= 0.0) || !(tol >= 0.0)) return set_error(QMC_ERR_ARG, "eps and tol must be >= 0");
  if (sr_workspace_doubles(n_samples, (long)n_params) > kSrStaticDoubles)
    return set_error(QMC_ERR_SHAPE, "SR problem needs more than the 16 MiB static workspace "
                                    "(qmc_sr_workspace_size > 16777216 bytes): use qmc_sr_step");
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(QMC_ERR_HIP, hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(QMC_ERR_UNSUPPORTED, "device ordinal beyond 63");
  double* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
      void* p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) return set_error(QMC_ERR_HIP, "hipGetSymbolAddress of the SR scratch failed");
      g_scratch_ptr[dev] = (double*)p;
    }
    ptr = g_scratch_ptr[dev];
  }
  e = launch_sr_step(n_samples, (long)n_params, O, e_loc, weights, eps, max_iter, tol, delta, force, residual, ptr,
                     stream);
  if (e != hipSuccess) return set_error(QMC_ERR_HIP, hipGetErrorString(e));
  return QMC_OK;
}
