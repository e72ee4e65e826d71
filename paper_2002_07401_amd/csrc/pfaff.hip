// Pfaffian wave function (Pfaffian wave function section): Psi = Pf(G~) exp J.
//
// G~ is the skew-symmetric (N + k) x (N + k) pairing matrix: for electrons i, j
// (spins s_i, s_j)  G~_ij = psi(r_i)^T A^{s_i s_j} psi(r_j)  with A^{uu}, A^{dd}
// skew-symmetric (triplet components +1 / -1), A^{ud} the unlike-spin
// singlet + triplet-zero coefficients and A^{du} = -(A^{ud})^T (eq:g,
// agp_expansion); k unpaired orbitals enter as fictitious electrons,
// G~_{i, N+l} = psi(r_i) . U^{s_i}_l (eq:pfodd).
//
// Per electron j two rows are kept, B^s_j = psi(r_j)^T K^{s s_j} with
// K^{s s'} = (A^{s s'})^T, so that row i of G~ is psi(r_i) . B^{s_i}_j: the
// rows are four FP64 MFMA products over the walkers, G~ one dot product per
// entry of its upper triangle (the lower one mirrored, so G~ is exactly
// skew-symmetric).  Pf(G~) (log|Pf| and sign) comes from a Parlett-Reid
// reduction with partial pivoting, one workgroup per walker on a copy in LDS;
// G~^{-1} from the Gauss-Jordan kernel of the determinant path.
//
// Pf is linear in row and column i, which alone depend on r_i, and
// d log Pf = 1/2 tr(G~^{-1} dG~) with G~^{-1} skew-symmetric, so the
// determinant's cofactor identities hold with Y_i = sum_j (G~^{-1})_ji B^{s_i}_j
// (+ sum_l (G~^{-1})_{N+l, i} U^{s_i}_l): grad_i Pf / Pf = grad psi(r_i) . Y_i and
// lap_i Pf / Pf = lap psi(r_i) . Y_i; the row-dot, Jastrow and assembly kernels
// of the determinant path then apply unchanged, and so do the lattice hops
// (a hop's ratio is psi(r') . Y_i).
//
// A move of electron e replaces row e (and column e, negated) by
//   g'_j = psi(r') . B^{s_e}_j  (j < N, j != e),  g'_e = 0,  g'_{N+l} = psi(r') . U^{s_e}_l,
// and Pf(G') / Pf(G) = sum_j g'_j (G^{-1})_je.  With delta = g' - G[e, :],
// G' = G + e_e delta^T - delta e_e^T, and Woodbury's identity for this skew
// rank-2 change gives, with p = G^{-1} e_e, q = G^{-1} delta and rho the ratio,
//   G'^{-1} = G^{-1} + (p q^T - q p^T) / rho.
// The accept also rewrites electron e's basis row and its two B rows (one
// MFMA product over all walkers, which move the same electron); the
// inverse is recomputed from the maintained G~ every refresh_every moves.
#include "move_dev.h"

namespace qmc {

constexpr int kPfMaxN = kLuRowMax;   // G~ dimension (Gauss-Jordan register kernel)

// ---------------------------------------------------------------------------
// B rows: P (B^u) and Bd (B^d), each as up rows times K^{s u} and down rows
// times K^{s d}, batched over walkers
// ---------------------------------------------------------------------------
hipError_t launch_pf_B_build(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const long rowst = (long)s.N * s.Lp;
  struct Part { const double* K; double* out; int row0, nrow; };
  const Part parts[4] = {{s.Kuu, (double*)w.P, 0, s.nu}, {s.Kud, (double*)w.P, s.nu, s.nd},
                         {s.Kdu, w.Bd, 0, s.nu}, {s.Kdd, w.Bd, s.nu, s.nd}};
  for (const Part& x : parts) {
    if (x.nrow == 0) continue;
    GemmArgs g = gemm_args(w.Wk * x.nrow, s.Lp, s.Lp);
    g.A = (const double*)w.phi + (long)x.row0 * s.Lp; g.lda = s.Lp; g.a_grp = x.nrow; g.a_gs = rowst;
    g.B = x.K; g.ldb = s.Lp;
    g.C = x.out + (long)x.row0 * s.Lp; g.ldc = s.Lp; g.c_grp = x.nrow; g.c_gs = rowst;
    const hipError_t e = gemm_f64(g, false, false, true, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// G~: rows of spin s are Phi_s (B^s)^T over the N electrons and Phi_s (U^s)^T
// over the fictitious ones (FP64 MFMA products batched over walkers, written
// into the rows of G~); the mirror kernel then makes G~ exactly skew-symmetric
// from its upper triangle and clears the fictitious block.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pf_mirror_kernel(SysDev s, WalkDev w) {
  const int wk = blockIdx.x, n = s.npf, N = s.N;
  double* G = w.W + (long)wk * n * n;
  for (int idx = threadIdx.x; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    if (i > j) G[idx] = (i >= N && j >= N) ? 0.0 : -G[(long)j * n + i];
    else if (i == j) G[idx] = 0.0;
    else if (i >= N) G[idx] = 0.0;   // fictitious-fictitious block
  }
}

hipError_t launch_pf_G_build(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (s.npf > kPfMaxN) return hipErrorNotSupported;
  const long rowst = (long)s.N * s.Lp, n = s.npf;
  for (int sp = 0; sp < 2; ++sp) {
    const int i0 = sp == 0 ? 0 : s.nu, ni = sp == 0 ? s.nu : s.nd;
    if (ni == 0) continue;
    GemmArgs g = gemm_args(ni, s.N, s.Lp);
    g.A = (const double*)w.phi + (long)i0 * s.Lp; g.lda = s.Lp; g.a_bs = rowst;
    g.B = sp == 0 ? (const double*)w.P : w.Bd; g.ldb = s.Lp; g.b_bs = rowst;   // stored [j][mu]
    g.C = w.W + (long)i0 * n; g.ldc = n; g.c_bs = n * n;
    g.batch = w.Wk;
    hipError_t e = gemm_f64(g, false, true, false, st);
    if (e != hipSuccess) return e;
    if (s.pk > 0) {
      GemmArgs u = gemm_args(ni, s.pk, s.Lp);
      u.A = (const double*)w.phi + (long)i0 * s.Lp; u.lda = s.Lp; u.a_bs = rowst;
      u.B = s.Upf + (long)sp * s.pk * s.Lp; u.ldb = s.Lp; u.b_bs = 0;
      u.C = w.W + (long)i0 * n + s.N; u.ldc = n; u.c_bs = n * n;
      u.batch = w.Wk;
      e = gemm_f64(u, false, true, false, st);
      if (e != hipSuccess) return e;
    }
  }
  hipLaunchKernelGGL(pf_mirror_kernel, dim3(w.Wk), dim3(256), 0, st, s, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Pfaffian by Parlett-Reid with partial pivoting, one workgroup per walker on
// the working copy X of G~: for k = 0, 2, ...  exchange row / column k+1 with
// the one of the largest |X[k][j]|, j > k (lowest index on ties; a sign
// change), multiply Pf by a = X[k][k+1], and with tau_j = X[k][j] / a update
//   X[i][j] -= tau_i X[k+1][j] - tau_j X[k+1][i]     (i, j >= k+2),
// a congruence by a unit lower triangular matrix, which leaves Pf unchanged.
// Rows k and k+1 are not written by that update, so it reads them in place.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pf_parlett_reid_kernel(SysDev s, WalkDev w) {
  __shared__ double X[kPfMaxN * kPfMaxN];   // 72 KB: the working copy stays in LDS
  __shared__ double pv[4];
  __shared__ int pj[4];
  __shared__ int piv;
  __shared__ double tau[kPfMaxN];
  const int wk = blockIdx.x, n = s.npf, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nw = blockDim.x >> 6;
  const double* G = w.W + (long)wk * n * n;
  for (int idx = tid; idx < n * n; idx += blockDim.x) X[idx] = G[idx];
  __syncthreads();
  double logabs = 0.0, sgn = 1.0;
  bool zero = false;
  for (int k = 0; k + 1 < n; k += 2) {
    // pivot: argmax_j>k |X[k][j]| (block reduction, lowest index on ties)
    double best = -1.0;
    int bj = k + 1;
    for (int j = k + 1 + tid; j < n; j += blockDim.x) {
      const double v = fabs(X[(long)k * n + j]);
      if (v > best) { best = v; bj = j; }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(best, o, 64);
      const int oj = __shfl_xor(bj, o, 64);
      if (ov > best || (ov == best && oj < bj)) { best = ov; bj = oj; }
    }
    if (lane == 0) { pv[wave] = best; pj[wave] = bj; }
    __syncthreads();
    if (tid == 0) {
      double b = pv[0];
      int j = pj[0];
      for (int q = 1; q < nw; ++q)
        if (pv[q] > b || (pv[q] == b && pj[q] < j)) { b = pv[q]; j = pj[q]; }
      piv = j;
    }
    __syncthreads();
    const int p = piv;
    if (p != k + 1) {
      // exchange rows k+1 and p, then columns k+1 and p
      for (int c = tid; c < n; c += blockDim.x) {
        const double a = X[(long)(k + 1) * n + c], b = X[(long)p * n + c];
        X[(long)(k + 1) * n + c] = b;
        X[(long)p * n + c] = a;
      }
      __syncthreads();
      for (int r = tid; r < n; r += blockDim.x) {
        const double a = X[(long)r * n + k + 1], b = X[(long)r * n + p];
        X[(long)r * n + k + 1] = b;
        X[(long)r * n + p] = a;
      }
      __syncthreads();
      sgn = -sgn;
    }
    const double a = X[(long)k * n + k + 1];
    if (a == 0.0) { zero = true; break; }   // uniform: every thread reads the same value
    logabs += log(fabs(a));
    if (a < 0.0) sgn = -sgn;
    const int m = n - (k + 2);
    if (m <= 0) break;
    for (int j = tid; j < m; j += blockDim.x) tau[j] = X[(long)k * n + k + 2 + j] / a;
    __syncthreads();
    const double* r1 = X + (long)(k + 1) * n + k + 2;
    for (int idx = tid; idx < m * m; idx += blockDim.x) {
      const int ii = idx / m, jj = idx % m;
      X[(long)(k + 2 + ii) * n + k + 2 + jj] += -tau[ii] * r1[jj] + tau[jj] * r1[ii];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (zero || (n & 1)) {
      w.logdet[wk] = -__builtin_inf();
      w.detsign[wk] = 0.0;
      w.singular[wk] = 1;
    } else {
      w.logdet[wk] = logabs;
      w.detsign[wk] = sgn;
    }
  }
}

hipError_t launch_pf_factor(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (s.npf > kPfMaxN) return hipErrorNotSupported;
  // G~^{-1} (and a singular flag) by Gauss-Jordan, then Pf overwrites log|det|, sign
  hipError_t e = launch_gj_inverse_n(w.Wk, s.npf, w.W, w.A, w.logdet, w.detsign, w.singular, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(pf_parlett_reid_kernel, dim3(w.Wk), dim3(256), 0, st, s, w);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cofactor vectors Y_i = sum_{j<N} (G~^{-1})_ji B^{s_i}_j + sum_l (G~^{-1})_{N+l,i} U^{s_i}_l
// ---------------------------------------------------------------------------
// Products sum_j X_ji B^{s_i}_j (+ unpaired rows) for any npf x npf matrix X
// (X = G~^{-1} gives the cofactor vectors; the adjoint uses other X).
hipError_t launch_pf_Y_products(const SysDev& s, const WalkDev& w, const double* X, double* out, hipStream_t st) {
  const long rowst = (long)s.N * s.Lp, n = s.npf;
  for (int sp = 0; sp < 2; ++sp) {
    const int i0 = sp == 0 ? 0 : s.nu, ni = sp == 0 ? s.nu : s.nd;
    if (ni == 0) continue;
    GemmArgs g = gemm_args(ni, s.Lp, s.N);
    g.A = X + i0; g.lda = n; g.a_bs = n * n;                    // stored [j][i]: op(A) = A^T
    g.B = sp == 0 ? (const double*)w.P : w.Bd; g.ldb = s.Lp; g.b_bs = rowst;
    g.C = out + (long)i0 * s.Lp; g.ldc = s.Lp; g.c_bs = rowst;
    g.batch = w.Wk;
    hipError_t e = gemm_f64(g, true, false, false, st);
    if (e != hipSuccess) return e;
    if (s.pk > 0) {
      GemmArgs u = gemm_args(ni, s.Lp, s.pk);
      u.A = X + (long)s.N * n + i0; u.lda = n; u.a_bs = n * n;
      u.B = s.Upf + (long)sp * s.pk * s.Lp; u.ldb = s.Lp; u.b_bs = 0;
      u.C = out + (long)i0 * s.Lp; u.ldc = s.Lp; u.c_bs = rowst;
      u.batch = w.Wk;
      u.accumulate = 1;
      e = gemm_f64(u, true, false, false, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_pf_Y_build(const SysDev& s, const WalkDev& w, hipStream_t st) {
  return launch_pf_Y_products(s, w, w.A, w.Yt, st);
}

// ---------------------------------------------------------------------------
// Proposal, one workgroup per walker: r', psi(r'), the Jastrow change, the new
// row g' of G~ (into w_new) and the ratio sum_j g'_j (G~^{-1})_je.
// ---------------------------------------------------------------------------
// With drift_o, also grad_e log|Psi| at r': column e of the updated inverse is
// the old one divided by the ratio (p (1 + q_e / rho) with q_e = 1 - rho and
// (G^{-1})_ee = 0), so grad_e log Pf(G') = sum_j (grad psi(r') . B_j) (G^{-1})_je / rho.
template <bool DRIFT>
__global__ void __launch_bounds__(512)
pf_propose_kernel(SysDev s, WalkDev w, int e, const double* __restrict__ r_new, const double* __restrict__ disp,
                  double* __restrict__ ratio_o, double* __restrict__ drift_o) {
  __shared__ double red[8];
  __shared__ double rn[3];
  __shared__ double part[kPfMaxN];
  __shared__ double gpart[DRIFT ? 3 * kPfMaxN : 1];
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = s.npf, N = s.N;
  const double* r = w.r + (long)wk * N * 3;
  if (tid < 3) {
    rn[tid] = disp ? r[3 * e + tid] + disp[(long)wk * 3 + tid] : r_new[(long)wk * 3 + tid];
    w.r_new[3 * wk + tid] = rn[tid];
  }
  __syncthreads();
  const double px = rn[0], py = rn[1], pz = rn[2];
  const double* psi = w.psi_new + (long)wk * s.Lp;
  const double* gpsi = w.gpsi_new + (long)wk * 3 * s.Lp;
  orbitals_at<DRIFT>(s, w, wk, px, py, pz);
  double dj, g0, g1, g2;
  jastrow_change<DRIFT>(s, w, wk, e, px, py, pz, dj, g0, g1, g2);
  const double dJ = block_sum_mv(dj, red);   // its barriers also publish psi
  if (DRIFT) { g0 = block_sum_mv(g0, red); g1 = block_sum_mv(g1, red); g2 = block_sum_mv(g2, red); }
  const bool up = e < s.nu;
  const double* B = (up ? (const double*)w.P : w.Bd) + (long)wk * N * s.Lp;
  const double* U = s.Upf + (up ? 0L : (long)s.pk * s.Lp);
  const double* Ai = w.A + (long)wk * n * n;
  double* wn = w.w_new + (long)wk * n;
  for (int j = wave; j < n; j += nw) {
    double v = 0.0, vx = 0.0, vy = 0.0, vz = 0.0;
    if (j != e) {
      const double* row = j < N ? B + (long)j * s.Lp : U + (long)(j - N) * s.Lp;
      for (int mu = lane; mu < s.Lp; mu += 64) {
        const double b = row[mu];
        v += psi[mu] * b;
        if (DRIFT) { vx += gpsi[mu] * b; vy += gpsi[s.Lp + mu] * b; vz += gpsi[2 * s.Lp + mu] * b; }
      }
      v = wave_sum(v);
      if (DRIFT) { vx = wave_sum(vx); vy = wave_sum(vy); vz = wave_sum(vz); }
    }
    if (lane == 0) {
      const double a = Ai[(long)j * n + e];
      wn[j] = v;
      part[j] = v * a;
      if (DRIFT) { gpart[3 * j] = vx * a; gpart[3 * j + 1] = vy * a; gpart[3 * j + 2] = vz * a; }
    }
  }
  __syncthreads();
  if (tid == 0) {
    double rd = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int j = 0; j < n; ++j) {   // fixed order
      rd += part[j];
      if (DRIFT) { gx += gpart[3 * j]; gy += gpart[3 * j + 1]; gz += gpart[3 * j + 2]; }
    }
    const double ratio = rd * exp(dJ);
    w.rdet[wk] = rd;
    w.dJ[wk] = dJ;
    w.ratio[wk] = ratio;
    if (ratio_o) ratio_o[wk] = ratio;
    if (DRIFT) {
      drift_o[3 * wk] = gx / rd + g0;
      drift_o[3 * wk + 1] = gy / rd + g1;
      drift_o[3 * wk + 2] = gz / rd + g2;
    }
  }
}

hipError_t launch_pf_propose(const SysDev& s, const WalkDev& w, int e, const double* r_new, const double* disp,
                             double* ratio, double* drift, hipStream_t st) {
  if (s.npf > kPfMaxN) return hipErrorNotSupported;
  // 8 waves per walker (block_sum_mv reduces over at most 8 waves)
  if (drift)
    hipLaunchKernelGGL(pf_propose_kernel<true>, dim3(w.Wk), dim3(512), 0, st, s, w, e, r_new, disp, ratio, drift);
  else
    hipLaunchKernelGGL(pf_propose_kernel<false>, dim3(w.Wk), dim3(512), 0, st, s, w, e, r_new, disp, ratio, drift);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Accept (host decisions acc[wk], or the device Metropolis test unif[wk] <
// ratio^2), one workgroup per walker: the rank-2 inverse update, row and
// column e of G~, electron e's basis row, B rows and position, the tracked
// log|Psi|, sign and Jastrow sum.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
pf_accept_kernel(SysDev s, WalkDev w, int e, const uint8_t* __restrict__ acc_in, const double* __restrict__ unif,
                 int32_t* __restrict__ cnt) {
  __shared__ double sp_[kPfMaxN], sq[kPfMaxN], sd[kPfMaxN];
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = s.npf, N = s.N;
  const double ratio = w.ratio[wk], rd = w.rdet[wk];
  const bool acc = unif ? (unif[wk] < ratio * ratio) : (acc_in[wk] != 0);
  if (tid == 0) w.acc[wk] = acc ? 1 : 0;
  if (!acc) return;   // uniform over the block
  double* G = w.W + (long)wk * n * n;
  double* Ai = w.A + (long)wk * n * n;
  const double* wn = w.w_new + (long)wk * n;
  for (int j = tid; j < n; j += blockDim.x) {
    sd[j] = wn[j] - G[(long)e * n + j];
    sp_[j] = Ai[(long)j * n + e];
  }
  __syncthreads();
  for (int i = wave; i < n; i += nw) {          // q = G^{-1} delta
    double v = 0.0;
    for (int j = lane; j < n; j += 64) v += Ai[(long)i * n + j] * sd[j];
    v = wave_sum(v);
    if (lane == 0) sq[i] = v;
  }
  __syncthreads();
  const double ir = 1.0 / rd;
  for (int idx = tid; idx < n * n; idx += blockDim.x) {
    const int i = idx / n, j = idx % n;
    Ai[idx] += (sp_[i] * sq[j] - sq[i] * sp_[j]) * ir;
  }
  for (int j = tid; j < n; j += blockDim.x) {
    G[(long)e * n + j] = wn[j];
    G[(long)j * n + e] = -wn[j];
  }
  // basis row and B rows of electron e (B^s_e = psi(r')^T K^{s s_e}, computed for
  // every walker by the product launched before this kernel)
  const double* pn = w.psi_new + (long)wk * s.Lp;
  const double* nb = w.pfB + (long)wk * 2 * s.Lp;
  double* ph = (double*)w.phi + ((long)wk * N + e) * s.Lp;
  double* bu = (double*)w.P + ((long)wk * N + e) * s.Lp;
  double* bd = w.Bd + ((long)wk * N + e) * s.Lp;
  for (int mu = tid; mu < s.Lp; mu += blockDim.x) {
    ph[mu] = pn[mu];
    bu[mu] = nb[mu];
    bd[mu] = nb[s.Lp + mu];
  }
  if (s.LJ) jastrow3_accept(s, w, wk, e);   // block-uniform
  if (tid == 0) {
    double* re = w.r + ((long)wk * N + e) * 3;
    re[0] = w.r_new[3 * wk]; re[1] = w.r_new[3 * wk + 1]; re[2] = w.r_new[3 * wk + 2];
    const double dJ = w.dJ[wk];
    w.logabs[wk] += log(fabs(rd)) + dJ;
    if (rd < 0.0) w.sign[wk] = -w.sign[wk];
    w.J[wk] += dJ;
    if (cnt) cnt[wk] += 1;
  }
}

hipError_t launch_pf_accept(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc, const double* unif,
                            int32_t* accept_count, hipStream_t st) {
  if (s.npf > kPfMaxN) return hipErrorNotSupported;
  // every walker moves electron e, of one spin: its two new B rows for all
  // walkers are the product psi_new [Wk x Lp] [K^{u s_e} | K^{d s_e}] (FP64 MFMA)
  // ([K^{u s_e} | K^{d s_e}] side by side: one product, 32 x 32 tiles)
  {
    GemmArgs g = gemm_args(w.Wk, 2 * s.Lp, s.Lp);
    g.A = w.psi_new; g.lda = s.Lp;
    g.B = e < s.nu ? s.Kcat_u : s.Kcat_d; g.ldb = 2 * s.Lp;
    g.C = w.pfB; g.ldc = 2 * s.Lp;
    const hipError_t err = gemm_f64(g, false, false, false, st);
    if (err != hipSuccess) return err;
  }
  hipLaunchKernelGGL(pf_accept_kernel, dim3(w.Wk), dim3(256), 0, st, s, w, e, acc, unif, accept_count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Logarithmic derivatives of the pairing coefficients, per walker, from
// d log Pf = 1/2 tr(G~^{-1} dG~) with G~^{-1} skew-symmetric (T = G~^{-1} blocks):
//   d / dA^{uu} = -1/2 Phi_u^T T_uu Phi_u      (skew: the gradient with respect to
//   d / dA^{dd} = -1/2 Phi_d^T T_dd Phi_d       a skew-symmetric matrix, written skew)
//   d / dA^{ud} = -Phi_u^T T_ud Phi_d
//   d / dU^s[:, l] = sum_{i of spin s} (G~^{-1})_{N+l, i} psi(r_i) = -Phi_s^T T_{s f}[:, l]
// as two FP64 MFMA products each (T Phi into the walkers' work rows, then Phi^T (T Phi)).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pf_scale_kernel(double* __restrict__ x, long n, double c) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] *= c;
}

hipError_t launch_pf_logderiv(const SysDev& s, const WalkDev& w, double* d_uu, double* d_dd, double* d_ud,
                              double* d_uup, double* d_udn, hipStream_t st) {
  const long n = s.npf, rowst = (long)s.N * s.Lp, L = s.L;
  const double* phi = (const double*)w.phi;
  // (row block rs of T) x Phi (column spin cs) -> pfT rows, then Phi_rs^T pfT -> out [L][L]
  auto pair = [&](int rs, int cs, double* out, double scale) -> hipError_t {
    const int r0 = rs == 0 ? 0 : s.nu, nr = rs == 0 ? s.nu : s.nd;
    const int c0 = cs == 0 ? 0 : s.nu, nc = cs == 0 ? s.nu : s.nd;
    if (!out) return hipSuccess;
    if (nr == 0 || nc == 0) return hipMemsetAsync(out, 0, sizeof(double) * L * L * w.Wk, st);
    GemmArgs g = gemm_args(nr, s.Lp, nc);
    g.A = w.A + (long)r0 * n + c0; g.lda = n; g.a_bs = n * n;
    g.B = phi + (long)c0 * s.Lp; g.ldb = s.Lp; g.b_bs = rowst;
    g.C = w.pfT; g.ldc = s.Lp; g.c_bs = rowst;
    g.batch = w.Wk;
    hipError_t e = gemm_f64(g, false, false, false, st);
    if (e != hipSuccess) return e;
    GemmArgs h = gemm_args((int)L, (int)L, nr);
    h.A = phi + (long)r0 * s.Lp; h.lda = s.Lp; h.a_bs = rowst;   // stored [i][mu]: op = A^T
    h.B = w.pfT; h.ldb = s.Lp; h.b_bs = rowst;
    h.C = out; h.ldc = L; h.c_bs = L * L;
    h.batch = w.Wk;
    e = gemm_f64(h, true, false, false, st);
    if (e != hipSuccess) return e;
    const long tot = (long)w.Wk * L * L;
    hipLaunchKernelGGL(pf_scale_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, out, tot, scale);
    return hipGetLastError();
  };
  hipError_t e = pair(0, 0, d_uu, -0.5);
  if (e == hipSuccess) e = pair(1, 1, d_dd, -0.5);
  if (e == hipSuccess) e = pair(0, 1, d_ud, -1.0);
  if (e != hipSuccess || s.pk == 0) return e;
  // unpaired orbitals: out_s[mu][l] = sum_{i of s} (G~^{-1})_{N+l, i} psi_mu(r_i)
  for (int sp = 0; sp < 2; ++sp) {
    double* out = sp == 0 ? d_uup : d_udn;
    const int r0 = sp == 0 ? 0 : s.nu, nr = sp == 0 ? s.nu : s.nd;
    if (!out) continue;
    if (nr == 0) {
      e = hipMemsetAsync(out, 0, sizeof(double) * L * s.pk * w.Wk, st);
      if (e != hipSuccess) return e;
      continue;
    }
    GemmArgs g = gemm_args((int)L, s.pk, nr);
    g.A = phi + (long)r0 * s.Lp; g.lda = s.Lp; g.a_bs = rowst;   // op = Phi_s^T
    g.B = w.A + (long)s.N * n + r0; g.ldb = n; g.b_bs = n * n;   // stored [l][i]: op = (.)^T
    g.C = out; g.ldc = s.pk; g.c_bs = L * s.pk;
    g.batch = w.Wk;
    e = gemm_f64(g, true, true, false, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// New pairing coefficients from device arrays (any may be null): A^{ud} (lam,
// [L][L]) -> K^{ud} = A^{ud T}, K^{du} = -A^{ud}; A^{uu}, A^{dd} -> K^{uu},
// K^{dd} (transposed); unpaired orbitals -> Upf; and the side-by-side copies
// [K^{uu} | K^{du}], [K^{ud} | K^{dd}] used by the accept.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
pf_set_kernel(SysDev s, const double* __restrict__ lam, const double* __restrict__ uu, const double* __restrict__ dd,
              const double* __restrict__ upu, const double* __restrict__ upd) {
  const long L = s.L, Lp = s.Lp;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx < L * L) {
    const long a = idx / L, b = idx % L;
    if (lam) {
      const double v = lam[idx];
      s.Kud[b * Lp + a] = v;
      s.Kdu[a * Lp + b] = -v;
      s.Kcat_d[b * 2 * Lp + a] = v;
      s.Kcat_u[a * 2 * Lp + Lp + b] = -v;
    }
    if (uu) { s.Kuu[b * Lp + a] = uu[idx]; s.Kcat_u[b * 2 * Lp + a] = uu[idx]; }
    if (dd) { s.Kdd[b * Lp + a] = dd[idx]; s.Kcat_d[b * 2 * Lp + Lp + a] = dd[idx]; }
  }
  if (idx < L * s.pk) {
    const long mu = idx / s.pk, l = idx % s.pk;
    if (upu) s.Upf[l * Lp + mu] = upu[idx];
    if (upd) s.Upf[((long)s.pk + l) * Lp + mu] = upd[idx];
  }
}

hipError_t launch_pf_set(const SysDev& s, const double* lam, const double* uu, const double* dd, const double* upu,
                         const double* upd, hipStream_t st) {
  const long n = (long)s.L * s.L > (long)s.L * s.pk ? (long)s.L * s.L : (long)s.L * s.pk;
  hipLaunchKernelGGL(pf_set_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, lam, uu, dd, upu, upd);
  return hipGetLastError();
}

}  // namespace qmc
