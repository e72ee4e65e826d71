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
#include "internal.h"

namespace qmc {

__device__ double block_sum_mv(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += red[k];
  __syncthreads();
  return t;
}

// Jastrow terms of electron e at position p: value and gradient (in g).
__device__ void jastrow_one(const SysDev& s, const double* r, int e, double px, double py, double pz,
                            bool want_grad, double& val, double& gx, double& gy, double& gz) {
  val = 0.0; gx = gy = gz = 0.0;
  if (s.j1_form) {
    for (int a = threadIdx.x; a < s.n_nuc; a += blockDim.x) {
      const double dx = px - s.R[3 * a], dy = py - s.R[3 * a + 1], dz = pz - s.R[3 * a + 2];
      const double ria = sqrt(dx * dx + dy * dy + dz * dz);
      double f, f1, f2;
      j1_radial(s.j1_form, s.Z[a], s.j1_b[a], ria, f, f1, f2);
      val += f;
      if (want_grad) { const double q = f1 / ria; gx += q * dx; gy += q * dy; gz += q * dz; }
    }
  }
  if (s.j2_form) {
    const bool up_e = e < s.nu;
    for (int j = threadIdx.x; j < s.N; j += blockDim.x) {
      if (j == e) continue;
      const double dx = px - r[3 * j], dy = py - r[3 * j + 1], dz = pz - r[3 * j + 2];
      const double rij = sqrt(dx * dx + dy * dy + dz * dz);
      double v, v1, v2;
      j2_radial(s.j2_form, s.j2, up_e == (j < s.nu), rij, v, v1, v2);
      val += v;
      if (want_grad) { const double q = v1 / rij; gx += q * dx; gy += q * dy; gz += q * dz; }
    }
  }
}

template <typename T, bool DRIFT>
__global__ void __launch_bounds__(256)
propose_kernel(SysDev s, WalkDev w, int e, const double* __restrict__ r_new_in,
               const double* __restrict__ disp, double* __restrict__ ratio_o,
               double* __restrict__ drift_o) {
  extern __shared__ double sm[];
  double* psi = sm;                          // [L]
  double* gpsi = psi + s.Lp;                 // [3][L] when DRIFT
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  double* wn = gpsi + (DRIFT ? 3 * s.Lp : 0); // [nmax]
  double* gwn = wn + nmax;                    // [3][nmax] when DRIFT
  __shared__ double red[8];
  __shared__ double rn[3];
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* r = w.r + (long)wk * s.N * 3;
  if (tid < 3) rn[tid] = disp ? r[3 * e + tid] + disp[3 * (long)wk + tid] : r_new_in[3 * (long)wk + tid];
  __syncthreads();
  const double px = rn[0], py = rn[1], pz = rn[2];
  double* psi_g = w.psi_new + (long)wk * s.Lp;
  for (int mu = tid; mu < s.L; mu += blockDim.x) {
    if (DRIFT) {
      double v, gx, gy, gz, lp;
      basis_vgl(s, mu, px, py, pz, v, gx, gy, gz, lp);
      psi[mu] = v; gpsi[mu] = gx; gpsi[s.Lp + mu] = gy; gpsi[2 * s.Lp + mu] = gz;
      psi_g[mu] = v;
    } else {
      const double v = basis_value(s, mu, px, py, pz);
      psi[mu] = v;
      psi_g[mu] = v;
    }
  }
  __syncthreads();
  const bool up = e < s.nu;
  const int row0 = up ? s.nu : 0;
  const int nrow = up ? s.nd : s.nu;
  const T* Pw = (const T*)w.P + ((long)wk * s.N + row0) * s.Lp;
  for (int j = wave; j < nrow; j += 4) {
    const T* prow = Pw + (long)j * s.Lp;
    double a0 = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
    for (int mu = lane; mu < s.L; mu += 64) {
      const double p = (double)prow[mu];
      a0 += p * psi[mu];
      if (DRIFT) { ax += p * gpsi[mu]; ay += p * gpsi[s.Lp + mu]; az += p * gpsi[2 * s.Lp + mu]; }
    }
    a0 = wave_sum(a0);
    if (DRIFT) { ax = wave_sum(ax); ay = wave_sum(ay); az = wave_sum(az); }
    if (lane == 0) {
      wn[j] = a0;
      if (DRIFT) { gwn[j] = ax; gwn[nmax + j] = ay; gwn[2 * nmax + j] = az; }
    }
  }
  __syncthreads();
  const double* Aw = w.A + (long)wk * s.nd * s.nu;
  double part = 0.0, pgx = 0.0, pgy = 0.0, pgz = 0.0;
  for (int j = tid; j < nrow; j += blockDim.x) {
    const double a = up ? Aw[(long)j * s.nu + e] : Aw[(long)(e - s.nu) * s.nu + j];
    part += wn[j] * a;
    if (DRIFT) { pgx += gwn[j] * a; pgy += gwn[nmax + j] * a; pgz += gwn[2 * nmax + j] * a; }
  }
  const double rdet = block_sum_mv(part, red);
  double jn, gxn, gyn, gzn, jo, d0, d1, d2;
  jastrow_one(s, r, e, px, py, pz, DRIFT, jn, gxn, gyn, gzn);
  jastrow_one(s, r, e, r[3 * e], r[3 * e + 1], r[3 * e + 2], false, jo, d0, d1, d2);
  const double dJ = block_sum_mv(jn - jo, red);
  double Gx = 0.0, Gy = 0.0, Gz = 0.0, Jx = 0.0, Jy = 0.0, Jz = 0.0;
  if (DRIFT) {
    Gx = block_sum_mv(pgx, red); Gy = block_sum_mv(pgy, red); Gz = block_sum_mv(pgz, red);
    Jx = block_sum_mv(gxn, red); Jy = block_sum_mv(gyn, red); Jz = block_sum_mv(gzn, red);
  }
  double* wn_g = w.w_new + (long)wk * nmax;
  for (int j = tid; j < nrow; j += blockDim.x) wn_g[j] = wn[j];
  if (tid == 0) {
    const double ratio = rdet * exp(dJ);
    w.rdet[wk] = rdet;
    w.dJ[wk] = dJ;
    w.ratio[wk] = ratio;
    w.r_new[3 * wk] = px; w.r_new[3 * wk + 1] = py; w.r_new[3 * wk + 2] = pz;
    if (ratio_o) ratio_o[wk] = ratio;
    if (DRIFT && drift_o) {
      // grad of log|det| for the moved electron at r' uses the updated inverse,
      // whose column e equals the old one divided by the determinant ratio
      drift_o[3 * wk] = Gx / rdet + Jx;
      drift_o[3 * wk + 1] = Gy / rdet + Jy;
      drift_o[3 * wk + 2] = Gz / rdet + Jz;
    }
  }
}

hipError_t launch_propose(const SysDev& s, const WalkDev& w, int e, const double* r_new,
                          const double* disp, double* ratio, double* drift_new, hipStream_t st) {
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  const bool drift = drift_new != nullptr;
  const size_t shm = sizeof(double) * ((drift ? 4 : 1) * (size_t)s.Lp + (drift ? 4 : 1) * (size_t)nmax);
  const bool f32 = s.precision == QMC_W_FP32;
  if (drift) {
    if (f32) hipLaunchKernelGGL((propose_kernel<float, true>), dim3(w.Wk), dim3(256), shm, st, s, w, e, r_new, disp, ratio, drift_new);
    else hipLaunchKernelGGL((propose_kernel<double, true>), dim3(w.Wk), dim3(256), shm, st, s, w, e, r_new, disp, ratio, drift_new);
  } else {
    if (f32) hipLaunchKernelGGL((propose_kernel<float, false>), dim3(w.Wk), dim3(256), shm, st, s, w, e, r_new, disp, ratio, drift_new);
    else hipLaunchKernelGGL((propose_kernel<double, false>), dim3(w.Wk), dim3(256), shm, st, s, w, e, r_new, disp, ratio, drift_new);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Accept: decide (device Metropolis, u < ratio^2, when unif is given) and
// apply the rank-1 Sherman-Morrison update of A = W^{-1} in FP64:
//   up e   (row e of W replaced by w'):    A <- A - A[:,e] (delta^T A) / R
//   down e (column e of W replaced by w'): A <- A - (A delta) A[e,:] / R
// with delta = w' - (old row/column) and R = det W'/det W.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256)
accept_kernel(SysDev s, WalkDev w, int e, const uint8_t* __restrict__ acc_in,
              const double* __restrict__ unif, int32_t* __restrict__ accept_count) {
  extern __shared__ double sm[];
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  double* delta = sm;          // [nmax]
  double* coef = delta + nmax; // [nmax]
  double* save = coef + nmax;  // [nmax]
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  bool acc;
  if (unif) {
    const double q = w.ratio[wk];
    acc = unif[wk] < q * q;
  } else {
    acc = acc_in[wk] != 0;
  }
  if (tid == 0) w.acc[wk] = acc ? 1 : 0;
  if (!acc) return;
  const double R = w.rdet[wk];
  const double invR = 1.0 / R;
  const bool up = e < s.nu;
  double* Aw = w.A + (long)wk * s.nd * s.nu;
  double* Ww = w.W + (long)wk * s.nu * s.nd;
  const double* wn = w.w_new + (long)wk * nmax;
  if (up) {
    for (int j = tid; j < s.nd; j += blockDim.x) {
      delta[j] = wn[j] - Ww[(long)e * s.nd + j];
      save[j] = Aw[(long)j * s.nu + e];
    }
    __syncthreads();
    for (int k = tid; k < s.nu; k += blockDim.x) {
      double t = 0.0;
      for (int j = 0; j < s.nd; ++j) t += delta[j] * Aw[(long)j * s.nu + k];
      coef[k] = t * invR;
    }
    __syncthreads();
    for (int idx = tid; idx < s.nd * s.nu; idx += blockDim.x) {
      const int j = idx / s.nu, k = idx - (idx / s.nu) * s.nu;
      Aw[idx] -= save[j] * coef[k];
    }
    for (int j = tid; j < s.nd; j += blockDim.x) Ww[(long)e * s.nd + j] = wn[j];
  } else {
    const int ed = e - s.nu;
    for (int i = tid; i < s.nu; i += blockDim.x) {
      delta[i] = wn[i] - Ww[(long)i * s.nd + ed];
      save[i] = Aw[(long)ed * s.nu + i];
    }
    __syncthreads();
    for (int j = wave; j < s.nd; j += 4) {
      double t = 0.0;
      for (int i = lane; i < s.nu; i += 64) t += Aw[(long)j * s.nu + i] * delta[i];
      t = wave_sum(t);
      if (lane == 0) coef[j] = t * invR;
    }
    __syncthreads();
    for (int idx = tid; idx < s.nd * s.nu; idx += blockDim.x) {
      const int j = idx / s.nu, k = idx - (idx / s.nu) * s.nu;
      Aw[idx] -= coef[j] * save[k];
    }
    for (int i = tid; i < s.nu; i += blockDim.x) Ww[(long)i * s.nd + ed] = wn[i];
  }
  T* prow = (T*)w.phi + ((long)wk * s.N + e) * s.Lp;
  const double* pn = w.psi_new + (long)wk * s.Lp;
  for (int mu = tid; mu < s.L; mu += blockDim.x) prow[mu] = (T)pn[mu];
  if (tid == 0) {
    double* re = w.r + ((long)wk * s.N + e) * 3;
    re[0] = w.r_new[3 * wk]; re[1] = w.r_new[3 * wk + 1]; re[2] = w.r_new[3 * wk + 2];
    const double dJ = w.dJ[wk];
    w.logabs[wk] += log(fabs(R)) + dJ;
    if (R < 0.0) w.sign[wk] = -w.sign[wk];
    w.J[wk] += dJ;
    if (accept_count) accept_count[wk] += 1;
  }
}

hipError_t launch_accept(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc,
                         hipStream_t st) {
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  const size_t shm = sizeof(double) * 3 * (size_t)nmax;
  if (s.precision == QMC_W_FP32)
    hipLaunchKernelGGL(accept_kernel<float>, dim3(w.Wk), dim3(256), shm, st, s, w, e, acc, nullptr, nullptr);
  else
    hipLaunchKernelGGL(accept_kernel<double>, dim3(w.Wk), dim3(256), shm, st, s, w, e, acc, nullptr, nullptr);
  return hipGetLastError();
}

hipError_t launch_metropolis_accept(const SysDev& s, const WalkDev& w, int e, const double* unif,
                                    int32_t* accept_count, hipStream_t st) {
  const int nmax = s.nu > s.nd ? s.nu : s.nd;
  const size_t shm = sizeof(double) * 3 * (size_t)nmax;
  if (s.precision == QMC_W_FP32)
    hipLaunchKernelGGL(accept_kernel<float>, dim3(w.Wk), dim3(256), shm, st, s, w, e, nullptr, unif, accept_count);
  else
    hipLaunchKernelGGL(accept_kernel<double>, dim3(w.Wk), dim3(256), shm, st, s, w, e, nullptr, unif, accept_count);
  return hipGetLastError();
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
