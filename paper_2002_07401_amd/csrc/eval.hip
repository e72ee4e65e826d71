// From-scratch evaluation kernels: basis values, the per-electron determinant
// derivatives, and the Jastrow / Coulomb / local-energy assembly.
#include "internal.h"

namespace qmc {

// ---------------------------------------------------------------------------
// Phi[w][i][mu] = psi_mu(r_i)  (eq. gaussian), zero for padding mu >= L.
// One workgroup per electron row; consecutive threads write consecutive mu.
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) basis_values_kernel(SysDev s, const double* __restrict__ r,
                                                           T* __restrict__ phi) {
  const long row = blockIdx.x;   // w * N + i
  const double px = r[3 * row], py = r[3 * row + 1], pz = r[3 * row + 2];
  T* out = phi + row * s.Lp;
  for (int mu = threadIdx.x; mu < s.Lp; mu += blockDim.x)
    out[mu] = (T)(mu < s.L ? basis_value(s, mu, px, py, pz) : 0.0);
}

// FP64 values plus (lo not null) their FP32 or BF16 copy (the rows the moves stream).  With
// ephi, also the exponent floor(log2 max_mu |psi_mu(r_i)|) of the row (0 for a
// row of zeros), the scale of its int8 digits: up electron i of walker w at
// ephi[w * n_up + i], down electron j at ephi[Wk * n_up + w * n_dn + j].
template <typename T2>
__global__ void __launch_bounds__(256) basis_values_dual_kernel(SysDev s, const double* __restrict__ r,
                                                                double* __restrict__ phi, T2* __restrict__ lo,
                                                                int* __restrict__ ephi, int Wk) {
  __shared__ double red[4];
  const long row = blockIdx.x;   // w * N + i
  const double px = r[3 * row], py = r[3 * row + 1], pz = r[3 * row + 2];
  double* out = phi + row * s.Lp;
  T2* out2 = lo ? lo + row * s.Lp : nullptr;
  double mx = 0.0;
  for (int mu = threadIdx.x; mu < s.Lp; mu += blockDim.x) {
    const double v = mu < s.L ? basis_value(s, mu, px, py, pz) : 0.0;
    out[mu] = v;
    if (out2) out2[mu] = (T2)v;
    mx = fmax(mx, fabs(v));
  }
  if (!ephi) return;   // uniform
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) m = fmax(m, red[k]);
    const long w = row / s.N, i = row % s.N;
    const long at = i < s.nu ? w * s.nu + i : (long)Wk * s.nu + w * s.nd + (i - s.nu);
    ephi[at] = m > 0.0 ? ilogb(m) : 0;
  }
}

// Contracted orbitals: the row's primitive values are staged in LDS, then
// phi_c = sum_t C_t psi_{idx_t} (a contraction mixes primitives of one row only).
// lo (optional, with T = double): the FP32 or BF16 copy (T2) of the same row.
template <typename T, typename T2 = float>
__global__ void __launch_bounds__(256) contracted_values_kernel(SysDev s, const double* __restrict__ r,
                                                                T* __restrict__ phi, T2* __restrict__ lo) {
  __shared__ double q[kMaxLq];
  const long row = blockIdx.x;   // w * N + i
  const double px = r[3 * row], py = r[3 * row + 1], pz = r[3 * row + 2];
  for (int mu = threadIdx.x; mu < s.Lq; mu += blockDim.x) q[mu] = basis_value(s, mu, px, py, pz);
  __syncthreads();
  T* out = phi + row * s.Lp;
  for (int c = threadIdx.x; c < s.Lp; c += blockDim.x) {
    double v = 0.0;
    if (c < s.L)
      for (int k = s.con_ptr[c]; k < s.con_ptr[c + 1]; ++k) v += s.con_coef[k] * q[s.con_idx[k]];
    out[c] = (T)v;
    if (lo) lo[row * s.Lp + c] = (T2)v;
  }
}

hipError_t launch_basis_values(const SysDev& s, const WalkDev& w, hipStream_t st, void* lo, bool lo_bf16,
                               int* ephi) {
  const dim3 grid((unsigned)((long)w.Wk * s.N));
  // FP64 values with a low-precision copy and / or the rows' digit exponents
  const bool dual = (lo || ephi) && !s.f32();
  if (dual && s.Lq == 0) {
    if (lo_bf16)
      hipLaunchKernelGGL(basis_values_dual_kernel<bf16s>, grid, dim3(256), 0, st, s, w.r, (double*)w.phi, (bf16s*)lo,
                         ephi, w.Wk);
    else
      hipLaunchKernelGGL(basis_values_dual_kernel<float>, grid, dim3(256), 0, st, s, w.r, (double*)w.phi, (float*)lo,
                         ephi, w.Wk);
    return hipGetLastError();
  }
  if (ephi) return hipErrorInvalidValue;   // exponents come with the FP64 + copy form only
  if (s.Lq > 0) {
    if (s.Lq > kMaxLq) return hipErrorNotSupported;
    if (dual && lo_bf16)
      hipLaunchKernelGGL((contracted_values_kernel<double, bf16s>), grid, dim3(256), 0, st, s, w.r, (double*)w.phi,
                         (bf16s*)lo);
    else if (dual)
      hipLaunchKernelGGL((contracted_values_kernel<double, float>), grid, dim3(256), 0, st, s, w.r, (double*)w.phi,
                         (float*)lo);
    else if (s.bf16())
      hipLaunchKernelGGL((contracted_values_kernel<bf16s>), grid, dim3(256), 0, st, s, w.r, (bf16s*)w.phi,
                         (float*)nullptr);
    else if (s.f32())
      hipLaunchKernelGGL((contracted_values_kernel<float>), grid, dim3(256), 0, st, s, w.r, (float*)w.phi,
                         (float*)nullptr);
    else
      hipLaunchKernelGGL((contracted_values_kernel<double>), grid, dim3(256), 0, st, s, w.r, (double*)w.phi,
                         (float*)nullptr);
    return hipGetLastError();
  }
  if (s.bf16())
    hipLaunchKernelGGL(basis_values_kernel<bf16s>, grid, dim3(256), 0, st, s, w.r, (bf16s*)w.phi);
  else if (s.f32())
    hipLaunchKernelGGL(basis_values_kernel<float>, grid, dim3(256), 0, st, s, w.r, (float*)w.phi);
  else
    hipLaunchKernelGGL(basis_values_kernel<double>, grid, dim3(256), 0, st, s, w.r, (double*)w.phi);
  return hipGetLastError();
}

// FP32 or BF16 copies of FP64 arrays (padding included), 4 elements per thread.
template <typename T>
__global__ void __launch_bounds__(256) downcast_kernel(const double* __restrict__ src, T* __restrict__ dst, long n) {
  const long i = 4 * ((long)blockIdx.x * blockDim.x + threadIdx.x);
  if (i + 3 < n) {
    const double4 v = *reinterpret_cast<const double4*>(src + i);
    dst[i] = (T)v.x; dst[i + 1] = (T)v.y; dst[i + 2] = (T)v.z; dst[i + 3] = (T)v.w;
  } else {
    for (long k = i; k < n; ++k) dst[k] = (T)src[k];
  }
}

hipError_t launch_downcast(const double* src, void* dst, bool to_bf16, long n, hipStream_t st) {
  const long threads = (n + 3) / 4;
  const dim3 grid((unsigned)((threads + 255) / 256));
  if (to_bf16) hipLaunchKernelGGL(downcast_kernel<bf16s>, grid, dim3(256), 0, st, src, (bf16s*)dst, n);
  else hipLaunchKernelGGL(downcast_kernel<float>, grid, dim3(256), 0, st, src, (float*)dst, n);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Row dots of the derivative rows with the cofactor vectors:
//   D[w][i][0:3] = sum_mu grad psi_mu(r_i) Yt[w][i][mu]  = grad_i det / det
//   D[w][i][3]   = sum_mu lap  psi_mu(r_i) Yt[w][i][mu]  = lap_i  det / det
// Exact because W depends on r_i through one row (or column) only.  The basis
// derivatives are recomputed here instead of being stored.  One wave per row.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) rowdot_kernel(SysDev s, int rows, const double* __restrict__ r,
                                                     const double* __restrict__ Yt,
                                                     double* __restrict__ D) {
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const double px = r[3 * row], py = r[3 * row + 1], pz = r[3 * row + 2];
  const double* y = Yt + row * s.Lp;
  double sx = 0.0, sy = 0.0, sz = 0.0, sl = 0.0;
  // contracted orbitals: sum_c y_c D phi_c = sum_mu (sum_c C[mu][c] y_c) D psi_mu
  const int nb = s.nprim();
  for (int mu = lane; mu < nb; mu += 64) {
    double v, gx, gy, gz, lp;
    basis_vgl(s, mu, px, py, pz, v, gx, gy, gz, lp);
    const double yy = s.Lq ? prim_weight(s, mu, y) : y[mu];
    sx += gx * yy; sy += gy * yy; sz += gz * yy; sl += lp * yy;
  }
  sx = wave_sum(sx); sy = wave_sum(sy); sz = wave_sum(sz); sl = wave_sum(sl);
  if (lane == 0) {
    D[4 * row] = sx; D[4 * row + 1] = sy; D[4 * row + 2] = sz; D[4 * row + 3] = sl;
  }
}

hipError_t launch_rowdots(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int rows = w.Wk * s.N;
  hipLaunchKernelGGL(rowdot_kernel, dim3((rows + 3) / 4), dim3(256), 0, st, s, rows, w.r, w.Yt, w.D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Block-wide FP64 sum (fixed order, deterministic).
// ---------------------------------------------------------------------------
__device__ double block_sum(double v, double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double t = 0.0;
  for (int k = 0; k < nw; ++k) t += red[k];
  return t;
}

// ---------------------------------------------------------------------------
// Jastrow J = J1 + J2 with per-electron gradient and Laplacian, the Coulomb
// potential, and the assembly of log|Psi|, drift and local energy:
//   drift_i = grad_i det/det + grad_i J
//   e_kin   = -1/2 sum_i [ lap_i det/det + 2 grad_i det/det . grad_i J
//                          + lap_i J + |grad_i J|^2 ]
//   e_loc   = e_kin + V     (local energy, VMC section)
// One workgroup of kAssembleThreads per walker.  The electrons go in chunks
// of at most the block size; a chunk of nc electrons is spread over G =
// blockDim / nc groups of threads, group g taking the nuclei and partners a,
// j = g, g + G, ... of every electron (so that short chunks keep most threads
// busy), and each electron's gradient and Laplacian of J add the groups'
// partial sums in order of g.
// ---------------------------------------------------------------------------
constexpr int kAssembleThreads = 512;
__global__ void __launch_bounds__(kAssembleThreads)
jastrow_assemble_kernel(SysDev s, WalkDev w, double* __restrict__ logabs_o, double* __restrict__ sign_o,
                        double* __restrict__ drift_o, double* __restrict__ ekin_o,
                        double* __restrict__ eloc_o, int32_t* __restrict__ status_o) {
  __shared__ double red[3 * (kAssembleThreads / 64)];
  __shared__ double part[kAssembleThreads][4];
  const int wk = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
  const double* r = w.r + (long)wk * s.N * 3;
  double Jp = 0.0, Vp = 0.0, Kp = 0.0;
  bool bad = false;
  for (int c0 = 0; c0 < s.N; c0 += T) {
    const int nc = min(s.N - c0, T);
    const int G = max(1, T / nc);
    const int g = tid / nc, i = c0 + tid % nc;
    if (g < G) {
      const double xi = r[3 * i], yi = r[3 * i + 1], zi = r[3 * i + 2];
      double gx = 0.0, gy = 0.0, gz = 0.0, h = 0.0;
      for (int a = g; a < s.n_nuc; a += G) {
        const double dx = xi - s.R[3 * a], dy = yi - s.R[3 * a + 1], dz = zi - s.R[3 * a + 2];
        const double ria = sqrt(dx * dx + dy * dy + dz * dz);
        Vp -= s.Z[a] / ria;
        if (s.j1_form) {
          double f, f1, f2;
          j1_radial(s.j1_form, s.Z[a], s.j1_b[a], ria, f, f1, f2);
          const double q = f1 / ria;
          Jp += f;
          gx += q * dx; gy += q * dy; gz += q * dz;
          h += f2 + 2.0 * q;
        }
      }
      const bool up_i = i < s.nu;
      for (int j = g; j < s.N; j += G) {
        if (j == i) continue;
        const double dx = xi - r[3 * j], dy = yi - r[3 * j + 1], dz = zi - r[3 * j + 2];
        const double rij = sqrt(dx * dx + dy * dy + dz * dz);
        Vp += 0.5 / rij;
        if (s.j2_form) {
          double v, v1, v2;
          j2_radial(s.j2_form, s.j2d, up_i == (j < s.nu), rij, v, v1, v2);
          const double q = v1 / rij;
          Jp += 0.5 * v;
          gx += q * dx; gy += q * dy; gz += q * dz;
          h += v2 + 2.0 * q;
        }
      }
      part[tid][0] = gx; part[tid][1] = gy; part[tid][2] = gz; part[tid][3] = h;
    }
    __syncthreads();
    if (tid < nc) {   // electron i = c0 + tid
      double gx = 0.0, gy = 0.0, gz = 0.0, h = 0.0;
      for (int q = 0; q < G; ++q) {
        const double* pq = part[q * nc + tid];
        gx += pq[0]; gy += pq[1]; gz += pq[2]; h += pq[3];
      }
      if (s.LJ) {   // Jastrow-basis terms (one-body inhomogeneous, three/four-body)
        const double* e3 = w.j3e + ((long)wk * s.N + i) * 5;
        Jp += e3[0];
        gx += e3[1]; gy += e3[2]; gz += e3[3];
        h += e3[4];
      }
      const double* Di = w.D + ((long)wk * s.N + i) * 4;
      const double ddx = Di[0], ddy = Di[1], ddz = Di[2], dl = Di[3];
      Kp += dl + 2.0 * (ddx * gx + ddy * gy + ddz * gz) + h + gx * gx + gy * gy + gz * gz;
      double* gj = w.gJ + ((long)wk * s.N + i) * 4;
      gj[0] = gx; gj[1] = gy; gj[2] = gz; gj[3] = h;
      double* dd = w.drift + ((long)wk * s.N + i) * 3;
      dd[0] = ddx + gx; dd[1] = ddy + gy; dd[2] = ddz + gz;
      if (drift_o) {
        double* o = drift_o + ((long)wk * s.N + i) * 3;
        o[0] = ddx + gx; o[1] = ddy + gy; o[2] = ddz + gz;
        bad |= !isfinite(o[0]) || !isfinite(o[1]) || !isfinite(o[2]);
      }
    }
    __syncthreads();   // the chunk's partial sums are read before the next chunk writes them
  }
  // nucleus-nucleus repulsion
  for (int p = threadIdx.x; p < s.n_nuc * s.n_nuc; p += blockDim.x) {
    const int a = p / s.n_nuc, b = p % s.n_nuc;
    if (b <= a) continue;
    const double dx = s.R[3 * a] - s.R[3 * b], dy = s.R[3 * a + 1] - s.R[3 * b + 1],
                 dz = s.R[3 * a + 2] - s.R[3 * b + 2];
    Vp += s.Z[a] * s.Z[b] / sqrt(dx * dx + dy * dy + dz * dz);
  }
  constexpr int NW = kAssembleThreads / 64;
  const double J = block_sum(Jp, red);
  const double V = block_sum(Vp, red + NW);
  const double K = block_sum(Kp, red + 2 * NW);
  __shared__ int bad_s;
  if (threadIdx.x == 0) bad_s = 0;
  __syncthreads();
  if (bad) atomicOr(&bad_s, 1);
  __syncthreads();
  if (threadIdx.x == 0) {
    const int sing = w.singular[wk];
    const double ekin = -0.5 * K;
    const double eloc = ekin + V;
    const double la = sing ? -__builtin_inf() : w.logdet[wk] + J;
    const double sg = w.detsign[wk];
    int st = 0;
    if (sing) st = 1;
    else if (!isfinite(la) || !isfinite(eloc) || bad_s) st = 2;
    w.logabs[wk] = la;
    w.sign[wk] = sg;
    w.J[wk] = J;
    w.wm[wk] = 0;   // the fresh inverse has no delayed updates
    if (logabs_o) logabs_o[wk] = la;
    if (sign_o) sign_o[wk] = sg;
    if (ekin_o) ekin_o[wk] = ekin;
    if (eloc_o) eloc_o[wk] = eloc;
    if (status_o) status_o[wk] = st;
  }
}

hipError_t launch_jastrow_assemble(const SysDev& s, const WalkDev& w, double* logabs, double* sign,
                                   double* drift, double* e_kin, double* e_loc, int32_t* status,
                                   hipStream_t st) {
  hipLaunchKernelGGL(jastrow_assemble_kernel, dim3(w.Wk), dim3(kAssembleThreads), 0, st, s, w, logabs, sign, drift,
                     e_kin, e_loc, status);
  return hipGetLastError();
}

// Copy the basis matrix out as FP64 (inspection).
template <typename T>
__global__ void export_phi_kernel(SysDev s, long rows, const T* __restrict__ phi, double* __restrict__ dst) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= rows * s.L) return;
  const long row = idx / s.L, mu = idx % s.L;
  dst[idx] = (double)phi[row * s.Lp + mu];
}

hipError_t launch_export_phi(const SysDev& s, const WalkDev& w, double* dst, hipStream_t st) {
  const long rows = (long)w.Wk * s.N;
  const unsigned nb = (unsigned)((rows * s.L + 255) / 256);
  if (s.bf16())
    hipLaunchKernelGGL(export_phi_kernel<bf16s>, dim3(nb), dim3(256), 0, st, s, rows, (const bf16s*)w.phi, dst);
  else if (s.f32())
    hipLaunchKernelGGL(export_phi_kernel<float>, dim3(nb), dim3(256), 0, st, s, rows, (const float*)w.phi, dst);
  else
    hipLaunchKernelGGL(export_phi_kernel<double>, dim3(nb), dim3(256), 0, st, s, rows, (const double*)w.phi, dst);
  return hipGetLastError();
}

// Scatter a dense [L][L] Lambda into the padded Lambda, its transpose and the
// FP32 copies.
__global__ void set_lambda_kernel(SysDev s, const double* __restrict__ lam) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)s.L * s.L) return;
  const int i = (int)(idx / s.L), j = (int)(idx % s.L);
  const double v = lam[idx];
  s.lam[(long)i * s.Lp + j] = v;
  s.lamT[(long)j * s.Lp + i] = v;
  if (s.lam32) {
    s.lam32[(long)i * s.Lp + j] = (float)v;
    s.lamT32[(long)j * s.Lp + i] = (float)v;
  }
  if (s.lamB) {   // hi / lo BF16 pair of v at (j, i) of Lambda^T's copy and (i, j) of Lambda's
    const long pl = (long)s.Lp * s.Lp;
    const bf16s hi(v);
    const bf16s lo(v - (double)hi);
    s.lamB[(long)j * s.Lp + i] = hi.x;
    s.lamB[pl + (long)j * s.Lp + i] = lo.x;
    s.lamB[2 * pl + (long)i * s.Lp + j] = hi.x;
    s.lamB[3 * pl + (long)i * s.Lp + j] = lo.x;
  }
}

// bfn[mu] = (centre of mu, zeta_mu) over the basis functions (the primitives
// of a contracted basis), and the Jastrow basis's centres (its exponents stay);
// rebuilt whenever R or zeta change.
__global__ void pack_basis_kernel(SysDev s) {
  const int mu = blockIdx.x * blockDim.x + threadIdx.x;
  if (mu < s.nprim()) {
    const int c = s.center[mu];
    s.bfn[mu] = make_double4(s.R[3 * c], s.R[3 * c + 1], s.R[3 * c + 2], s.zeta[mu]);
  }
  if (mu < s.LJ) {
    const int c = s.jcenter[mu];
    s.jbfn[mu] = make_double4(s.R[3 * c], s.R[3 * c + 1], s.R[3 * c + 2], s.jbfn[mu].w);
  }
}

hipError_t launch_pack_basis(const SysDev& s, hipStream_t st) {
  const int n = s.nprim() > s.LJ ? s.nprim() : s.LJ;
  hipLaunchKernelGGL(pack_basis_kernel, dim3((n + 255) / 256), dim3(256), 0, st, s);
  return hipGetLastError();
}

// New Jastrow-basis coefficients / exponents from device arrays (any may be null):
// jm <- j1_inh, M3 <- [[Muu, Mud], [Mud^T, Mdd]], jbfn[k].w <- jb_zeta[k].
__global__ void set_jastrow_basis_kernel(SysDev s, const double* __restrict__ j1_inh, const double* __restrict__ j3,
                                         const double* __restrict__ jz) {
  const int LJ = s.LJ;
  const long LL = (long)LJ * LJ;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j3 && idx < LL) {
    const int a = (int)(idx / LJ), b = (int)(idx % LJ);
    const long n2 = 2L * LJ;
    s.M3[a * n2 + b] = j3[idx];
    s.M3[(LJ + a) * n2 + LJ + b] = j3[LL + idx];
    s.M3[a * n2 + LJ + b] = j3[2 * LL + idx];
    s.M3[(LJ + b) * n2 + a] = j3[2 * LL + idx];
  }
  if (j1_inh && idx < 2L * LJ) s.jm[idx] = j1_inh[idx];
  if (jz && idx < LJ) {
    const double4 f = s.jbfn[idx];
    s.jbfn[idx] = make_double4(f.x, f.y, f.z, jz[idx]);
  }
}

hipError_t launch_set_jastrow_basis(const SysDev& s, const double* j1_inh, const double* j3, const double* jz,
                                    hipStream_t st) {
  const long n = (long)s.LJ * s.LJ > 2L * s.LJ ? (long)s.LJ * s.LJ : 2L * s.LJ;
  hipLaunchKernelGGL(set_jastrow_basis_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, j1_inh, j3,
                     jz);
  return hipGetLastError();
}

// Nonzero flags of the [kLamTileK x kLamTileN] tiles of Lambda and Lambda^T
// (one block per tile pair); a banded Lambda lets the P products skip most tiles.
__global__ void __launch_bounds__(256) lam_mask_kernel(SysDev s) {
  const int nt = blockIdx.x, kt = blockIdx.y;
  const int mask_ld = gridDim.x;
  int nz = 0, nzT = 0;
  for (int idx = threadIdx.x; idx < kLamTileK * kLamTileN; idx += blockDim.x) {
    const int r = kt * kLamTileK + idx / kLamTileN, c = nt * kLamTileN + idx % kLamTileN;
    if (r < s.Lp && c < s.Lp) {
      nz |= s.lam[(long)r * s.Lp + c] != 0.0;
      nzT |= s.lamT[(long)r * s.Lp + c] != 0.0;
    }
  }
  nz = __syncthreads_or(nz);
  nzT = __syncthreads_or(nzT);
  if (threadIdx.x == 0) {
    s.lam_mask[(long)kt * mask_ld + nt] = nz ? 1 : 0;
    s.lamT_mask[(long)kt * mask_ld + nt] = nzT ? 1 : 0;
  }
}

hipError_t launch_lam_mask(const SysDev& s, hipStream_t st) {
  const dim3 grid((s.Lp + kLamTileN - 1) / kLamTileN, (s.Lp + kLamTileK - 1) / kLamTileK);
  hipLaunchKernelGGL(lam_mask_kernel, grid, dim3(256), 0, st, s);
  return hipGetLastError();
}

hipError_t launch_set_lambda(const SysDev& s, const double* lam, hipStream_t st) {
  const long tot = (long)s.L * s.L;
  hipLaunchKernelGGL(set_lambda_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, s, lam);
  return hipGetLastError();
}

}  // namespace qmc
