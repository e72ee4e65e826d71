// Hand-written reverse pass (adjoint) of the whole evaluation: gradients of
//   F_w = a_w log|Psi_w| + b_w e_L,w
// with respect to nuclear positions R, basis exponents zeta, the pairing
// matrix Lambda (all L^2 entries, unconstrained), the Jastrow parameters and
// the electron positions r.  (Derivatives of energy section: O_k = d ln Psi /
// d alpha_k and the local-energy derivatives needed for forces; the adjoint
// gives all of them at a small multiple of the cost of one evaluation.)
//
// Forward quantities per walker (FP64): Phi, W = Phi_U Lambda Phi_D^T,
// A = W^{-1}, P = [Phi_U Lambda ; Phi_D Lambda^T], Yt = [A^T P_D ; A P_U],
// Jastrow gradient g_i and Laplacian h_i, drift.  With
//   Q = lap Phi + 2 grad Phi . g          (per electron row)
//   V = Q_U Lambda Phi_D^T + Phi_U Lambda Q_D^T,
// the determinant part of the kinetic sum is tr(A V) and
//   e_kin = -1/2 [ tr(A V) + sum_i (h_i + |g_i|^2) ].
// Reverse pass:
//   G_W = a A^T + b/2 (A V A)^T       (d F / d W)
//   G_V = -b/2 A^T                      (d F / d V)
//   X_U = G_W Phi_D + G_V Q_D,  X_D = G_W^T Phi_U + G_V^T Q_U,  Z_U = G_V Phi_D
//   dF/dPhi_U = X_U Lambda^T,  dF/dPhi_D = X_D Lambda
//   dF/dLambda = Phi_U^T X_U + Q_U^T Z_U
//   dF/dQ = -b/2 Yt,  so dF/dlap Phi = -b/2 Yt and dF/dgrad Phi = -b Yt g
//   dF/dg_i = -b drift_i,  dF/dh_i = -b/2,  dF/dJ = a,  dF/dV_coulomb = b
// then through the basis functions (values, gradients, Hessians, gradient of
// the Laplacian, exponent derivatives) and the radial Jastrow terms.
#include <vector>

#include "internal.h"

namespace qmc {

// ---------------------------------------------------------------------------
// forward-mode dual numbers for the radial Jastrow functions
// ---------------------------------------------------------------------------
struct Dl {
  double v, d;
};
__device__ __forceinline__ Dl operator+(Dl a, Dl b) { return {a.v + b.v, a.d + b.d}; }
__device__ __forceinline__ Dl operator-(Dl a, Dl b) { return {a.v - b.v, a.d - b.d}; }
__device__ __forceinline__ Dl operator-(Dl a) { return {-a.v, -a.d}; }
__device__ __forceinline__ Dl operator*(Dl a, Dl b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__device__ __forceinline__ Dl operator/(Dl a, Dl b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
__device__ __forceinline__ Dl operator+(double a, Dl b) { return {a + b.v, b.d}; }
__device__ __forceinline__ Dl operator*(double a, Dl b) { return {a * b.v, a * b.d}; }
__device__ __forceinline__ Dl operator*(Dl a, double b) { return {a.v * b, a.d * b}; }
__device__ __forceinline__ Dl operator/(double a, Dl b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }
__device__ __forceinline__ Dl dexp(Dl a) { const double e = exp(a.v); return {e, e * a.d}; }
__device__ __forceinline__ Dl dexpm1(Dl a) { return {expm1(a.v), exp(a.v) * a.d}; }
__device__ __forceinline__ double dexp(double a) { return exp(a); }
__device__ __forceinline__ double dexpm1(double a) { return expm1(a); }

template <class S>
__device__ void j1_radial_t(int form, double Z, S b, S r, S& f, S& f1, S& f2) {
  const double q = sqrt(sqrt(2.0 * Z));
  const S s = q * r;
  S u, u1, u2;
  if (form == 1) {
    const S e = dexp(-(b * s));
    u = -dexpm1(-(b * s)) / (2.0 * b);
    u1 = 0.5 * e;
    u2 = -0.5 * (b * e);
  } else {
    const S den = 1.0 / (1.0 + b * s);
    u = 0.5 * (s * den);
    u1 = 0.5 * (den * den);
    u2 = -(b * den * den * den);
  }
  const double q3 = q * q * q;
  f = -q3 * u;
  f1 = -(q3 * q) * u1;
  f2 = -(q3 * q * q) * u2;
}

// two-body: c t + a1 t^2 + a2 t^3 + a3 t^4 with t = r/(1+b r); c = 1/4 or 1/2
template <class S>
__device__ void j2_radial_t(double c, S b, S a1, S a2, S a3, S r, S& v, S& v1, S& v2) {
  const S den = 1.0 / (1.0 + b * r);
  const S t = r * den;
  const S dt = den * den;
  const S d2t = -2.0 * (b * den * den * den);
  const S g = t * (c + t * (a1 + t * (a2 + t * a3)));
  const S g1 = c + t * (2.0 * a1 + t * (3.0 * a2 + t * (4.0 * a3)));
  const S g2 = 2.0 * a1 + t * (6.0 * a2 + t * (12.0 * a3));
  v = g;
  v1 = g1 * dt;
  v2 = g2 * dt * dt + g1 * d2t;
}

__device__ __forceinline__ Dl cst(double x) { return {x, 0.0}; }
__device__ __forceinline__ Dl var(double x) { return {x, 1.0}; }

// Parameters (b, a1, a2, a3) of the two-body channel of a pair.
__device__ __forceinline__ void j2_params(const SysDev& s, bool same, double p[4]) {
  if (s.j2_form == 1) {
    p[0] = same ? s.j2d[0] : s.j2d[1]; p[1] = p[2] = p[3] = 0.0;
  } else {
    const int o = same ? 0 : 4;
    p[0] = s.j2d[o]; p[1] = s.j2d[o + 1]; p[2] = s.j2d[o + 2]; p[3] = s.j2d[o + 3];
  }
}

// Gradient, w.r.t. the displacement d (|d| = r), of the pair term
//   T = cv f(r) + gb . d f'(r)/r + ch (f''(r) + 2 f'(r)/r)
// given f', f'', f''' at r.
__device__ __forceinline__ void pair_term_grad(double cv, double ch, const double gb[3], const double d[3],
                                               double r, double f1, double f2, double f3, double out[3]) {
  const double ir = 1.0 / r;
  const double gd = gb[0] * d[0] + gb[1] * d[1] + gb[2] * d[2];
  const double radial = cv * f1 + ch * (f3 + 2.0 * f2 * ir - 2.0 * f1 * ir * ir);
  const double k = (f2 * ir - f1 * ir * ir) * ir * gd;
  for (int c = 0; c < 3; ++c) out[c] = radial * d[c] * ir + gb[c] * f1 * ir + k * d[c];
}

// ---------------------------------------------------------------------------
// 1. stacked basis rows: SU = [Phi_U ; Q_U], SD = [Phi_D ; Q_D] per walker,
//    Q = lap Phi + 2 grad Phi . g_i  (one workgroup per electron row)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) stack_basis_kernel(SysDev s, WalkDev w, double* __restrict__ SU,
                                                          double* __restrict__ SD) {
  const long row = blockIdx.x;           // wk * N + i
  const int wk = (int)(row / s.N), i = (int)(row % s.N);
  const double px = w.r[3 * row], py = w.r[3 * row + 1], pz = w.r[3 * row + 2];
  const double* g = w.gJ + 4 * row;
  const double gx = g[0], gy = g[1], gz = g[2];
  const int n = s.nu;
  double *dphi, *dq;
  if (i < s.nu) {
    dphi = SU + ((long)wk * 2 * n + i) * s.Lp;
    dq = SU + ((long)wk * 2 * n + n + i) * s.Lp;
  } else {
    dphi = SD + ((long)wk * 2 * n + (i - s.nu)) * s.Lp;
    dq = SD + ((long)wk * 2 * n + n + (i - s.nu)) * s.Lp;
  }
  for (int mu = threadIdx.x; mu < s.Lp; mu += blockDim.x) {
    double v = 0.0, q = 0.0;
    if (mu < s.L) {
      double bx = 0.0, by = 0.0, bz = 0.0, lp = 0.0;
      if (s.Lq) {   // contracted orbital: the same combination of the primitives' values and derivatives
        for (int k = s.con_ptr[mu]; k < s.con_ptr[mu + 1]; ++k) {
          double pv, px_, py_, pz_, pl;
          basis_vgl(s, s.con_idx[k], px, py, pz, pv, px_, py_, pz_, pl);
          const double cf = s.con_coef[k];
          v += cf * pv; bx += cf * px_; by += cf * py_; bz += cf * pz_; lp += cf * pl;
        }
      } else {
        basis_vgl(s, mu, px, py, pz, v, bx, by, bz, lp);
      }
      q = lp + 2.0 * (bx * gx + by * gy + bz * gz);
    }
    dphi[mu] = v;
    dq[mu] = q;
  }
}

// Contracted orbitals: rows over the orbitals (dF/dPhi, Yt) as rows over the
// primitives, out[mu] = sum_c C[mu][c] in[c] (zero past Lq), so that the basis
// backward runs over the primitives.
__global__ void __launch_bounds__(256) prim_rows_kernel(SysDev s, const double* __restrict__ in, int lq_pad,
                                                        double* __restrict__ out) {
  const long row = blockIdx.x;
  const double* y = in + row * s.Lp;
  double* o = out + row * lq_pad;
  for (int mu = threadIdx.x; mu < lq_pad; mu += blockDim.x) o[mu] = mu < s.Lq ? prim_weight(s, mu, y) : 0.0;
}

// ---------------------------------------------------------------------------
// 2. G_W = a A^T + b/2 M^T (M = A V A), G_V = -b/2 A^T, stored as
//    GG  = [G_W | G_V]  (n x 2n)  and  GGt = [G_W ; G_V]  (2n x n)
// ---------------------------------------------------------------------------
__global__ void gw_kernel(int n, int Wk, const double* __restrict__ A, const double* __restrict__ M,
                          const double* __restrict__ ga, const double* __restrict__ gb,
                          double* __restrict__ GG, double* __restrict__ GGt) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Wk * n * n) return;
  const int wk = (int)(idx / ((long)n * n));
  const int rem = (int)(idx % ((long)n * n));
  const int i = rem / n, j = rem % n;       // G[i][j], i up, j down
  const double a = ga ? ga[wk] : 0.0, b = gb ? gb[wk] : 0.0;
  const double Aji = A[(long)wk * n * n + (long)j * n + i];
  const double Mji = M[(long)wk * n * n + (long)j * n + i];
  const double gw = a * Aji + 0.5 * b * Mji;
  const double gv = -0.5 * b * Aji;
  double* gg = GG + (long)wk * 2 * n * n;
  gg[(long)i * 2 * n + j] = gw;
  gg[(long)i * 2 * n + n + j] = gv;
  double* gt = GGt + (long)wk * 2 * n * n;
  gt[(long)i * n + j] = gw;
  gt[(long)(n + i) * n + j] = gv;
}

// ---------------------------------------------------------------------------
// 3. basis backward, one workgroup per walker; threads own basis functions mu
//    and loop over electrons.  For each (i, mu):
//      pb = dF/dPhi, qb = dF/dQ = -b/2 Yt, gbar = 2 qb g_i, hbar = qb
//      t  = pb grad psi + Hess psi . gbar + hbar grad(lap psi)      (= dF/dr_i)
//      zeta_bar_mu += pb d_zeta psi + gbar . d_zeta grad psi + hbar d_zeta lap psi
//    dF/dR_center(mu) -= t.  Per-electron sums of t reduce per wave (fixed order).
// ---------------------------------------------------------------------------
__device__ __forceinline__ void hess_P(int kind, double H[6]) {   // xx yy zz xy yz zx
  for (int k = 0; k < 6; ++k) H[k] = 0.0;
  switch (kind) {
    case 4: H[3] = 1.0; break;
    case 5: H[4] = 1.0; break;
    case 6: H[5] = 1.0; break;
    case 7: H[0] = 2.0; H[1] = -2.0; break;
    case 8: H[0] = -2.0; H[1] = -2.0; H[2] = 4.0; break;
    default: break;
  }
}

// Launched with kBackThreads threads (five waves: 300 functions in one pass at
// L = 300, 600 in two).
constexpr int kBackThreads = 320;
__global__ void __launch_bounds__(kBackThreads)
basis_backward_kernel(SysDev s, WalkDev w, const double* __restrict__ phibar, const double* __restrict__ gb,
                      double* __restrict__ dr, double* __restrict__ Rbar_w, double* __restrict__ zbar_w,
                      double* __restrict__ tmu, int acc) {
  constexpr int NC = kLuMaxN * 2;   // electrons per chunk (rows of rpart)
  __shared__ double rpart[kBackThreads / 64][NC][3];
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double b = gb ? gb[wk] : 0.0;
  const double* r = w.r + (long)wk * s.N * 3;
  const double* Yt = w.Yt + (long)wk * s.N * s.Lp;
  const double* PB = phibar + (long)wk * s.N * s.Lp;
  const double* gJ = w.gJ + (long)wk * s.N * 4;
  double* tm = tmu + (long)wk * s.L * 3;
  double* zw = zbar_w + (long)wk * s.L;
  const int nmu = (s.L + blockDim.x - 1) / blockDim.x;
  // electrons in chunks of NC: a function's sums over the electrons continue
  // from the previous chunk's (its own thread stored them), so every sum runs
  // over i in increasing order whatever the chunking
  for (int c0 = 0; c0 < s.N; c0 += NC) {
    const int c1 = min(s.N, c0 + NC);
    for (int k = 0; k < nmu; ++k) {
      const int mu = tid + k * blockDim.x;
      const bool act = mu < s.L;
      int kind = 0;
      double zt = 0.0, Rx = 0.0, Ry = 0.0, Rz = 0.0, HP[6];
      if (act) {
        const double4 f = s.bfn[mu];
        kind = s.kind[mu]; zt = f.w;
        Rx = f.x; Ry = f.y; Rz = f.z;
      }
      hess_P(kind_ang(kind), HP);
      double zacc = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
      if (c0 > 0 && act) { zacc = zw[mu]; tx = tm[3 * mu]; ty = tm[3 * mu + 1]; tz = tm[3 * mu + 2]; }
      for (int i = c0; i < c1; ++i) {
        double t0 = 0.0, t1 = 0.0, t2 = 0.0;
        if (act) {
          const double pb = PB[(long)i * s.Lp + mu];
          const double qb = -0.5 * b * Yt[(long)i * s.Lp + mu];
          const double gbx = 2.0 * qb * gJ[4 * i], gby = 2.0 * qb * gJ[4 * i + 1], gbz = 2.0 * qb * gJ[4 * i + 2];
          const double hb = qb;
          const double d[3] = {r[3 * i] - Rx, r[3 * i + 1] - Ry, r[3 * i + 2] - Rz};
          const double sq = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          double P, Pg[3];
          angular(kind_ang(kind), d[0], d[1], d[2], P, Pg[0], Pg[1], Pg[2]);
          const Radial rd = radial_all(kind, zt, sq);
          const double e = rd.e;
          const double psi = P * e;
          double gpsi[3];
          for (int a = 0; a < 3; ++a) gpsi[a] = (Pg[a] + rd.h1 * d[a] * P) * e;
          // Hessian of psi
          const int ia[6] = {0, 1, 2, 0, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 0};
          double Hs[3][3];
          for (int q = 0; q < 6; ++q) {
            const int a = ia[q], bb = ib[q];
            const double v = (HP[q] + rd.h1 * (d[a] * Pg[bb] + d[bb] * Pg[a]) +
                              (a == bb ? rd.h1 * P : 0.0) + rd.h2 * d[a] * d[bb] * P) * e;
            Hs[a][bb] = v; Hs[bb][a] = v;
          }
          const double cl = rd.cl;   // lap psi = cl psi
          double glap[3];
          for (int a = 0; a < 3; ++a) glap[a] = rd.gl * d[a] * psi + cl * gpsi[a];
          const double gbv[3] = {gbx, gby, gbz};
          t0 = pb * gpsi[0] + Hs[0][0] * gbv[0] + Hs[0][1] * gbv[1] + Hs[0][2] * gbv[2] + hb * glap[0];
          t1 = pb * gpsi[1] + Hs[1][0] * gbv[0] + Hs[1][1] * gbv[1] + Hs[1][2] * gbv[2] + hb * glap[1];
          t2 = pb * gpsi[2] + Hs[2][0] * gbv[0] + Hs[2][1] * gbv[1] + Hs[2][2] * gbv[2] + hb * glap[2];
          // exponent derivatives
          const double zpsi = -rd.zp * psi;
          double zg = 0.0;
          for (int a = 0; a < 3; ++a) zg += gbv[a] * (-rd.zq * d[a] * psi - rd.zp * gpsi[a]);
          const double zlap = rd.dcl * psi - rd.zp * cl * psi;
          zacc += pb * zpsi + zg + hb * zlap;
          tx += t0; ty += t1; tz += t2;
        }
        const double s0 = wave_sum(t0), s1 = wave_sum(t1), s2 = wave_sum(t2);
        if (lane == 0) {
          double* rp = rpart[wave][i - c0];
          if (k == 0) { rp[0] = s0; rp[1] = s1; rp[2] = s2; }
          else { rp[0] += s0; rp[1] += s1; rp[2] += s2; }
        }
      }
      if (act) {
        zw[mu] = zacc;
        tm[3 * mu] = tx; tm[3 * mu + 1] = ty; tm[3 * mu + 2] = tz;
      }
    }
    __syncthreads();
    for (int i = c0 + tid; i < c1; i += blockDim.x) {
      for (int c = 0; c < 3; ++c) {
        double t = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) t += rpart[q][i - c0][c];
        if (acc) dr[((long)wk * s.N + i) * 3 + c] += t;
        else dr[((long)wk * s.N + i) * 3 + c] = t;
      }
    }
    __syncthreads();   // rpart is refilled by the next chunk; tm complete for the nuclei below
  }
  // nuclear positions: dF/dR_a = - sum over the functions centred on a (CSR order)
  for (int a = tid; a < s.n_nuc; a += blockDim.x) {
    double t[3] = {0.0, 0.0, 0.0};
    for (int k = s.cptr[a]; k < s.cptr[a + 1]; ++k) {
      const int mu = s.cmu[k];
      for (int c = 0; c < 3; ++c) t[c] += tm[3 * mu + c];
    }
    for (int c = 0; c < 3; ++c) {
      if (acc) Rbar_w[((long)wk * s.n_nuc + a) * 3 + c] -= t[c];
      else Rbar_w[((long)wk * s.n_nuc + a) * 3 + c] = -t[c];
    }
  }
}

// ---------------------------------------------------------------------------
// 4. Jastrow and Coulomb backward, one workgroup per walker, thread = electron
//    (in chunks of the block size).
//    Pair terms of F: a_w J + sum_i gbar_i . grad_i J - b_w/2 sum_i lap_i J + b_w V,
//    gbar_i = -b_w drift_i.  Accumulates into dr, Rbar_w and writes jbar_w.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
jastrow_backward_kernel(SysDev s, WalkDev w, const double* __restrict__ ga, const double* __restrict__ gbw,
                        double* __restrict__ dr, double* __restrict__ Rbar_w, double* __restrict__ jbar_w) {
  __shared__ double rbin[4][kMaxNucBack][4];   // per wave: dR (3) and d b_a
  __shared__ double red[4][8];
  __shared__ double rpair[256][3];              // per thread: its partners' share of dF/dr_i
  const int wk = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double av = ga ? ga[wk] : 0.0, bv = gbw ? gbw[wk] : 0.0;
  const double* r = w.r + (long)wk * s.N * 3;
  const double* drift = w.drift + (long)wk * s.N * 3;
  double th[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // jas slots after the one-body b's
  // electrons in chunks of the block size (thread = electron c0 + tid); the
  // per-nucleus sums continue over the chunks in order
  for (int c0 = 0; c0 < s.N; c0 += blockDim.x) {
    const int i = c0 + tid;
    const bool act = i < s.N;
    double xi[3] = {0.0, 0.0, 0.0}, gi[3] = {0.0, 0.0, 0.0};
    if (act) {
      for (int c = 0; c < 3; ++c) { xi[c] = r[3 * i + c]; gi[c] = -bv * drift[3 * i + c]; }
    }
    double rb[3] = {0.0, 0.0, 0.0};
    // one-body terms and electron-nucleus attraction, nucleus by nucleus
    for (int a = 0; a < s.n_nuc; ++a) {
      double cR[3] = {0.0, 0.0, 0.0}, cb = 0.0;
      if (act) {
        const double d[3] = {xi[0] - s.R[3 * a], xi[1] - s.R[3 * a + 1], xi[2] - s.R[3 * a + 2]};
        const double ria = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double Z = s.Z[a];
        double t[3] = {0.0, 0.0, 0.0};
        if (s.j1_form) {
          Dl f, f1, f2;
          j1_radial_t<Dl>(s.j1_form, Z, cst(s.j1_b[a]), var(ria), f, f1, f2);
          pair_term_grad(av, -0.5 * bv, gi, d, ria, f1.v, f2.v, f2.d, t);
          Dl pf, pf1, pf2;
          j1_radial_t<Dl>(s.j1_form, Z, var(s.j1_b[a]), cst(ria), pf, pf1, pf2);
          const double gd = (gi[0] * d[0] + gi[1] * d[1] + gi[2] * d[2]) / ria;
          cb = av * pf.d + gd * pf1.d - 0.5 * bv * (pf2.d + 2.0 * pf1.d / ria);
        }
        // b_w * (-Z / r_ia): d/dr_i = b Z d / r^3
        const double ir3 = 1.0 / (ria * ria * ria);
        for (int c = 0; c < 3; ++c) t[c] += bv * Z * d[c] * ir3;
        for (int c = 0; c < 3; ++c) { rb[c] += t[c]; cR[c] = -t[c]; }
      }
      const double s0 = wave_sum(cR[0]), s1 = wave_sum(cR[1]), s2 = wave_sum(cR[2]), s3 = wave_sum(cb);
      if (lane == 0 && a < kMaxNucBack) {
        double* rbw = rbin[wave][a];
        if (c0 == 0) { rbw[0] = s0; rbw[1] = s1; rbw[2] = s2; rbw[3] = s3; }
        else { rbw[0] += s0; rbw[1] += s1; rbw[2] += s2; rbw[3] += s3; }
      }
    }
    // two-body terms and electron-electron repulsion: the chunk's nc electrons
    // times G groups of partners (thread = electron c0 + tid % nc, partners
    // j = g, g + G, ... for g = tid / nc), so that short chunks keep most
    // threads busy; the groups' sums for an electron meet in LDS in order of g
    const int nc = min(s.N - c0, (int)blockDim.x);
    const int G = max(1, (int)blockDim.x / nc);
    const int ip = c0 + tid % nc, gp = tid / nc;
    double rp[3] = {0.0, 0.0, 0.0};
    if (gp < G) {
      double xp[3], gq[3];
      for (int c = 0; c < 3; ++c) { xp[c] = r[3 * ip + c]; gq[c] = -bv * drift[3 * ip + c]; }
      for (int j = gp; j < s.N; j += G) {
        if (j == ip) continue;
        const double d[3] = {xp[0] - r[3 * j], xp[1] - r[3 * j + 1], xp[2] - r[3 * j + 2]};
        const double rij = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        const double ir3 = 1.0 / (rij * rij * rij);
        for (int c = 0; c < 3; ++c) rp[c] += -bv * d[c] * ir3;    // b_w * 1/r_ij
        if (!s.j2_form) continue;
        const bool same = (ip < s.nu) == (j < s.nu);
        double p[4];
        j2_params(s, same, p);
        const double cc = same ? 0.25 : 0.5;
        double dg[3];
        for (int c = 0; c < 3; ++c) dg[c] = gq[c] + bv * drift[3 * j + c];    // gbar_i - gbar_j
        Dl v, v1, v2;
        j2_radial_t<Dl>(cc, cst(p[0]), cst(p[1]), cst(p[2]), cst(p[3]), var(rij), v, v1, v2);
        double t[3];
        pair_term_grad(av, -bv, dg, d, rij, v1.v, v2.v, v2.d, t);
        for (int c = 0; c < 3; ++c) rp[c] += t[c];
        const double gd = (dg[0] * d[0] + dg[1] * d[1] + dg[2] * d[2]) / rij;
        const int np = s.j2_form == 1 ? 1 : 4;
        const int slot0 = s.j2_form == 1 ? (same ? 0 : 1) : (same ? 0 : 4);
        for (int k = 0; k < np; ++k) {
          Dl q[4] = {cst(p[0]), cst(p[1]), cst(p[2]), cst(p[3])};
          q[k].d = 1.0;
          Dl pv, pv1, pv2;
          j2_radial_t<Dl>(cc, q[0], q[1], q[2], q[3], cst(rij), pv, pv1, pv2);
          // each pair is visited from both electrons: half weight
          th[slot0 + k] += 0.5 * (av * pv.d + gd * pv1.d - bv * (pv2.d + 2.0 * pv1.d / rij));
        }
      }
    }
    __syncthreads();   // the previous chunk's partner sums are read
    if (gp < G)
      for (int c = 0; c < 3; ++c) rpair[tid][c] = rp[c];
    __syncthreads();
    if (act) {
      for (int g = 0; g < G; ++g)
        for (int c = 0; c < 3; ++c) rb[c] += rpair[g * nc + tid][c];
      for (int c = 0; c < 3; ++c) dr[((long)wk * s.N + i) * 3 + c] += rb[c];
    }
  }
  for (int k = 0; k < 8; ++k) {
    const double t = wave_sum(th[k]);
    if (lane == 0) red[wave][k] = t;
  }
  __syncthreads();
  const int n2 = s.j2_form == 1 ? 2 : (s.j2_form == 2 ? 8 : 0);
  const int nj = s.n_nuc + n2;
  double* jb = jbar_w + (long)wk * nj;
  for (int a = tid; a < s.n_nuc; a += blockDim.x) {
    double t[4] = {0.0, 0.0, 0.0, 0.0};
    for (int q = 0; q < 4; ++q)
      for (int c = 0; c < 4; ++c) t[c] += rbin[q][a][c];
    // nucleus-nucleus repulsion b_w Z_a Z_b / R_ab
    for (int bb = 0; bb < s.n_nuc; ++bb) {
      if (bb == a) continue;
      const double d[3] = {s.R[3 * a] - s.R[3 * bb], s.R[3 * a + 1] - s.R[3 * bb + 1],
                           s.R[3 * a + 2] - s.R[3 * bb + 2]};
      const double R2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      const double k3 = -bv * s.Z[a] * s.Z[bb] / (R2 * sqrt(R2));
      for (int c = 0; c < 3; ++c) t[c] += k3 * d[c];
    }
    for (int c = 0; c < 3; ++c) Rbar_w[((long)wk * s.n_nuc + a) * 3 + c] += t[c];
    jb[a] = s.j1_form ? t[3] : 0.0;
  }
  if (tid < n2) {
    double t = 0.0;
    for (int q = 0; q < 4; ++q) t += red[q][tid];
    jb[s.n_nuc + tid] = t;
  }
}

// Sum per-walker (or per-chunk) rows: out[k] = sum_w in[w][k], fixed order.
// The rows are added in order; their values are loaded sixteen at a time (a
// short output, such as dF/dR over 512 walkers, is otherwise one dependent
// load per row).
__global__ void sum_rows_kernel(const double* __restrict__ in, long n_rows, long len, double* __restrict__ out) {
  const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  constexpr int U = 16;
  double t = 0.0;
  long w = 0;
  for (; w + U <= n_rows; w += U) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = in[(w + u) * len + k];
#pragma unroll
    for (int u = 0; u < U; ++u) t += v[u];
  }
  for (; w < n_rows; ++w) t += in[w * len + k];
  out[k] = t;
}

static hipError_t sum_rows(const double* in, long n_rows, long len, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_rows_kernel, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, in, n_rows, len, out);
  return hipGetLastError();
}

#define HT(x)                              \
  do {                                     \
    hipError_t _e = (x);                   \
    if (_e != hipSuccess) return _e;       \
  } while (0)

// The reverse pass.  The forward state (Phi rows are recomputed here; P, A,
// Yt, gJ, drift come from the evaluation that the caller ran just before).
// ---------------------------------------------------------------------------
// Jastrow-basis terms (onebody_J_inh, threebody_jastrow).  With
// gvec_i = G_{s_i} - h_i + m_{s_i}, the terms' share of F is
//   F_3 = sum_i sum_{j != i} u_i^T M^{s_i s_j} chi_j + sum_i (a chi_i + c_i) . m_{s_i},
//   c_i = gbar_i . grad chi(r_i) + hbar lap chi(r_i),  u_i = a/2 chi_i + c_i,
// gbar_i = -b drift_i, hbar = -b/2 (dF/dgrad_i J, dF/dlap_i J).  Hence
//   dF/dchi_j      = [M3 U]_{s_j} - M^{s_j s_j} u_j + a/2 (G_{s_j} - h_j) + a m_{s_j},
//                    U = [sum_{i up} u_i ; sum_{i down} u_i]
//   dF/dgrad chi_j = gbar_j gvec_j,  dF/dlap chi_j = hbar gvec_j
//   dF/dm_s        = sum_{i of s} (a chi_i + c_i)
//   dF/dM^{ss}     = sym(U_s X_s^T - sum_{i of s} u_i chi_i^T)   (gradient w.r.t. a symmetric matrix)
//   dF/dM^{ud}     = U_u X_d^T + X_u U_d^T,   X_s = sum_{i of s} chi_i,
// and the basis backward over chi (with "Yt" = gvec and "g" = drift, so that
// its gbar = 2 (-b/2 gvec) drift and hbar = -b/2 gvec) gives dF/dr, dF/dR and
// the exponents' gradients.
// ---------------------------------------------------------------------------
// Per (walker, electron), one wave: U rows, gvec rows, (a chi + c) rows, drift4.
__global__ void __launch_bounds__(256)
j3_adj_rows_kernel(SysDev s, WalkDev w, AdjWork aw, const double* __restrict__ ga, const double* __restrict__ gb,
                   int rows) {
  const int lane = threadIdx.x & 63;
  const long row = (long)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const int LJ = s.LJ, LJp = aw.LJp;
  const int wk = (int)(row / s.N), i = (int)(row % s.N);
  const int sp = i < s.nu ? 0 : 1;
  const double a = ga ? ga[wk] : 0.0, b = gb ? gb[wk] : 0.0;
  const double px = w.r[3 * row], py = w.r[3 * row + 1], pz = w.r[3 * row + 2];
  const double* dft = w.drift + row * 3;
  const double gbx = -b * dft[0], gby = -b * dft[1], gbz = -b * dft[2], hb = -0.5 * b;
  const double* G = w.G3 + ((long)wk * 2 + sp) * LJ;
  const double* h = w.hv + row * LJ;
  const double* m = s.jm + (long)sp * LJ;
  for (int k = lane; k < LJp; k += 64) {
    double u = 0.0, gv = 0.0, ac = 0.0;
    if (k < LJ) {
      double v, vx, vy, vz, vl;
      basis_vgl_tab(s.jbfn, s.jkind, k, px, py, pz, v, vx, vy, vz, vl);
      const double c = gbx * vx + gby * vy + gbz * vz + hb * vl;
      u = 0.5 * a * v + c;
      ac = a * v + c;
      gv = G[k] - h[k] + m[k];
    }
    aw.ju[row * LJp + k] = u;
    aw.jgv[row * LJp + k] = gv;
    aw.jac[row * LJp + k] = ac;
  }
  if (lane < 4) aw.drift4[row * 4 + lane] = lane < 3 ? dft[lane] : 0.0;
}

// Per walker: U_s, X_s, dF/dm_s and H = M3 U (LDS), then the dF/dchi rows.
__global__ void __launch_bounds__(256) j3_adj_sum_kernel(SysDev s, WalkDev w, AdjWork aw, const double* __restrict__ ga) {
  __shared__ double U[2 * kMaxLJ];
  const int wk = blockIdx.x, LJ = s.LJ, LJp = aw.LJp;
  const double a = ga ? ga[wk] : 0.0;
  const double* u = aw.ju + (long)wk * s.N * LJp;
  const double* ac = aw.jac + (long)wk * s.N * LJp;
  const double* chi = w.chi + (long)wk * s.N * LJ;
  double* X = aw.jX + (long)wk * 4 * LJ;   // X_u, X_d, U_u, U_d
  for (int k = threadIdx.x; k < LJ; k += blockDim.x) {
    double uu = 0.0, ud = 0.0, xu = 0.0, xd = 0.0, mu_ = 0.0, md = 0.0;
    for (int i = 0; i < s.nu; ++i) { uu += u[(long)i * LJp + k]; xu += chi[(long)i * LJ + k]; mu_ += ac[(long)i * LJp + k]; }
    for (int i = s.nu; i < s.N; ++i) { ud += u[(long)i * LJp + k]; xd += chi[(long)i * LJ + k]; md += ac[(long)i * LJp + k]; }
    U[k] = uu; U[LJ + k] = ud;
    X[k] = xu; X[LJ + k] = xd; X[2 * LJ + k] = uu; X[3 * LJ + k] = ud;
    aw.jdm[(long)wk * 2 * LJ + k] = mu_;
    aw.jdm[(long)wk * 2 * LJ + LJ + k] = md;
  }
  __syncthreads();
  double* Hs = aw.jH + (long)wk * 2 * LJ;
  for (int o = threadIdx.x; o < 2 * LJ; o += blockDim.x) {
    const double* row = s.M3 + (long)o * 2 * LJ;
    double g = 0.0;
    for (int c = 0; c < 2 * LJ; ++c) g += row[c] * U[c];
    Hs[o] = g;
  }
  (void)a;
}

// dF/dchi rows: [M3 U]_s - (M^{ss} u_j) + a/2 (G_s - h_j) + a m_s   (hu holds M^{ss} u_j)
__global__ void __launch_bounds__(256) j3_adj_chibar_kernel(SysDev s, WalkDev w, AdjWork aw,
                                                            const double* __restrict__ ga, long total) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int LJ = s.LJ, LJp = aw.LJp;
  const long row = idx / LJp;
  const int k = (int)(idx % LJp);
  if (k >= LJ) { aw.jpb[idx] = 0.0; return; }
  const int wk = (int)(row / s.N), i = (int)(row % s.N), sp = i < s.nu ? 0 : 1;
  const double a = ga ? ga[wk] : 0.0;
  const double H = aw.jH[((long)wk * 2 + sp) * LJ + k];
  const double G = w.G3[((long)wk * 2 + sp) * LJ + k];
  const double h = w.hv[row * LJ + k];
  aw.jpb[idx] = H - aw.jhu[idx] + 0.5 * a * (G - h) + a * s.jm[(long)sp * LJ + k];
}

// dF/dM: the slots hold sum_{i of s} u_i chi_i^T (same-spin) on entry
__global__ void __launch_bounds__(256) j3_adj_dM_kernel(SysDev s, AdjWork aw, int Wk) {
  const int LJ = s.LJ;
  const long LL = (long)LJ * LJ;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)Wk * LL) return;
  const int wk = (int)(idx / LL);
  const long e = idx % LL;
  const int k = (int)(e / LJ), l = (int)(e % LJ);
  const double* X = aw.jX + (long)wk * 4 * LJ;   // X_u, X_d, U_u, U_d
  const double* Xu = X, *Xd = X + LJ, *Uu = X + 2 * LJ, *Ud = X + 3 * LJ;
  double* D = aw.jdM + (long)wk * 3 * LL;
  const double* Cw = aw.jC + (long)wk * 2 * LL;   // sum u chi^T per spin
  // symmetric parts: 1/2 (raw_kl + raw_lk)
  D[e] = 0.5 * ((Uu[k] * Xu[l] - Cw[(long)k * LJ + l]) + (Uu[l] * Xu[k] - Cw[(long)l * LJ + k]));
  D[LL + e] = 0.5 * ((Ud[k] * Xd[l] - Cw[LL + (long)k * LJ + l]) + (Ud[l] * Xd[k] - Cw[LL + (long)l * LJ + k]));
  D[2 * LL + e] = Uu[k] * Xd[l] + Xu[k] * Ud[l];
}

static hipError_t launch_jastrow3_backward(const SysDev& s, const WalkDev& w, const AdjWork& aw, const double* ga,
                                           const double* gb, double* drw, hipStream_t st) {
  const int LJ = s.LJ, LJp = aw.LJp, Wk = w.Wk;
  const long rows = (long)Wk * s.N;
  hipLaunchKernelGGL(j3_adj_rows_kernel, dim3((unsigned)((rows + 3) / 4)), dim3(256), 0, st, s, w, aw, ga, gb,
                     (int)rows);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(j3_adj_sum_kernel, dim3(Wk), dim3(256), 0, st, s, w, aw, ga);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  for (int sp = 0; sp < 2; ++sp) {
    const int row0 = sp == 0 ? 0 : s.nu, nrow = sp == 0 ? s.nu : s.nd;
    if (nrow == 0) continue;
    // hu = u_j M^{ss} (M^{ss} symmetric) for the electrons of spin s
    GemmArgs g = gemm_args(nrow, LJ, LJ);
    g.A = aw.ju + (long)row0 * LJp; g.lda = LJp; g.a_bs = (long)s.N * LJp;
    g.B = s.M3 + (long)sp * LJ * 2 * LJ + (long)sp * LJ; g.ldb = 2 * LJ; g.b_bs = 0;
    g.C = aw.jhu + (long)row0 * LJp; g.ldc = LJp; g.c_bs = (long)s.N * LJp;
    g.batch = Wk;
    if ((e = gemm_f64(g, false, false, false, st)) != hipSuccess) return e;
    // C_s = sum_{i of s} u_i chi_i^T  ([LJ][LJ] per walker)
    GemmArgs c = gemm_args(LJ, LJ, nrow);
    c.A = aw.ju + (long)row0 * LJp; c.lda = LJp; c.a_bs = (long)s.N * LJp;   // op = A^T
    c.B = w.chi + (long)row0 * LJ; c.ldb = LJ; c.b_bs = (long)s.N * LJ;
    c.C = aw.jC + (long)sp * LJ * LJ; c.ldc = LJ; c.c_bs = 2L * LJ * LJ;
    c.batch = Wk;
    if ((e = gemm_f64(c, true, false, false, st)) != hipSuccess) return e;
  }
  const long tot = rows * LJp;
  hipLaunchKernelGGL(j3_adj_chibar_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, s, w, aw, ga, tot);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const long tm = (long)Wk * LJ * LJ;
  hipLaunchKernelGGL(j3_adj_dM_kernel, dim3((unsigned)((tm + 255) / 256)), dim3(256), 0, st, s, aw, Wk);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  // the chi basis backward: functions = the Jastrow basis, "Yt" = gvec, "g" = drift
  SysDev sj = s;
  sj.L = LJ; sj.Lp = LJp; sj.Lq = 0;
  sj.bfn = s.jbfn; sj.kind = s.jkind; sj.center = s.jcenter; sj.cptr = s.jcptr; sj.cmu = s.jcmu;
  WalkDev wj = w;
  wj.Yt = aw.jgv;
  wj.gJ = aw.drift4;
  hipLaunchKernelGGL(basis_backward_kernel, dim3(Wk), dim3(kBackThreads), 0, st, sj, wj, aw.jpb, gb, drw, aw.Rbar,
                     aw.jzbar, aw.jtmu, 1);
  return hipGetLastError();
}

// Zero fill (the down stacks' rows past n_dn when there are unpaired orbitals).
__global__ void __launch_bounds__(256) zero_fill_kernel(double* __restrict__ x, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// With k = n_up - n_dn unpaired orbitals W is n x n (n = n_up) with columns
// n_dn + l = Phi_U U_l and V's columns n_dn + l = Q_U U_l.  The down stacks hold
// n_dn real rows and zero rows after them, so every product over the down side
// sees only the paired columns; the unpaired columns add G_W[:, n_dn:] U to
// dF/dPhi_U, and their share of dF/dQ_U is already in Yt_U.
// dF/dPhi (aw.PB) and dF/dLambda of the geminal determinant, steps 1 to 7 of
// the backward pass.
static hipError_t geminal_backward(const SysDev& s, const WalkDev& w, const AdjWork& aw, const double* ga,
                                   const double* gb, int per_walker, double* dlambda, double* dunp,
                                   hipStream_t st) {
  const int n = s.nu, nd = s.nd, Wk = w.Wk, Lp = s.Lp, L = s.L, N = s.N;
  const long rowst = (long)N * Lp, stk = 2L * n * Lp;
  // 1. stacked rows [Phi_U; Q_U], [Phi_D; Q_D]
  if (s.nk > 0) {
    const long cnt = (long)Wk * stk;
    hipLaunchKernelGGL(zero_fill_kernel, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, st, aw.SD, cnt);
    HT(hipGetLastError());
  }
  hipLaunchKernelGGL(stack_basis_kernel, dim3((unsigned)((long)Wk * N)), dim3(256), 0, st, s, w, aw.SU, aw.SD);
  HT(hipGetLastError());
  // 2. V = Q_U P_D^T + P_U Q_D^T   (paired columns), V[:, n_dn + l] = Q_U U_l
  {
    GemmArgs g = gemm_args(n, nd, Lp);
    g.A = aw.SU + (long)n * Lp; g.lda = Lp; g.a_bs = stk;
    g.B = (const double*)w.P + (long)n * Lp; g.ldb = Lp; g.b_bs = rowst;
    g.C = aw.VQ; g.ldc = n; g.c_bs = (long)n * n; g.batch = Wk;
    HT(gemm_f64(g, false, true, false, st));
    g.A = w.P; g.a_bs = rowst;
    g.B = aw.SD + (long)n * Lp; g.b_bs = stk;
    g.accumulate = 1;
    HT(gemm_f64(g, false, true, false, st));
    if (s.nk > 0) {
      GemmArgs u = gemm_args(n, s.nk, Lp);
      u.A = aw.SU + (long)n * Lp; u.lda = Lp; u.a_bs = stk;
      u.B = s.Uph; u.ldb = Lp; u.b_bs = 0;
      u.C = aw.VQ + nd; u.ldc = n; u.c_bs = (long)n * n; u.batch = Wk;
      HT(gemm_f64(u, false, true, false, st));
    }
  }
  // 3. M = A V A
  {
    GemmArgs g = gemm_args(n, n, n);
    g.A = w.A; g.lda = n; g.a_bs = (long)n * n;
    g.B = aw.VQ; g.ldb = n; g.b_bs = (long)n * n;
    g.C = aw.T1; g.ldc = n; g.c_bs = (long)n * n; g.batch = Wk;
    HT(gemm_f64(g, false, false, false, st));
    g.A = aw.T1; g.B = w.A; g.C = aw.M;
    HT(gemm_f64(g, false, false, false, st));
  }
  // 4. G_W, G_V
  {
    const long tot = (long)Wk * n * n;
    hipLaunchKernelGGL(gw_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, n, Wk, w.A, aw.M, ga, gb,
                       aw.GG, aw.GGt);
    HT(hipGetLastError());
  }
  // 5. X_U = [G_W | G_V] [Phi_D; Q_D],  Z_U = G_V Phi_D,  X_D = [G_W; G_V]^T [Phi_U; Q_U]
  {
    GemmArgs g = gemm_args(n, Lp, 2 * n);
    g.A = aw.GG; g.lda = 2 * n; g.a_bs = 2L * n * n;
    g.B = aw.SD; g.ldb = Lp; g.b_bs = stk;
    g.C = aw.XZ; g.ldc = Lp; g.c_bs = stk; g.batch = Wk;
    HT(gemm_f64(g, false, false, false, st));
    GemmArgs z = gemm_args(n, Lp, n);
    z.A = aw.GG + n; z.lda = 2 * n; z.a_bs = 2L * n * n;
    z.B = aw.SD; z.ldb = Lp; z.b_bs = stk;
    z.C = aw.XZ + (long)n * Lp; z.ldc = Lp; z.c_bs = stk; z.batch = Wk;
    HT(gemm_f64(z, false, false, false, st));
    GemmArgs x = gemm_args(n, Lp, 2 * n);
    x.A = aw.GGt; x.lda = n; x.a_bs = 2L * n * n;
    x.B = aw.SU; x.ldb = Lp; x.b_bs = stk;
    x.C = aw.XD; x.ldc = Lp; x.c_bs = (long)n * Lp; x.batch = Wk;
    HT(gemm_f64(x, true, false, false, st));
  }
  // 6. dF/dPhi: rows of the up spin X_U Lambda^T, of the down spin X_D Lambda
  {
    GemmArgs g = gemm_args(Wk * n, Lp, Lp);
    g.A = aw.XZ; g.lda = Lp; g.a_grp = n; g.a_gs = stk;
    g.B = s.lamT; g.ldb = Lp;
    g.C = aw.PB; g.ldc = Lp; g.c_grp = n; g.c_gs = rowst;
    HT(gemm_f64(g, false, false, true, st));
    GemmArgs h = gemm_args(Wk * nd, Lp, Lp);
    h.A = aw.XD; h.lda = Lp; h.a_grp = nd; h.a_gs = (long)n * Lp;
    h.B = s.lam; h.ldb = Lp;
    h.C = aw.PB + (long)n * Lp; h.ldc = Lp; h.c_grp = nd; h.c_gs = rowst;
    HT(gemm_f64(h, false, false, true, st));
    if (s.nk > 0) {   // dF/dPhi_U += G_W[:, n_dn:] U
      GemmArgs u = gemm_args(n, Lp, s.nk);
      u.A = aw.GG + nd; u.lda = 2 * n; u.a_bs = 2L * n * n;
      u.B = s.Uph; u.ldb = Lp; u.b_bs = 0;
      u.C = aw.PB; u.ldc = Lp; u.c_bs = rowst; u.batch = Wk;
      u.accumulate = 1;
      HT(gemm_f64(u, false, false, false, st));
    }
  }
  // 7. dF/dLambda = [Phi_U; Q_U]^T [X_U; Z_U]
  if (dlambda) {
    if (per_walker) {
      GemmArgs g = gemm_args(L, L, 2 * n);
      g.A = aw.SU; g.lda = Lp; g.a_bs = stk;
      g.B = aw.XZ; g.ldb = Lp; g.b_bs = stk;
      g.C = dlambda; g.ldc = L; g.c_bs = (long)L * L; g.batch = Wk;
      HT(gemm_f64(g, true, false, true, st));
    } else {
      const int cw = aw.chunk_walkers, nfull = Wk / cw, rest = Wk % cw;
      GemmArgs g = gemm_args(L, L, 2 * n * cw);
      g.A = aw.SU; g.lda = Lp; g.a_bs = stk * cw;
      g.B = aw.XZ; g.ldb = Lp; g.b_bs = stk * cw;
      g.C = aw.lam_part; g.ldc = L; g.c_bs = (long)L * L; g.batch = nfull;
      if (nfull) HT(gemm_f64(g, true, false, true, st));
      if (rest) {
        GemmArgs h = g;
        h.K = 2 * n * rest;
        h.A = aw.SU + stk * cw * nfull; h.B = aw.XZ + stk * cw * nfull;
        h.C = aw.lam_part + (long)nfull * L * L; h.batch = 1;
        HT(gemm_f64(h, true, false, true, st));
      }
      HT(sum_rows(aw.lam_part, nfull + (rest ? 1 : 0), (long)L * L, dlambda, st));
    }
  }
  // 7b. unpaired orbitals: W[:, n_dn + l] = Phi_U U_l and V[:, n_dn + l] = Q_U U_l give
  //     dF/dU_l = [Phi_U; Q_U]^T [G_W; G_V][:, n_dn + l]
  if (dunp && s.nk > 0) {
    const int k = s.nk;
    if (per_walker) {
      GemmArgs g = gemm_args(L, k, 2 * n);
      g.A = aw.SU; g.lda = Lp; g.a_bs = stk;
      g.B = aw.GGt + nd; g.ldb = n; g.b_bs = 2L * n * n;
      g.C = dunp; g.ldc = k; g.c_bs = (long)L * k; g.batch = Wk;
      HT(gemm_f64(g, true, false, false, st));
    } else {
      const int cw = aw.chunk_walkers, nfull = Wk / cw, rest = Wk % cw;
      GemmArgs g = gemm_args(L, k, 2 * n * cw);
      g.A = aw.SU; g.lda = Lp; g.a_bs = stk * cw;
      g.B = aw.GGt + nd; g.ldb = n; g.b_bs = 2L * n * n * cw;
      g.C = aw.lam_part; g.ldc = k; g.c_bs = (long)L * k; g.batch = nfull;
      if (nfull) HT(gemm_f64(g, true, false, false, st));
      if (rest) {
        GemmArgs h = g;
        h.K = 2 * n * rest;
        h.A = aw.SU + stk * cw * nfull; h.B = aw.GGt + nd + 2L * n * n * cw * nfull;
        h.C = aw.lam_part + (long)nfull * L * k; h.batch = 1;
        HT(gemm_f64(h, true, false, false, st));
      }
      HT(sum_rows(aw.lam_part, nfull + (rest ? 1 : 0), (long)L * k, dunp, st));
    }
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Pfaffian: dF/dPhi for F = ga log|Psi| + gb e_L.
//  * log|Psi|: d log Pf / d phi(r_i) is the cofactor vector Y_i =
//    sum_j H_ji B^{s_i}_j (H = G~^{-1}), the vector whose gradient row dot is
//    the drift.
//  * e_L depends on Phi directly (the basis backward's derivative channels) and
//    through Y, with dF/dY_i = c Q_i, c = -gb/2, Q_i = lap phi_i + 2 grad J_i .
//    grad phi_i.  Y depends on H and on the rows B^s_j = A^{s s_j} phi_j:
//      dF/dH_ji = c T_ij,  T_ij = Q_i . B^{s_i}_j (unpaired j: Q_i . U^{s_i}_l);
//      dH = -H dG~ H gives dF/dG~ = -c (H T H)^T = -c Z^T, and as G~_ij =
//      phi_i^T A^{s_i s_j} phi_j with A^{s' s} = -(A^{s s'})^T,
//      dF/dphi_i = c sum_j (Z^T - Z)_ji B^{s_i}_j (the cofactor products with
//      X = Z^T - Z in place of H);
//      dF/dB^s_j = c sum_{i of spin s} H_ji Q_i, and B^s_j = A^{s s_j} phi_j
//      gives dF/dphi_j += c [H Q_up | H Q_dn]_j [A^{u s_j} ; A^{d s_j}].
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
pf_skew_kernel(const double* __restrict__ Z, long np, long tot, double* __restrict__ X) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const long w = idx / (np * np), ab = idx % (np * np), a = ab / np, b = ab % np;
  const double* z = Z + w * np * np;
  X[idx] = z[b * np + a] - z[a * np + b];
}

__global__ void __launch_bounds__(256)
pf_phibar_kernel(const double* __restrict__ Yt, const double* __restrict__ Yb, const double* __restrict__ ga,
                 const double* __restrict__ gb, long per_w, long tot, double* __restrict__ PB) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const long w = idx / per_w;
  double v = ga ? ga[w] * Yt[idx] : 0.0;
  if (gb) v += Yb[idx];
  PB[idx] = v;
}

// Q rows of the stacks times c_w = -gb[w]/2 (rows n .. 2n of every walker).
__global__ void __launch_bounds__(256)
pf_scale_q_kernel(double* __restrict__ SU, double* __restrict__ SD, const double* __restrict__ gb, int n, int Lp,
                  long tot) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const long per = (long)n * Lp, w = idx / per, o = w * 2 * per + per + idx % per;
  const double c = -0.5 * gb[w];
  SU[o] *= c;
  SD[o] *= c;
}

// M = D - D^T for D = dF/dG~ = ga/2 H^T - Z^T (Z = H T' H with the scaled Q rows;
// omitted without local-energy weights): M[a][b] = ga/2 (H[b][a] - H[a][b]) + Z[a][b] - Z[b][a].
__global__ void __launch_bounds__(256)
pf_gbar_kernel(const double* __restrict__ H, const double* __restrict__ Z, const double* __restrict__ ga, long np,
               long tot, double* __restrict__ M) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const long w = idx / (np * np), ab = idx % (np * np), a = ab / np, b = ab % np;
  const double* h = H + w * np * np;
  double v = ga ? 0.5 * ga[w] * (h[b * np + a] - h[a * np + b]) : 0.0;
  if (Z) {
    const double* z = Z + w * np * np;
    v += z[a * np + b] - z[b * np + a];
  }
  M[idx] = v;
}

// E[i][mu] -= Bb[row0 + i][half * Lp + mu] for i < ni (every walker).
__global__ void __launch_bounds__(256)
pf_sub_bb_kernel(double* __restrict__ E, const double* __restrict__ Bb, int ni, int Lp, int N, int row0, int half,
                 long tot) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  const long per = (long)ni * Lp, w = idx / per, i = (idx % per) / Lp, mu = idx % Lp;
  E[w * (long)N * Lp + i * Lp + mu] -= Bb[(w * N + row0 + i) * 2L * Lp + (long)half * Lp + mu];
}

__global__ void __launch_bounds__(256) pf_half_kernel(double* __restrict__ X, long per, long stride, long tot) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  X[(idx / per) * stride + idx % per] *= 0.5;
}

__global__ void __launch_bounds__(256) pf_zero_kernel(double* __restrict__ X, long per, long stride, long tot) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= tot) return;
  X[(idx / per) * stride + idx % per] = 0.0;
}

// dcoef (optional): pairing-coefficient gradients, per walker
// [Wk][3 L L + 2 L k]: A^{ud}, A^{uu}, A^{dd} (the same-spin ones as gradients
// with respect to skew matrices), then U^u and U^d [L][k].
static hipError_t pf_backward(const SysDev& s, const WalkDev& w, const AdjWork& aw, const double* ga,
                              const double* gb, double* dcoef, hipStream_t st) {
  const int Wk = w.Wk, Lp = s.Lp, N = s.N, n = s.nu, nd = s.nd, np = s.npf, pk = s.pk, L = s.L;
  const long rowst = (long)N * Lp, stk = 2L * n * Lp, nn = (long)np * np;
  if (gb || dcoef) {   // the stacks [Phi; Q] of both spins
    hipLaunchKernelGGL(stack_basis_kernel, dim3((unsigned)((long)Wk * N)), dim3(256), 0, st, s, w, aw.SU, aw.SD);
    HT(hipGetLastError());
  }
  if (gb) {
    {   // Q rows times c = -gb/2: every product below carries the factor
      const long tot = (long)Wk * n * Lp;
      hipLaunchKernelGGL(pf_scale_q_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, aw.SU, aw.SD, gb,
                         n, Lp, tot);
      HT(hipGetLastError());
    }
    // T rows of the up then the down electrons (rows N.. stay zero)
    for (int sp = 0; sp < 2; ++sp) {
      const int i0 = sp ? n : 0, ni = sp ? nd : n;
      if (ni == 0) continue;
      const double* Q = (sp ? aw.SD : aw.SU) + (long)n * Lp;
      GemmArgs g = gemm_args(ni, N, Lp);
      g.A = Q; g.lda = Lp; g.a_bs = stk;
      g.B = sp ? w.Bd : (const double*)w.P; g.ldb = Lp; g.b_bs = rowst;
      g.C = aw.pfT + (long)i0 * np; g.ldc = np; g.c_bs = nn; g.batch = Wk;
      HT(gemm_f64(g, false, true, false, st));
      if (pk > 0) {
        GemmArgs u = gemm_args(ni, pk, Lp);
        u.A = Q; u.lda = Lp; u.a_bs = stk;
        u.B = s.Upf + (long)sp * pk * Lp; u.ldb = Lp; u.b_bs = 0;
        u.C = aw.pfT + (long)i0 * np + N; u.ldc = np; u.c_bs = nn; u.batch = Wk;
        HT(gemm_f64(u, false, true, false, st));
      }
    }
    // Z = H T H, then X = Z^T - Z (into pfZ1)
    {
      GemmArgs g = gemm_args(np, np, np);
      g.A = w.A; g.lda = np; g.a_bs = nn;
      g.B = aw.pfT; g.ldb = np; g.b_bs = nn;
      g.C = aw.pfZ1; g.ldc = np; g.c_bs = nn; g.batch = Wk;
      HT(gemm_f64(g, false, false, false, st));
      g.A = aw.pfZ1; g.B = w.A; g.C = aw.pfZ;
      HT(gemm_f64(g, false, false, false, st));
      const long tot = nn * Wk;
      hipLaunchKernelGGL(pf_skew_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, aw.pfZ, (long)np,
                         tot, aw.pfZ1);
      HT(hipGetLastError());
    }
    HT(launch_pf_Y_products(s, w, aw.pfZ1, aw.pfY, st));
    // [H Q_up | H Q_dn] rows j < N, then times [A^{u s_j} ; A^{d s_j}] = Kcat_{s_j}^T
    {
      GemmArgs g = gemm_args(N, Lp, n);
      g.A = w.A; g.lda = np; g.a_bs = nn;
      g.B = aw.SU + (long)n * Lp; g.ldb = Lp; g.b_bs = stk;
      g.C = aw.pfBb; g.ldc = 2L * Lp; g.c_bs = 2 * rowst; g.batch = Wk;
      HT(gemm_f64(g, false, false, false, st));
      if (nd > 0) {
        g.K = nd;
        g.A = w.A + n;
        g.B = aw.SD + (long)n * Lp;
        g.C = aw.pfBb + Lp;
        HT(gemm_f64(g, false, false, false, st));
      }
      for (int sp = 0; sp < 2; ++sp) {
        const int j0 = sp ? n : 0, nj = sp ? nd : n;
        if (nj == 0) continue;
        // with no down electrons only the H Q_up half exists
        GemmArgs k = gemm_args(nj, Lp, nd > 0 ? 2 * Lp : Lp);
        k.A = aw.pfBb + (long)j0 * 2 * Lp; k.lda = 2L * Lp; k.a_bs = 2 * rowst;
        k.B = sp ? s.Kcat_d : s.Kcat_u; k.ldb = 2L * Lp; k.b_bs = 0;
        k.C = aw.pfY + (long)j0 * Lp; k.ldc = Lp; k.c_bs = rowst; k.batch = Wk;
        k.accumulate = 1;
        HT(gemm_f64(k, false, true, false, st));
      }
    }
  }
  const long tot = rowst * Wk;
  hipLaunchKernelGGL(pf_phibar_kernel, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, w.Yt, aw.pfY, ga, gb,
                     rowst, tot, aw.PB);
  HT(hipGetLastError());
  if (!dcoef) return hipSuccess;
  // pairing coefficients: G~_ij = phi_i^T A^{s_i s_j} phi_j (A^{du} = -A^{ud T}) and
  // B^s_j = A^{s s_j} phi_j give, with M = D - D^T and Bb = [H Q'_u | H Q'_d],
  //   out_{st} = f (Phi_s^T (M_{st} Phi_t - Bb_t[s rows]) + Bb_s[t rows]^T Phi_t)
  // (f = 1/2 for the skew same-spin blocks, 1 for A^{ud}), and
  //   dU^s = Phi_s^T M[s rows, N:] + Q'_s^T H[N:, s cols]^T.
  const long per = 3L * L * L + 2L * L * pk, totm = nn * Wk;
  hipLaunchKernelGGL(pf_gbar_kernel, dim3((unsigned)((totm + 255) / 256)), dim3(256), 0, st, w.A,
                     gb ? aw.pfZ : nullptr, ga, (long)np, totm, aw.pfZ1);
  HT(hipGetLastError());
  const int blk[3][2] = {{0, 1}, {0, 0}, {1, 1}};   // (s, t): A^{ud}, A^{uu}, A^{dd}
  for (int q = 0; q < 3; ++q) {
    const int sg = blk[q][0], tg = blk[q][1];
    const int s0 = sg ? n : 0, ns = sg ? nd : n, t0 = tg ? n : 0, nt = tg ? nd : n;
    double* O = dcoef + (long)q * L * L;
    if (ns == 0 || nt == 0) {
      const long tz = (long)Wk * L * L;
      hipLaunchKernelGGL(pf_zero_kernel, dim3((unsigned)((tz + 255) / 256)), dim3(256), 0, st, O, (long)L * L, per,
                         tz);
      HT(hipGetLastError());
      continue;
    }
    const double* Phs = sg ? aw.SD : aw.SU;   // Phi rows of spin s (rows 0 .. ns of the stack)
    const double* Pht = tg ? aw.SD : aw.SU;
    // E = M[s rows, t cols] Phi_t  (into pfY rows 0 .. ns)
    GemmArgs g = gemm_args(ns, Lp, nt);
    g.A = aw.pfZ1 + (long)s0 * np + t0; g.lda = np; g.a_bs = nn;
    g.B = Pht; g.ldb = Lp; g.b_bs = stk;
    g.C = aw.pfY; g.ldc = Lp; g.c_bs = rowst; g.batch = Wk;
    HT(gemm_f64(g, false, false, false, st));
    if (gb) {
      const long te = (long)Wk * ns * Lp;
      hipLaunchKernelGGL(pf_sub_bb_kernel, dim3((unsigned)((te + 255) / 256)), dim3(256), 0, st, aw.pfY, aw.pfBb, ns,
                         Lp, N, s0, tg, te);
      HT(hipGetLastError());
    }
    // O = Phi_s^T E (+ Bb_s[t rows]^T Phi_t)
    GemmArgs o = gemm_args(L, L, ns);
    o.A = Phs; o.lda = Lp; o.a_bs = stk;
    o.B = aw.pfY; o.ldb = Lp; o.b_bs = rowst;
    o.C = O; o.ldc = L; o.c_bs = per; o.batch = Wk;
    HT(gemm_f64(o, true, false, false, st));
    if (gb) {
      GemmArgs b = gemm_args(L, L, nt);
      b.A = aw.pfBb + (long)t0 * 2 * Lp + (long)sg * Lp; b.lda = 2L * Lp; b.a_bs = 2 * rowst;
      b.B = Pht; b.ldb = Lp; b.b_bs = stk;
      b.C = O; b.ldc = L; b.c_bs = per; b.batch = Wk;
      b.accumulate = 1;
      HT(gemm_f64(b, true, false, false, st));
    }
    if (q > 0) {
      const long th = (long)Wk * L * L;
      hipLaunchKernelGGL(pf_half_kernel, dim3((unsigned)((th + 255) / 256)), dim3(256), 0, st, O, (long)L * L, per,
                         th);
      HT(hipGetLastError());
    }
  }
  for (int sg = 0; sg < 2 && pk > 0; ++sg) {
    const int s0 = sg ? n : 0, ns = sg ? nd : n;
    double* O = dcoef + 3L * L * L + (long)sg * L * pk;
    if (ns == 0) {
      const long tz = (long)Wk * L * pk;
      hipLaunchKernelGGL(pf_zero_kernel, dim3((unsigned)((tz + 255) / 256)), dim3(256), 0, st, O, (long)L * pk, per,
                         tz);
      HT(hipGetLastError());
      continue;
    }
    const double* S = sg ? aw.SD : aw.SU;
    GemmArgs u = gemm_args(L, pk, ns);
    u.A = S; u.lda = Lp; u.a_bs = stk;
    u.B = aw.pfZ1 + (long)s0 * np + N; u.ldb = np; u.b_bs = nn;
    u.C = O; u.ldc = pk; u.c_bs = per; u.batch = Wk;
    HT(gemm_f64(u, true, false, false, st));
    if (gb) {
      GemmArgs v = gemm_args(L, pk, ns);
      v.A = S + (long)n * Lp; v.lda = Lp; v.a_bs = stk;
      v.B = w.A + (long)N * np + s0; v.ldb = np; v.b_bs = nn;
      v.C = O; v.ldc = pk; v.c_bs = per; v.batch = Wk;
      v.accumulate = 1;
      HT(gemm_f64(v, true, true, false, st));
    }
  }
  return hipSuccess;
}

// Contraction coefficients: phi_c = sum_t C_t psi_{mu_t} and its gradient and
// Laplacian are linear in C, so with dF/dphi (PB), dF/d(lap phi) = c Y and
// dF/d(grad phi) = 2 c grad J Y (c = -gb/2) over the orbitals
//   dF/dC_t = sum_i PB[i][c_t] psi_mu(r_i) + c Y[i][c_t] (lap psi_mu + 2 grad J_i . grad psi_mu)(r_i),
// the primitives' values and derivatives recomputed per electron.  One
// workgroup per walker, one thread per orbital and its coefficients.
__global__ void __launch_bounds__(256)
con_grad_kernel(SysDev s, WalkDev w, const double* __restrict__ PB, const double* __restrict__ gb,
                double* __restrict__ out) {
  const int wk = blockIdx.x;
  const double cq = gb ? -0.5 * gb[wk] : 0.0;
  const double* r = w.r + (long)wk * s.N * 3;
  const double* pb = PB + (long)wk * s.N * s.Lp;
  const double* yt = w.Yt + (long)wk * s.N * s.Lp;
  const double* gJ = w.gJ + (long)wk * s.N * 4;
  const int nnz = s.con_ptr[s.L];
  double* o = out + (long)wk * nnz;
  for (int c = threadIdx.x; c < s.L; c += blockDim.x)
    for (int k = s.con_ptr[c]; k < s.con_ptr[c + 1]; ++k) {
      const int mu = s.con_idx[k];
      double acc = 0.0;
      for (int i = 0; i < s.N; ++i) {
        double v, bx, by, bz, lp;
        basis_vgl(s, mu, r[3 * i], r[3 * i + 1], r[3 * i + 2], v, bx, by, bz, lp);
        acc += pb[(long)i * s.Lp + c] * v;
        if (gb) acc += cq * yt[(long)i * s.Lp + c] * (lp + 2.0 * (bx * gJ[4 * i] + by * gJ[4 * i + 1] + bz * gJ[4 * i + 2]));
      }
      o[k] = acc;
    }
}

hipError_t launch_forces(const SysDev& s, const WalkDev& w, const AdjWork& aw, const double* ga,
                         const double* gb, int per_walker, double* dR, double* dzeta, double* dlambda,
                         double* djas, double* dr, double* dj1_inh, double* dj3, double* djb_zeta,
                         double* dunpaired, double* dcon, double* dpf_uu, double* dpf_dd,
                         double* dunpaired_dn, hipStream_t st) {
  const int Wk = w.Wk, Lp = s.Lp, N = s.N;
  if (s.pairing) {
    const bool coef = dlambda || dunpaired || dpf_uu || dpf_dd || dunpaired_dn;
    HT(pf_backward(s, w, aw, ga, gb, coef ? aw.pfD : nullptr, st));
    if (coef) {   // [Wk][A^{ud} | A^{uu} | A^{dd} | U^u | U^d] -> the outputs
      const long L2 = (long)s.L * s.L, Lk = (long)s.L * s.pk, per = 3 * L2 + 2 * Lk;
      const double* src = aw.pfD;
      if (!per_walker) {
        HT(sum_rows(aw.pfD, Wk, per, aw.pfS, st));
        src = aw.pfS;
      }
      const int rows = per_walker ? Wk : 1;
      double* dst[5] = {dlambda, dpf_uu, dpf_dd, s.pk ? dunpaired : nullptr, s.pk ? dunpaired_dn : nullptr};
      const long off[5] = {0, L2, 2 * L2, 3 * L2, 3 * L2 + Lk};
      const long len[5] = {L2, L2, L2, Lk, Lk};
      for (int q = 0; q < 5; ++q)
        if (dst[q] && len[q] > 0)
          HT(hipMemcpy2DAsync(dst[q], sizeof(double) * len[q], src + off[q], sizeof(double) * per,
                              sizeof(double) * len[q], rows, hipMemcpyDeviceToDevice, st));
    }
  } else {
    HT(geminal_backward(s, w, aw, ga, gb, per_walker, dlambda, dunpaired, st));
  }
  // 8. basis and Jastrow/Coulomb backward (over the primitives of a contracted basis)
  double* drw = dr ? dr : aw.dr;
  if (s.Lq && dcon) {
    hipLaunchKernelGGL(con_grad_kernel, dim3(Wk), dim3(256), 0, st, s, w, aw.PB, gb, per_walker ? dcon : aw.dcw);
    HT(hipGetLastError());
  }
  if (s.Lq) {
    const int lqp = (s.Lq + 31) / 32 * 32;
    const unsigned rows = (unsigned)((long)Wk * N);
    hipLaunchKernelGGL(prim_rows_kernel, dim3(rows), dim3(256), 0, st, s, aw.PB, lqp, aw.PBq);
    HT(hipGetLastError());
    hipLaunchKernelGGL(prim_rows_kernel, dim3(rows), dim3(256), 0, st, s, w.Yt, lqp, aw.Ytq);
    HT(hipGetLastError());
    SysDev sq = s;
    sq.L = s.Lq; sq.Lp = lqp; sq.Lq = 0;
    WalkDev wq = w;
    wq.Yt = aw.Ytq;
    hipLaunchKernelGGL(basis_backward_kernel, dim3(Wk), dim3(kBackThreads), 0, st, sq, wq, aw.PBq, gb, drw, aw.Rbar,
                       aw.zbar, aw.tmu, 0);
  } else {
    hipLaunchKernelGGL(basis_backward_kernel, dim3(Wk), dim3(kBackThreads), 0, st, s, w, aw.PB, gb, drw, aw.Rbar,
                       aw.zbar, aw.tmu, 0);
  }
  HT(hipGetLastError());
  if (s.LJ) HT(launch_jastrow3_backward(s, w, aw, ga, gb, drw, st));
  hipLaunchKernelGGL(jastrow_backward_kernel, dim3(Wk), dim3(256), 0, st, s, w, ga, gb, drw, aw.Rbar, aw.jbar);
  HT(hipGetLastError());
  // 9. outputs
  const int nj = s.n_nuc + (s.j2_form == 1 ? 2 : (s.j2_form == 2 ? 8 : 0));
  if (per_walker) {
    if (dR) HT(hipMemcpyAsync(dR, aw.Rbar, sizeof(double) * Wk * s.n_nuc * 3, hipMemcpyDeviceToDevice, st));
    if (dzeta) HT(hipMemcpyAsync(dzeta, aw.zbar, sizeof(double) * Wk * s.nprim(), hipMemcpyDeviceToDevice, st));
    if (djas) HT(hipMemcpyAsync(djas, aw.jbar, sizeof(double) * Wk * nj, hipMemcpyDeviceToDevice, st));
    if (s.LJ) {
      const size_t LJ = s.LJ;
      if (dj1_inh) HT(hipMemcpyAsync(dj1_inh, aw.jdm, sizeof(double) * Wk * 2 * LJ, hipMemcpyDeviceToDevice, st));
      if (dj3) HT(hipMemcpyAsync(dj3, aw.jdM, sizeof(double) * Wk * 3 * LJ * LJ, hipMemcpyDeviceToDevice, st));
      if (djb_zeta) HT(hipMemcpyAsync(djb_zeta, aw.jzbar, sizeof(double) * Wk * LJ, hipMemcpyDeviceToDevice, st));
    }
  } else {
    if (s.Lq && dcon) HT(sum_rows(aw.dcw, Wk, s.nnz_con, dcon, st));
    if (dR) HT(sum_rows(aw.Rbar, Wk, (long)s.n_nuc * 3, dR, st));
    if (dzeta) HT(sum_rows(aw.zbar, Wk, s.nprim(), dzeta, st));
    if (djas) HT(sum_rows(aw.jbar, Wk, nj, djas, st));
    if (s.LJ) {
      const long LJ = s.LJ;
      if (dj1_inh) HT(sum_rows(aw.jdm, Wk, 2 * LJ, dj1_inh, st));
      if (dj3) HT(sum_rows(aw.jdM, Wk, 3 * LJ * LJ, dj3, st));
      if (djb_zeta) HT(sum_rows(aw.jzbar, Wk, LJ, djb_zeta, st));
    }
  }
  return hipSuccess;
}

}  // namespace qmc
