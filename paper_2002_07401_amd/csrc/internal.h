// Internal declarations of the gfx950 JAGP library: device data of a system
// and of a walker batch, device helpers for the basis and Jastrow terms, and
// the kernel launchers the C ABI layer calls.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include "../../include/qmc.h"

namespace qmc {

// ---------------------------------------------------------------------------
// sizes
// ---------------------------------------------------------------------------
constexpr int kMaxNuc = 4096;
constexpr int kLuMaxN = 128;      // one-workgroup (register / LDS) Sherman-Morrison limit
constexpr int kLuRowMax = 96;     // register (row-per-thread) Gauss-Jordan limit
constexpr int kPropRowsMin = 8;   // smallest rows-per-workgroup the autotuner may pick
// P rows per proposal workgroup (swept on MI355X: 8 for FP64 rows, 16 for the
// narrower FP32 / BF16 rows); rdet_part holds ceil(n / kPropRowsMin) partial
// sums per walker, so no choice may go below kPropRowsMin
constexpr int kPropRowsF64 = 8, kPropRowsNarrow = 16;
static_assert(kPropRowsF64 >= kPropRowsMin && kPropRowsNarrow >= kPropRowsMin, "partial-sum buffer too small");
constexpr int kMaxNucBack = 256;  // nuclei handled by the Jastrow backward kernel
constexpr int kFuseMaxLp = 1024;   // accept fused with the next set-up: psi(r') staged in LDS
constexpr int kMaxLJ = 1024;       // Jastrow basis functions (J1 inhomogeneous, J3/4)
constexpr int kMaxLq = 2048;       // primitives of a contracted basis (LDS stage of the basis kernel)
constexpr int kBigMaxN = 1024;    // blocked Gauss-Jordan limit
constexpr int kWbMax = 64;        // capacity of the delayed-update buffer (moves between refreshes)
constexpr int kGjPanel = 64;      // panel width of the blocked Gauss-Jordan
constexpr int kLamTileK = 16;     // Lambda tile mask granularity: rows (GEMM K step) ...
constexpr int kLamTileN = 64;     // ... and columns (GEMM N tile)
constexpr int kOzMaxSlices = 8;   // int8 digits per FP64 row in the error-free products
constexpr int kOzSlices = 7;      // digits used by the refined evaluation (error 7e-14 of max|x| max|y| K)
// Screened proposals (QMC_REFINED): the basis functions skipped at r' change the
// determinant ratio by at most this much in total (absolute)
constexpr double kScreenTol = 1e-13;

inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

// Record msg as this host thread's last error (qmc_last_error) and return st.
qmc_status set_error(qmc_status st, const char* msg);

// BF16 storage (the bit pattern).  Widening is exact; narrowing rounds to
// nearest even through FP32 (NaN stays a quiet NaN).
struct bf16s {
  uint16_t x;
  bf16s() = default;
  __host__ __device__ static uint16_t narrow(float f) {
    uint32_t u;
    __builtin_memcpy(&u, &f, 4);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
  }
  __host__ __device__ explicit bf16s(float f) : x(narrow(f)) {}
  __host__ __device__ explicit bf16s(double d) : x(narrow((float)d)) {}
  __host__ __device__ explicit operator float() const {
    const uint32_t u = (uint32_t)x << 16;
    float f;
    __builtin_memcpy(&f, &u, 4);
    return f;
  }
  __host__ __device__ explicit operator double() const { return (double)(float)*this; }
};

// Device-resident description of one system.
struct SysDev {
  int n_nuc, L, Lp, nu, nd, N;
  int j1_form, j2_form;
  double j2[8];      // two-body parameters as created (host copy)
  const double* j2d; // [8] the same on the device: kernels read these, so that
                     // qmc_system_set_params can replace them without a host sync
  int precision, refresh_every;
  // reduced-precision storage of Phi and P (the move path): FP32 in QMC_W_FP32
  // and QMC_MIXED, BF16 in QMC_MIXED_BF16 (FP64 in QMC_FP64 and QMC_REFINED)
  __host__ __device__ bool f32() const {
    return precision == QMC_W_FP32 || precision == QMC_MIXED || precision == QMC_MIXED_BF16;
  }
  // QMC_REFINED: FP64 storage, refined int8 products, screened proposals
  // (determinant systems)
  __host__ __device__ bool screened() const { return precision == QMC_REFINED && !pairing; }
  // QMC_REFINED Pfaffian: the B rows from int8 digit products, FP64 otherwise
  __host__ __device__ bool pf_refined() const { return precision == QMC_REFINED && pairing; }
  __host__ __device__ bool bf16() const { return precision == QMC_MIXED_BF16; }
  __host__ __device__ bool refined() const { return precision == QMC_MIXED || precision == QMC_MIXED_BF16; }
  // 0: FP64, 1: FP32, 2: BF16 storage
  __host__ __device__ int store() const { return f32() ? (bf16() ? 2 : 1) : 0; }
  __host__ __device__ int prop_rows() const { return store() == 0 ? kPropRowsF64 : kPropRowsNarrow; }
  // entries per basis function of the transposed rows of the screened
  // proposals: the N electrons, then the nk unpaired orbitals' values
  __host__ __device__ int pt_ld() const { return N + nk; }
  double* R;        // [A][3]
  double* Z;        // [A]
  double* j1_b;     // [A]
  int* center;      // [L]
  int* kind;        // [L]  0 s | 1..3 p(x,y,z) | 4..8 d(xy,yz,zx,x2-y2,2z2-x2-y2), plus
                    //      kSlaterBit for a Slater radial factor e^{-zeta r}
  double* zeta;     // [L]
  double* lam;      // [Lp][Lp]  Lambda, zero padded
  double* lamT;     // [Lp][Lp]  Lambda^T
  float* lam32;     // [Lp][Lp]  FP32 copies (precision QMC_W_FP32)
  float* lamT32;
  uint16_t* lamB;   // QMC_MIXED_BF16: [2][2][Lp][Lp] BF16, half h (0: Lambda^T, the
                    // transposed operand of P_up = Phi_up Lambda; 1: Lambda, of
                    // P_dn = Phi_dn Lambda^T), hi then lo = bf16(x - hi)
  int* cptr;        // [A+1] basis functions of nucleus a: cmu[cptr[a] .. cptr[a+1])
  int* cmu;         // [L]
  double4* bfn;     // [L] packed (x, y, z) of the function's centre and its zeta
  // nonzero flags of the [kLamTileK x kLamTileN] tiles of Lambda and Lambda^T
  // ([Lp/16][Lp/64]); the P products skip zero tiles (banded Lambda)
  uint8_t* lam_mask;
  uint8_t* lamT_mask;
  int np;           // n rounded up to 64 (blocked Gauss-Jordan, n > kLuRowMax)
  // Jastrow basis chi (onebody_J_inh, threebody_jastrow); LJ = 0: absent
  int LJ;
  double4* jbfn;    // [LJ] centre and zeta
  int* jkind;       // [LJ] as kind
  double* jm;       // [2][LJ] one-body inhomogeneous coefficients, up then down
  double* M3;       // [2LJ][2LJ] [[M_uu, M_ud], [M_ud^T, M_dd]] (symmetric)
  int* jcenter;     // [LJ] nucleus of each Jastrow-basis function
  int* jcptr;       // [A+1] Jastrow-basis functions of nucleus a: jcmu[jcptr[a] .. jcptr[a+1])
  int* jcmu;        // [LJ]
  // Contracted orbitals (Lq > 0): center, kind, zeta and bfn then describe Lq
  // primitives and orbital c < L is sum_t con_coef[t] psi_{con_idx[t]},
  // t in [con_ptr[c], con_ptr[c+1]); pri_* hold the same matrix by primitive
  // (orbitals c with coefficient pri_coef[t] = C[mu][c] for t in
  // [pri_ptr[mu], pri_ptr[mu+1])), so that sum_c C[mu][c] y_c is one short loop.
  int Lq;
  int nnz_con;       // number of contraction coefficients (con_ptr[L])
  int* con_ptr;      // [L+1]
  int* con_idx;      // [nnz]
  double* con_coef;  // [nnz]
  int* pri_ptr;      // [Lq+1]
  int* pri_idx;      // [nnz]
  double* pri_coef;  // [nnz]
  __host__ __device__ int nprim() const { return Lq ? Lq : L; }
  // Unpaired orbitals (nk = n_up - n_dn > 0): W is n_up x n_up, its columns
  // n_dn .. n_up-1 hold psi(r_i) . U[:, l].  Row l of Uph is U[:, l] (zero
  // padded to Lp), the fixed "P row" of column n_dn + l; UphS is the copy in the
  // move rows' storage type (Uph, Uph32 or a BF16 copy).
  int nk;
  double* Uph;       // [nk][Lp]
  float* Uph32;      // [nk][Lp] (reduced-precision storage)
  const void* UphS;  // [nk][Lp]
  // Pfaffian pairing (pairing = 1): G~ is npf x npf (npf = N + pk, pk
  // unpaired orbitals as fictitious electrons), G~_ij = psi(r_i) . B^{s_i}_j
  // with the rows B^s_j = psi(r_j)^T K^{s s_j}, K^{s s'} = (A^{s s'})^T; the
  // walkers keep B^u in P and B^d in Bd.  FP64 (QMC_REFINED: the evaluation's
  // B rows from int8 digit products), npf <= kLuRowMax.
  int pairing, npf, pk;
  double* Kuu;       // [Lp][Lp]  (A^{uu})^T
  double* Kud;       // [Lp][Lp]  (A^{ud})^T
  double* Kdu;       // [Lp][Lp]  (A^{du})^T = -A^{ud}
  double* Kdd;       // [Lp][Lp]  (A^{dd})^T
  double* Upf;       // [2][pk][Lp] unpaired orbitals of up, then down electrons
  double* Kcat_u;    // [Lp][2Lp] [K^{uu} | K^{du}]: the B rows of a moved up electron
  double* Kcat_d;    // [Lp][2Lp] [K^{ud} | K^{dd}]: the B rows of a moved down electron
  // int8 digits of Lambda for the error-free products (refined modes): tiles
  // [2][oz_s][Lp * Lp] (rows of Lambda^T, then rows of Lambda) and one exponent
  // per row [2][Lp]; for a QMC_REFINED Pfaffian the rows of the four K^T
  // (uu, ud, du, dd): [4][oz_s][Lp * Lp] and [4][Lp], with an Lp x Lp FP64
  // work array for the transposes
  int oz_s;
  int8_t* oz_lam;
  int* oz_elam;
  double* oz_tmp;
};

// Device state of a batch of walkers.
struct WalkDev {
  int Wk;
  double* r;        // [Wk][N][3]
  void* phi;        // [Wk][N][Lp]  basis values (double or float)
  void* P;          // [Wk][N][Lp]  rows i<nu: Phi_up Lambda ; rows i>=nu: Phi_dn Lambda^T
  double* W;        // [Wk][nu][nu]  columns: n_dn paired, then nk unpaired
  double* A;        // [Wk][nu][nu]  W^{-1}
  double* Yt;       // [Wk][N][Lp]  eval workspace: Yt_up = A^T P_dn, Yt_dn = A P_up
  double* D;        // [Wk][N][4]   grad det/det (3), lap det/det
  double* logdet;   // [Wk]
  double* detsign;  // [Wk]
  int* singular;    // [Wk]
  double* logabs;   // [Wk] log|Psi| tracked through moves
  double* sign;     // [Wk]
  double* J;        // [Wk] Jastrow exponent tracked through moves
  // pending proposal
  double* psi_new;  // [Wk][Lp] basis values at r' (zero-padded)
  double* w_new;    // [Wk][nmax] new row (up) or column (down) of W
  double* rdet;     // [Wk]
  double* dJ;       // [Wk]
  double* r_new;    // [Wk][3]
  double* ratio;    // [Wk] ratio of the pending proposal
  uint8_t* acc;     // [Wk]
  double* rdet_part;  // [Wk][S] partial determinant ratios (one per proposal block)
  double* gdet_part;  // [Wk][S][3] partial gradients (drift at r')
  double* gJ_new;     // [Wk][3] Jastrow gradient at r'
  double* gpsi_new;   // [Wk][3][Lp] basis gradients at r' (drift requests)
  double* gJ;         // [Wk][N][4] Jastrow gradient (3) and Laplacian per electron
  double* drift;      // [Wk][N][3] grad_i log|Psi| of the last evaluation
  double* phi64;      // [Wk][N][Lp] FP64 evaluation work arrays (QMC_MIXED only)
  double* P64;        // [Wk][N][Lp]
  // blocked Gauss-Jordan (n > kLuRowMax) and two-pass Sherman-Morrison
  // (n > kLuMaxN) work arrays
  double* T;          // [Wk][np][np] identity-padded working copy of W
  double* Tsave;      // [Wk][kGjPanel][np] pivot rows of the current panel, before it
  int* rowk;          // [Wk][np] step at which row i was pivoted (-1: not yet)
  int* prow;          // [Wk][np] row pivoted at step k
  double* pivv;       // [Wk][np] pivot value of step k
  // Delayed updates since the last refresh (A0 = W^{-1} at the refresh):
  //   W^{-1} = A0 - V S^{-1} (D^T A0)    (up moves: v_i = A0[:, e_i], d_i = row change)
  //   W^{-1} = A0 - (A0 D) S^{-T} V^T    (down moves: v_i = A0[e_i, :], d_i = column change)
  // with S_ij = d_i . v_j + [i == j] (m x m); one move direction per buffer.
  int* wm;            // [Wk] stored updates m
  double* wv;         // [Wk][kb][n] v_i
  double* wd;         // [Wk][kb][n] d_i
  double* wS;         // [Wk][kb][kb] S^{-1}
  double* cvec;       // [Wk][n] current W^{-1} column e (up) or row e (down) of the pending proposal
  double* v0;         // [Wk][n] A0's column / row e of the pending proposal
  double* tz;         // [Wk][2][kb] t = D^T v0 and z = S^{-1} t of the pending proposal
  int kb;             // buffer capacity (<= kWbMax)
  // Jastrow-basis state (LJ > 0): chi(r_i), h_i = M^{ss} chi(r_i) over the
  // electron's own spin block, G_s = sum of M^{s s'} chi(r_j) over all j of
  // spin s' (i.e. [G_u; G_d] = M3 [X_u; X_d], X_s = sum_{j in s} chi(r_j)),
  // chi at the pending proposal's r', and per-electron evaluation terms
  double* chi;        // [Wk][N][LJ]
  double* hv;         // [Wk][N][LJ]
  double* G3;         // [Wk][2][LJ]
  double* chi_new;    // [Wk][LJ]
  double* j3e;        // [Wk][N][5] value part, gradient (3), Laplacian
  double* qbuf;       // [Wk][4][Lq] primitive values (and gradients) at r' (contracted orbitals)
  double* Bd;         // [Wk][N][Lp] B^d rows (Pfaffian pairing; B^u rows are in P)
  double* pfB;        // [Wk][2][Lp] B^u, B^d rows of the proposal's r' (Pfaffian pairing)
  double* pfT;        // [Wk][N][Lp] work rows of the Pfaffian log-derivatives
  // int8 digits of the FP64 basis rows (refined modes): tiles of the up rows
  // [oz_s][Wk * n_up], then of the down rows [oz_s][Wk * n_dn] (rows padded to 32,
  // Lp digits each), and one exponent per row [Wk * n_up + Wk * n_dn]
  int8_t* oz_phi;
  int* oz_ephi;
  // screened proposals (QMC_REFINED): P transposed per walker, PT[w][mu][i] =
  // P[w][i][mu] for the N electrons and PT[w][mu][N + l] = U[mu][l] for the
  // nk unpaired orbitals ([Wk][Lp][N + nk]: one basis function's column over
  // the rows an up move streams, the down electrons and the unpaired
  // orbitals, and over the up rows a down move streams is contiguous); per
  // walker and spin the largest |value| of each column over those rows
  // [Wk][2][Lp] (0: up rows, 1: down rows and unpaired orbitals); the pending
  // proposal's kept basis functions (index and value at r') and their count
  double* PT;
  double* cmax;
  int* muk;
  double* psk;
  int* nkeep;
  // (QMC_REFINED) the positions at which each electron's P row was last built
  // [Wk][N][3]; the rows of a P half whose electron has moved since, as
  // indices into the half's row order (walker * n + i), and their count per
  // half; the int8 row exponents in that compacted order
  double* rpos_P;
  int* dirty_idx;
  int* dirty_cnt;
  int* dirty_blk;   // per block of 256 rows: count, then offset [Wk * N / 256 + 1]
  int* oz_ephi_c;
};

// Workspace of the reverse pass (allocated on the first qmc_forces call).
struct AdjWork {
  double* SU;       // [Wk][2n][Lp]  [Phi_U ; Q_U]
  double* SD;       // [Wk][2n][Lp]  [Phi_D ; Q_D]
  double* VQ;       // [Wk][n][n]
  double* T1;       // [Wk][n][n]
  double* M;        // [Wk][n][n]
  double* GG;       // [Wk][n][2n]   [G_W | G_V]
  double* GGt;      // [Wk][2n][n]   [G_W ; G_V]
  double* XZ;       // [Wk][2n][Lp]  [X_U ; Z_U]
  double* XD;       // [Wk][n][Lp]
  double* PB;       // [Wk][N][Lp]   dF/dPhi
  double* tmu;      // [Wk][L or Lq][3]
  double* Rbar;     // [Wk][A][3]
  double* zbar;     // [Wk][L or Lq]
  double* jbar;     // [Wk][A + n_j2]
  double* dr;       // [Wk][N][3]    used when the caller passes no dr
  double* lam_part; // [chunks][L][L]
  double* PBq;      // [Wk][N][Lq pad 32] dF/dPhi over the primitives (contracted orbitals)
  double* Ytq;      // [Wk][N][Lq pad 32] Yt over the primitives
  // Jastrow basis (LJ > 0): rows [Wk][N][LJp] of u, gvec, a chi + c, dF/dchi and
  // M^{ss} u; per walker X_s, U_s [4][LJ], M3 U [2][LJ], dF/dm [2][LJ],
  // sum u chi^T [2][LJ][LJ], dF/dM [3][LJ][LJ], exponent gradients [LJ] and
  // per-function position sums [LJ][3]; drift as 4-vectors [Wk][N][4]
  int LJp;
  double *ju, *jgv, *jac, *jpb, *jhu, *jX, *jH, *jdm, *jC, *jdM, *jzbar, *jtmu, *drift4;
  // Pfaffian (npf = N + k): T = [Q_i . B^{s_i}_j] and the products H T, H T H
  // [Wk][npf][npf]; [H Q_up | H Q_dn] rows [Wk][N][2 Lp]; dF/dPhi through G~
  // and the B rows [Wk][N][Lp]
  double *pfT, *pfZ1, *pfZ, *pfBb, *pfY;
  // pairing-coefficient gradients per walker [Wk][3 L L + 2 L k] and summed
  double *pfD, *pfS;
  // contracted orbitals: per-walker gradients of the coefficients [Wk][nnz]
  double* dcw;
  int chunk_walkers;
  int chunks;
};
// Arguments of the persistent multi-system phase kernels.
struct MultiArgs {
  const SysDev* sysv;             // [members] device copies
  const WalkDev* wkv;             // [members]
  const long long* steps;         // [members] attempted moves so far (device)
  const int* rows;                // [members] P rows per proposal work item
  const double* const* disp;      // [members] explicit displacements [n_steps][Wk][3], or null
  const double* const* unif;      // [members] explicit uniforms [n_steps][Wk], or null
  int t;                          // step index within the call (explicit arrays)
  unsigned long long seed;        // Philox key
  double sigma;                   // displacement width
};
hipError_t launch_multi_prep(const MultiArgs& a, const int2* items, int n_items, int grid, hipStream_t st);
// screened_lds > 0: QMC_REFINED members (the screened streams, with that much
// dynamic LDS)
hipError_t launch_multi_rows(const MultiArgs& a, int store, int nc, const int4* items, int n_items, int grid,
                             hipStream_t st, size_t screened_lds = 0);
hipError_t launch_multi_accept(const MultiArgs& a, int store, const int2* items, int n_items, int grid,
                               hipStream_t st);
hipError_t launch_multi_advance(long long* steps, int n, hipStream_t st);
hipError_t launch_philox_draws(unsigned long long seed, int member, int Wk, unsigned long long step, double sigma,
                               double* disp, double* unif, hipStream_t st);

hipError_t launch_forces(const SysDev& s, const WalkDev& w, const AdjWork& aw, const double* ga,
                         const double* gb, int per_walker, double* dR, double* dzeta, double* dlambda,
                         double* djas, double* dr, double* dj1_inh, double* dj3, double* djb_zeta,
                         double* dunpaired, double* dcon, double* dpf_uu, double* dpf_dd,
                         double* dunpaired_dn, hipStream_t st);

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

// Angular factor P and its gradient for an unnormalised real solid harmonic.
__device__ __forceinline__ void angular(int kind, double x, double y, double z,
                                        double& P, double& Px, double& Py, double& Pz) {
  switch (kind) {
    case 0: P = 1.0;     Px = 0.0;      Py = 0.0;      Pz = 0.0;     break;
    case 1: P = x;       Px = 1.0;      Py = 0.0;      Pz = 0.0;     break;
    case 2: P = y;       Px = 0.0;      Py = 1.0;      Pz = 0.0;     break;
    case 3: P = z;       Px = 0.0;      Py = 0.0;      Pz = 1.0;     break;
    case 4: P = x * y;   Px = y;        Py = x;        Pz = 0.0;     break;
    case 5: P = y * z;   Px = 0.0;      Py = z;        Pz = y;       break;
    case 6: P = z * x;   Px = z;        Py = 0.0;      Pz = x;       break;
    case 7: P = x * x - y * y;  Px = 2.0 * x;  Py = -2.0 * y;  Pz = 0.0;  break;
    default: P = 2.0 * z * z - x * x - y * y;  Px = -2.0 * x;  Py = -2.0 * y;  Pz = 4.0 * z;  break;
  }
}

__device__ __forceinline__ int kind_l(int kind) { return kind == 0 ? 0 : (kind < 4 ? 1 : 2); }

// Radial factors (eq. gaussian: e^{-zeta r^2}; eq. slater: e^{-zeta r}).  The
// basis function is psi = P(d) e(r), P an unnormalised real solid harmonic of
// degree l (harmonic and homogeneous), d the displacement from the centre.
// With h = e(r) and its radial derivatives, every derivative the path needs
// is P, grad P, Hess P and these coefficients (q = r^2):
//   grad psi   = e (grad P + h1 P d)                      h1 = h'/(r h)
//   Hess psi   = e (Hess P + h1 (d grad P^T + grad P d^T) + P (h2 d d^T + h1 I))
//                                                         h2 = (h''/r^2 - h'/r^3)/h
//   lap psi    = cl psi                                   cl = (h'' + 2(l+1) h'/r)/h
//   grad lap   = cl grad psi + gl psi d                   gl = cl'/r
//   dpsi/dzeta = -zp psi,  d grad psi/dzeta = -(zp grad psi + zq psi d),
//   d lap psi/dzeta = (dcl - zp cl) psi                   zp = r^2 or r, zq = 2 or 1/r, dcl = dcl/dzeta
// Gaussian: h1 = -2 zeta, h2 = 4 zeta^2, cl = 4 zeta^2 q - (4l+6) zeta, gl = 8 zeta^2.
// Slater:   h1 = -zeta/r, h2 = zeta^2/r^2 + zeta/r^3, cl = zeta^2 - 2 zeta (l+1)/r,
//           gl = 2 zeta (l+1)/r^3.
constexpr int kSlaterBit = 16;
__device__ __forceinline__ int kind_ang(int kind) { return kind & (kSlaterBit - 1); }

__device__ __forceinline__ double radial_e(int kind, double zt, double q) {
  return (kind & kSlaterBit) ? exp(-zt * sqrt(q)) : exp(-zt * q);
}

struct Radial { double e, h1, h2, cl, gl, zp, zq, dcl; };

__device__ __forceinline__ Radial radial_all(int kind, double zt, double q) {
  const double l = (double)kind_l(kind_ang(kind));
  Radial o;
  if (kind & kSlaterBit) {
    const double r = sqrt(q), ir = 1.0 / r;
    o.e = exp(-zt * r);
    o.h1 = -zt * ir;
    o.h2 = zt * zt * ir * ir + zt * ir * ir * ir;
    o.cl = zt * zt - 2.0 * zt * (l + 1.0) * ir;
    o.gl = 2.0 * zt * (l + 1.0) * ir * ir * ir;
    o.zp = r;
    o.zq = ir;
    o.dcl = 2.0 * zt - 2.0 * (l + 1.0) * ir;
  } else {
    const double lq = 4.0 * l + 6.0;
    o.e = exp(-zt * q);
    o.h1 = -2.0 * zt;
    o.h2 = 4.0 * zt * zt;
    o.cl = 4.0 * zt * zt * q - lq * zt;
    o.gl = 8.0 * zt * zt;
    o.zp = q;
    o.zq = 2.0;
    o.dcl = 8.0 * zt * q - lq;
  }
  return o;
}

__device__ __forceinline__ double angular_value(int kind, double x, double y, double z) {
  switch (kind) {
    case 0: return 1.0;
    case 1: return x;
    case 2: return y;
    case 3: return z;
    case 4: return x * y;
    case 5: return y * z;
    case 6: return z * x;
    case 7: return x * x - y * y;
    default: return 2.0 * z * z - x * x - y * y;
  }
}

// Function mu of a basis table (packed centre + zeta, kind) at point
// (px,py,pz): value only.  One packed record per function (one round trip).
// The value from the function's record f and kind k (already loaded).
__device__ __forceinline__ double basis_value_rec(const double4& f, int k, double px, double py, double pz) {
  const double x = px - f.x, y = py - f.y, z = pz - f.z;
  const double r2 = x * x + y * y + z * z;
  return angular_value(kind_ang(k), x, y, z) * radial_e(k, f.w, r2);
}

__device__ __forceinline__ double basis_value_tab(const double4* __restrict__ bfn, const int* __restrict__ kinds,
                                                  int mu, double px, double py, double pz) {
  return basis_value_rec(bfn[mu], kinds[mu], px, py, pz);
}

__device__ __forceinline__ double basis_value(const SysDev& s, int mu, double px, double py, double pz) {
  return basis_value_tab(s.bfn, s.kind, mu, px, py, pz);
}

// Value, gradient and Laplacian (see Radial).
__device__ __forceinline__ void basis_vgl_tab(const double4* __restrict__ bfn, const int* __restrict__ kinds, int mu,
                                              double px, double py, double pz, double& v, double& gx, double& gy,
                                              double& gz, double& lap) {
  const double4 f = bfn[mu];
  const double x = px - f.x, y = py - f.y, z = pz - f.z;
  const double r2 = x * x + y * y + z * z;
  const int k = kinds[mu];
  double P, Px, Py, Pz;
  angular(kind_ang(k), x, y, z, P, Px, Py, Pz);
  const Radial rd = radial_all(k, f.w, r2);
  const double t = rd.h1 * P;
  v = P * rd.e;
  gx = (Px + t * x) * rd.e;
  gy = (Py + t * y) * rd.e;
  gz = (Pz + t * z) * rd.e;
  lap = rd.cl * v;
}

__device__ __forceinline__ void basis_vgl(const SysDev& s, int mu, double px, double py, double pz,
                                          double& v, double& gx, double& gy, double& gz, double& lap) {
  basis_vgl_tab(s.bfn, s.kind, mu, px, py, pz, v, gx, gy, gz, lap);
}

// sum_c C[mu][c] y[c] over the orbitals that contain primitive mu: the
// coefficient of psi_mu in sum_c y_c phi_c (contracted orbitals only).
__device__ __forceinline__ double prim_weight(const SysDev& s, int mu, const double* __restrict__ y) {
  double t = 0.0;
  for (int k = s.pri_ptr[mu]; k < s.pri_ptr[mu + 1]; ++k) t += s.pri_coef[k] * y[s.pri_idx[k]];
  return t;
}

// One-body term f(r) = -(2Z)^{3/4} u((2Z)^{1/4} r) and its radial derivatives.
__device__ __forceinline__ void j1_radial(int form, double Z, double b, double r,
                                          double& f, double& f1, double& f2) {
  const double q = sqrt(sqrt(2.0 * Z));     // (2Z)^{1/4}
  const double s = q * r;
  double u, u1, u2;
  if (form == 1) {
    const double e = exp(-b * s);
    u = -expm1(-b * s) / (2.0 * b);
    u1 = 0.5 * e;
    u2 = -0.5 * b * e;
  } else {
    const double den = 1.0 / (1.0 + b * s);
    u = 0.5 * s * den;
    u1 = 0.5 * den * den;
    u2 = -b * den * den * den;
  }
  const double q3 = q * q * q;
  f = -q3 * u;
  f1 = -q3 * q * u1;
  f2 = -q3 * q * q * u2;
}

// Two-body term v(r) and its radial derivatives; same = parallel spins.
// form 1: v = c r/(1+b r); form 2: v = c t + a1 t^2 + a2 t^3 + a3 t^4, t = r/(1+b r).
__device__ __forceinline__ void j2_radial(int form, const double* p, bool same, double r,
                                          double& v, double& v1, double& v2) {
  const double c = same ? 0.25 : 0.5;
  double b, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  // constant indices only: p may point into a kernel argument, which a
  // run-time index would copy to scratch memory
  if (form == 1) {
    b = same ? p[0] : p[1];
  } else {
    b = same ? p[0] : p[4];
    a1 = same ? p[1] : p[5];
    a2 = same ? p[2] : p[6];
    a3 = same ? p[3] : p[7];
  }
  const double den = 1.0 / (1.0 + b * r);
  const double t = r * den;
  const double dt = den * den;
  const double d2t = -2.0 * b * den * den * den;
  // g(t) = c t + a1 t^2 + a2 t^3 + a3 t^4
  const double g = t * (c + t * (a1 + t * (a2 + t * a3)));
  const double g1 = c + t * (2.0 * a1 + t * (3.0 * a2 + t * 4.0 * a3));
  const double g2 = 2.0 * a1 + t * (6.0 * a2 + t * 12.0 * a3);
  v = g;
  v1 = g1 * dt;
  v2 = g2 * dt * dt + g1 * d2t;
}

// ---------------------------------------------------------------------------
// wave-level reductions (64 lanes)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------------------
// launchers (all asynchronous on `st`)
// ---------------------------------------------------------------------------
hipError_t launch_basis_values(const SysDev& s, const WalkDev& w, hipStream_t st, void* lo = nullptr,
                               bool lo_bf16 = false, int* ephi = nullptr);
hipError_t launch_downcast(const double* src, void* dst, bool to_bf16, long n, hipStream_t st);
// dirty (FP64 and FP32 products, bit h for half h): only the rows whose
// electron has moved since the row was last built (launch_moved_rows)
hipError_t launch_P_build(const SysDev& s, const WalkDev& w, int halves, hipStream_t st,
                          void* lo = nullptr, bool lo_bf16 = false, int dirty = 0);
// The rows of P half h (0: up, 1: down) whose electron has moved since the row
// was last built, in increasing order (*ridx, count at *rcnt on the device),
// recording the positions; moved_only = false: every row (positions only, no
// list).  Nothing to do (and no list) when the walker set keeps no positions.
hipError_t launch_moved_rows(const SysDev& s, const WalkDev& w, int h, bool moved_only, int** ridx, int** rcnt,
                             hipStream_t st);
hipError_t launch_W_build(const SysDev& s, const WalkDev& w, hipStream_t st);
// int8 digit tiles of FP64 rows and the error-free products built from them
long oz_plane_bytes(long rows, int Kp);
long oz_phi_bytes(const SysDev& s, long Wk);
hipError_t launch_slice_tiles(const double* X, long rows, int K, int Kp, int grp, long gs, long ld, int S,
                              int8_t* out, long plane, int* expo, hipStream_t st, bool have_expo = false,
                              const int* ridx = nullptr, const int* rcnt = nullptr, int* expo_c = nullptr);
hipError_t launch_oz_lambda(const SysDev& s, hipStream_t st);
// QMC_REFINED Pfaffian: digits of the rows of the four K^T, and the B rows
// (P = B^u, Bd = B^d) of the evaluation from the walkers' FP64 basis rows
hipError_t launch_oz_pf_K(const SysDev& s, hipStream_t st);
hipError_t launch_pf_B_build_oz(const SysDev& s, const WalkDev& w, hipStream_t st);
// dirty (QMC_REFINED, bit h for half h): build only the rows whose electron
// has moved since its row was last built (the other rows of P, PT stand); every
// half built records its positions for the next such build.
hipError_t launch_P_build_oz(const SysDev& s, const WalkDev& w, int halves, const double* phi64, double* P64,
                             void* lo, bool lo_bf16, hipStream_t st, bool have_expo = false, double* PT = nullptr,
                             int dirty = 0);
// screened proposals: column maxima of the P halves, and the streaming kernel
hipError_t launch_screen_colmax(const SysDev& s, const WalkDev& w, int halves, hipStream_t st);
// dynamic LDS of the blocked screened stream for a proposal of e (0: the plain one runs)
size_t screened_stream_lds(const SysDev& s, const WalkDev& w, int e);
// the unpaired orbitals' entries of every walker's transposed rows
hipError_t launch_pt_unpaired(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_export_kept(const WalkDev& w, double* dst, hipStream_t st);
hipError_t launch_propose_screened(const SysDev& s, const WalkDev& w, int e, double* ratio, bool finalize,
                                   hipStream_t st, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
hipError_t launch_Y_build(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_lu_inverse(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_lam_mask(const SysDev& s, hipStream_t st);
hipError_t launch_rowdots(const SysDev& s, const WalkDev& w, hipStream_t st);
// Gauss-Jordan inverse and log|det| of Wk dense n x n matrices (n <= kLuRowMax)
hipError_t launch_gj_inverse_n(int Wk, int n, const double* W, double* A, double* logdet, double* detsign,
                               int* singular, hipStream_t st);
// Pfaffian pairing: B rows, G~, its Pfaffian (log|Pf|, sign into logdet / detsign)
// and inverse, cofactor vectors; proposal and accept of a single-electron move
hipError_t launch_pf_B_build(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_pf_G_build(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_pf_factor(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_pf_Y_products(const SysDev& s, const WalkDev& w, const double* X, double* out, hipStream_t st);
hipError_t launch_pf_Y_build(const SysDev& s, const WalkDev& w, hipStream_t st);
hipError_t launch_pf_propose(const SysDev& s, const WalkDev& w, int e, const double* r_new, const double* disp,
                             double* ratio, double* drift, hipStream_t st);
hipError_t launch_pf_logderiv(const SysDev& s, const WalkDev& w, double* d_uu, double* d_dd, double* d_ud,
                              double* d_uup, double* d_udn, hipStream_t st);
hipError_t launch_pf_set(const SysDev& s, const double* lam, const double* uu, const double* dd, const double* upu,
                         const double* upd, hipStream_t st);
hipError_t launch_pf_accept(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc, const double* unif,
                            int32_t* accept_count, hipStream_t st);

// Jastrow-basis terms of an evaluation (LJ > 0): chi, X -> G, h, per-electron terms
hipError_t launch_jastrow3_eval(const SysDev& s, const WalkDev& w, hipStream_t st);
// d log Psi / d (one-body inhomogeneous, three/four-body coefficients), per walker
hipError_t launch_jastrow3_logderiv(const SysDev& s, const WalkDev& w, double* dm, double* dM, hipStream_t st);
// Estimators (space warp, reweighting factor, stochastic reconfiguration)
hipError_t launch_swct(const SysDev& s, int Wk, const double* r, const double* dR, const double* dr, int jac,
                       double* out, hipStream_t st);
hipError_t launch_reweight(const SysDev& s, const WalkDev& w, double theta, double eps, double* R, double* weight,
                           hipStream_t st);
size_t sr_workspace_doubles(int M, long P);
hipError_t launch_sr_step(int M, long P, const double* O, const double* el, const double* wts, double eps,
                          int max_iter, double tol, double* delta, double* force, double* resid, double* work,
                          hipStream_t st);
hipError_t launch_jastrow_assemble(const SysDev& s, const WalkDev& w, double* logabs, double* sign,
                                   double* drift, double* e_kin, double* e_loc, int32_t* status,
                                   hipStream_t st);
int propose_splits(const SysDev& s);
// Proposal in two launches: per-walker psi(r') and Jastrow change, then the
// streaming row kernel (and, when finalize, the ratio sum).
hipError_t launch_propose_prep(const SysDev& s, const WalkDev& w, int e, const double* r_new,
                               const double* disp, bool drift, hipStream_t st);
hipError_t launch_propose_rows(const SysDev& s, const WalkDev& w, int e, double* ratio,
                               double* drift_new, bool finalize, hipStream_t st, hipEvent_t ev_start = nullptr,
                               hipEvent_t ev_stop = nullptr);
hipError_t launch_metropolis_accept(const SysDev& s, const WalkDev& w, int e, const double* unif,
                                    int32_t* accept_count, hipStream_t st);
// Metropolis accept of e fused with the set-up of the next proposal (electron
// e2, displacements disp2 [Wk][3]); needs s.Lp <= kFuseMaxLp.  since: the
// attempted moves since the last refresh (a bound on the buffered updates).
hipError_t launch_metropolis_accept_prep(const SysDev& s, const WalkDev& w, int e, const double* unif,
                                         int32_t* accept_count, int e2, const double* disp2, int since,
                                         hipStream_t st);
hipError_t launch_accept(const SysDev& s, const WalkDev& w, int e, const uint8_t* acc,
                         hipStream_t st);
// Persistent sweep of k >= 2 moves e0, e0 + 1, ... (mod N): the k proposals and
// the k - 1 accepts between them fused with the next set-up, in one launch
// (one workgroup per walker); the set-up of e0 must have run, and the last
// proposal is left for a plain accept.  No refresh, change of spin or P
// rebuild may fall inside.  since0: the attempts since the last refresh at the
// first accept.  sweep_segment_ok: whether the kernel is built for the system
// and the spin of e0 (hipErrorNotSupported from the launch otherwise).
bool sweep_segment_ok(const SysDev& s, const WalkDev& w, int e0);
hipError_t launch_sweep_segment(const SysDev& s, const WalkDev& w, int e0, int k, const double* disp,
                                const double* unif, int32_t* accept_count, int since0, hipStream_t st,
                                hipEvent_t ev_start, hipEvent_t ev_stop);
hipError_t launch_refresh_finish(const SysDev& s, const WalkDev& w, int32_t* status, hipStream_t st);
// max |W X - I| per walker (P = W X given) and status 3 where it exceeds tol
hipError_t launch_refresh_residual(const double* Pm, int n, int Wk, double tol, double* res, int32_t* status,
                                   hipStream_t st);
// scratch: [Wk][2][kb][n]
hipError_t launch_materialize_inverse(const SysDev& s, const WalkDev& w, bool down, double* scratch, double* dst,
                                      hipStream_t st);
// moves that fit the delayed-update buffer between refreshes
inline int wb_cap(const SysDev& s) { return s.refresh_every < kWbMax ? s.refresh_every : kWbMax; }
hipError_t launch_export_phi(const SysDev& s, const WalkDev& w, double* dst, hipStream_t st);
hipError_t launch_set_lambda(const SysDev& s, const double* lam, hipStream_t st);
hipError_t launch_pack_basis(const SysDev& s, hipStream_t st);
hipError_t launch_set_jastrow_basis(const SysDev& s, const double* j1_inh, const double* j3, const double* jz,
                                    hipStream_t st);

// FP64 MFMA GEMM, exposed for the launchers above.
struct GemmArgs {
  int M, N, K;
  const void* A; long lda; long a_bs; int a_grp; long a_gs;
  const void* B; long ldb; long b_bs;
  void* C; long ldc; long c_bs; int c_grp; long c_gs;
  int batch;
  int accumulate;   // 1: C += op(A) op(B); 0: C = op(A) op(B)
  // optional second output written beside C (same layout, no accumulation):
  // C2 != null stores each result also as FP32 (c2_bf16 = 0) or BF16 (1)
  void* C2;
  int c2_bf16;
  // optional nonzero flags of B's [kLamTileK x kLamTileN] tiles ([K/16][kmask_ld]);
  // honoured by the 64-column-tile kernels, which skip zero tiles
  const uint8_t* kmask;
  int kmask_ld;
  // optional row list (row-major A, not TA): output row m is row ridx[m] of A
  // and of C, for m < *rcnt (the grid is sized for M rows)
  const int* ridx;
  const int* rcnt;
};

// Plain (ungathered) argument block for an M x N x K product.
GemmArgs gemm_args(int M, int N, int K);
// FP64 products on MFMA; big = 64x64 tiles (else 32x32).
hipError_t gemm_f64(const GemmArgs& g, bool ta, bool tb, bool big, hipStream_t st);

}  // namespace qmc
