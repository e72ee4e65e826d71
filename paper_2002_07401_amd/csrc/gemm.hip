// Dense products of the geminal construction on the gfx950 matrix cores.
//
//   P_up = Phi_up Lambda        P_dn = Phi_dn Lambda^T          (agp_expansion)
//   W    = P_up Phi_dn^T        (the geminal matrix, eq:wfAGPs)
//   Yt_up = W^{-T} P_dn ... see launch_Y_build
//
// One templated kernel: C = op(A) op(B), row-major operands, 256 threads as a
// 2x2 grid of waves, each wave owning (BM/2) x (BN/2) of the tile as 16x16
// MFMA blocks.  K is staged through LDS in steps of 16.  Rows of A and C may be
// "gathered": row m lives at (m / grp) * gs + (m % grp) * ld, which lets the
// up (or down) rows of every walker form one tall matrix that multiplies the
// shared Lambda.
#include "internal.h"

namespace qmc {

typedef double dx4 __attribute__((ext_vector_type(4)));
typedef float fx4 __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
// Output row of accumulator register r in lane `lane` (column is lane % 16):
// the FP64 instruction interleaves rows across registers, the FP32 one blocks them.
template <> struct Mfma<double> {
  typedef dx4 acc_t;
  static __device__ __forceinline__ acc_t run(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <> struct Mfma<float> {
  typedef fx4 acc_t;
  static __device__ __forceinline__ acc_t run(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

// Logical block of a hardware block id.  Workgroups are dealt to the 8 XCDs in
// turn; regrouping the ids gives each XCD one contiguous range of logical
// blocks, so blocks that share operand tiles (the N tiles of one A tile, the
// tiles of one walker's batched product) share that XCD's L2.  A bijection on
// [0, total) whatever the dispatch order.
__device__ __forceinline__ long xcd_remap(long id, long total) {
  const long per = total / 8, rem = total % 8;
  const long x = id % 8, slot = id / 8;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + slot;
}

// TA: A stored [K][M] (op(A) = A^T); TB: B stored [N][K] (op(B) = B^T).
// SA, SB: storage types of A and B (converted exactly to TI on load);
// TI: MFMA operand type; TO: output type.  K advances in steps of BK; the
// next step's operands are loaded into registers while the current step's
// MFMAs run.  Products accumulate in k order (the result does not depend on
// BK or on skipped all-zero tiles).
template <int BM, int BN, bool TA, bool TB, typename SA, typename SB, typename TI, typename TO, int BK = 32>
__global__ void __launch_bounds__(256) gemm_kernel(GemmArgs g, int gx, int gy) {
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int FM = WM / 16, FN = WN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(FM >= 1 && FN >= 1, "tile too small");
  __shared__ TI As[BK][BM + 1];
  __shared__ TI Bs[BK][BN + 1];
  typedef typename Mfma<TI>::acc_t acc_t;

  // with a row list, only its tiles are dealt out (the grid is sized for M
  // rows; the workgroups past the list's tiles leave at once)
  const int Mr = g.ridx ? min(g.M, *g.rcnt) : g.M;
  const int gyr = g.ridx ? (Mr + BM - 1) / BM : gy;
  const long nt = g.ridx ? (long)gx * gyr * g.batch : (long)gridDim.x;
  if ((long)blockIdx.x >= nt) return;   // (uniform, before any barrier)
  const long L = xcd_remap(blockIdx.x, nt);
  const int bx = (int)(L % gx);
  const long rest = L / gx;
  const int by = (int)(rest % gyr);
  const long bz = rest / gyr;
  const SA* __restrict__ A = (const SA*)g.A + bz * g.a_bs;
  const SB* __restrict__ B = (const SB*)g.B + bz * g.b_bs;
  TO* __restrict__ C = (TO*)g.C + bz * g.c_bs;
  float* __restrict__ C2f = (g.C2 && !g.c2_bf16) ? (float*)g.C2 + bz * g.c_bs : nullptr;
  bf16s* __restrict__ C2h = (g.C2 && g.c2_bf16) ? (bf16s*)g.C2 + bz * g.c_bs : nullptr;
  const int m0 = by * BM, n0 = bx * BN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;

  // staging coordinates of this thread's EA + EB elements, fixed over K
  long aoff[EA], boff[EB];
  int akk[EA], amm[EA], bkk[EB], bnn[EB];
  bool aok[EA], bok[EB];
#pragma unroll
  for (int q = 0; q < EA; ++q) {
    const int idx = tid + 256 * q;
    int mm, kk;
    if (TA) { kk = idx / BM; mm = idx % BM; } else { mm = idx / BK; kk = idx % BK; }
    const int gm = m0 + mm;
    akk[q] = kk; amm[q] = mm; aok[q] = gm < Mr;
    const int gr = (g.ridx && gm < Mr) ? g.ridx[gm] : gm;   // the row of A
    aoff[q] = TA ? (long)kk * g.lda + gm
                 : (long)(gr / g.a_grp) * g.a_gs + (long)(gr % g.a_grp) * g.lda + kk;
  }
#pragma unroll
  for (int q = 0; q < EB; ++q) {
    const int idx = tid + 256 * q;
    int nn, kk;
    if (TB) { nn = idx / BK; kk = idx % BK; } else { kk = idx / BN; nn = idx % BN; }
    const int gn = n0 + nn;
    bkk[q] = kk; bnn[q] = nn; bok[q] = gn < g.N;
    boff[q] = TB ? (long)gn * g.ldb + kk : (long)kk * g.ldb + gn;
  }
  TI ra[EA], rb[EB];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < EA; ++q)
      ra[q] = (aok[q] && k0 + akk[q] < g.K) ? (TI)A[aoff[q] + (TA ? (long)k0 * g.lda : (long)k0)] : (TI)0;
#pragma unroll
    for (int q = 0; q < EB; ++q)
      rb[q] = (bok[q] && k0 + bkk[q] < g.K) ? (TI)B[boff[q] + (TB ? (long)k0 : (long)k0 * g.ldb)] : (TI)0;
  };
  // first K step at or after k whose B tile is not entirely zero (uniform per block)
  auto next_k = [&](int k) -> int {
    if constexpr (kLamTileN % BN == 0 && BK % kLamTileK == 0 && !TB) {
      if (g.kmask) {
        const int nt = n0 / kLamTileN;
        while (k < g.K) {
          const int t = k / kLamTileK;
          bool nz = false;
#pragma unroll
          for (int h = 0; h < BK / kLamTileK; ++h)
            nz |= (k + h * kLamTileK < g.K) && g.kmask[(long)(t + h) * g.kmask_ld + nt];
          if (nz) break;
          k += BK;
        }
      }
    }
    return k;
  };

  acc_t acc[FM][FN];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
      for (int r = 0; r < 4; ++r) acc[i][j][r] = 0;

  int k0 = next_k(0);
  if (k0 < g.K) load(k0);
  while (k0 < g.K) {
#pragma unroll
    for (int q = 0; q < EA; ++q) As[akk[q]][amm[q]] = ra[q];
#pragma unroll
    for (int q = 0; q < EB; ++q) Bs[bkk[q]][bnn[q]] = rb[q];
    __syncthreads();
    const int k1 = next_k(k0 + BK);
    if (k1 < g.K) load(k1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      TI a[FM], b[FN];
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[kk + (lane >> 4)][wm * WM + i * 16 + (lane & 15)];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[kk + (lane >> 4)][wn * WN + j * 16 + (lane & 15)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = Mfma<TI>::run(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
    k0 = k1;
  }
  // 16x16 block layout: lane holds column lane%16 and the rows given by
  // Mfma::row.  The output rows' offsets (their row-list entries loaded, the
  // row index split into group and row) are formed for all of this lane's
  // rows before any store: a load issued after a store of C would wait for it
  // (the two may alias as far as the compiler knows).
  long roff[FM][4];
  bool rok[FM][4];
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + wm * WM + i * 16 + Mfma<TI>::row(lane, r);
      rok[i][r] = gm < Mr;
      const int gr = rok[i][r] ? (g.ridx ? g.ridx[gm] : gm) : 0;   // the row of C
      const int q = gr / g.c_grp;
      roff[i][r] = (long)q * g.c_gs + (long)(gr - q * g.c_grp) * g.ldc;
    }
#pragma unroll
  for (int i = 0; i < FM; ++i)
#pragma unroll
    for (int j = 0; j < FN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gn = n0 + wn * WN + j * 16 + (lane & 15);
        if (rok[i][r] && gn < g.N) {
          const long off = roff[i][r] + gn;
          TO* cp = C + off;
          if constexpr (sizeof(TO) == 2) {
            *cp = (TO)acc[i][j][r];   // BF16 output: never accumulated
          } else {
            const TO v = g.accumulate ? (TO)(*cp + (TO)acc[i][j][r]) : (TO)acc[i][j][r];
            *cp = v;
            if (C2f) C2f[off] = (float)v;
            if (C2h) C2h[off] = bf16s(v);
          }
        }
      }
}

template <int BM, int BN, bool TA, bool TB, typename SA, typename SB, typename TI, typename TO, int BK = 32>
static hipError_t run_gemm(const GemmArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  const int gx = (g.N + BN - 1) / BN, gy = (g.M + BM - 1) / BM;
  const long total = (long)gx * gy * g.batch;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((gemm_kernel<BM, BN, TA, TB, SA, SB, TI, TO, BK>), dim3((unsigned)total), dim3(256), 0, st, g,
                     gx, gy);
  return hipGetLastError();
}

GemmArgs gemm_args(int M, int N, int K) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K;
  g.a_grp = 1 << 30; g.a_gs = 0;
  g.c_grp = 1 << 30; g.c_gs = 0;
  g.batch = 1;
  return g;
}

static GemmArgs plain(int M, int N, int K) { return gemm_args(M, N, K); }

hipError_t gemm_f64(const GemmArgs& g, bool ta, bool tb, bool big, hipStream_t st) {
#define QMC_G(BM, BN, TA_, TB_) run_gemm<BM, BN, TA_, TB_, double, double, double, double, 16>(g, st)
  if (big) {
    if (ta) return tb ? QMC_G(64, 64, true, true) : QMC_G(64, 64, true, false);
    return tb ? QMC_G(64, 64, false, true) : QMC_G(64, 64, false, false);
  }
  if (ta) return tb ? QMC_G(32, 32, true, true) : QMC_G(32, 32, true, false);
  return tb ? QMC_G(32, 32, false, true) : QMC_G(32, 32, false, false);
#undef QMC_G
}

// Tile shapes from sweeps on MI355X (1024 walkers x 80 rows, L = 608, all
// rows or a list of 60 per walker): FP64 64 x 64 with K steps of 16 (61-63 %
// of the FP64 matrix peak, against 51-57 % for 64 x 32, 57-58 % for 128 x 32
// and 32 x 64, 49-51 % for 128 x 128); FP32 / BF16 rows 64 x 64 with K steps
// of 32.
template <typename T, typename TL>
static hipError_t P_gemm(const GemmArgs& g, hipStream_t st) {
  if constexpr (sizeof(TL) == 8) return run_gemm<64, 64, false, false, T, TL, TL, T, 16>(g, st);
  else return run_gemm<64, 64, false, false, T, TL, TL, T, 32>(g, st);
}

// T: storage of Phi and P; TL: storage of Lambda and the MFMA operand type
// (BF16 rows multiply the FP32 Lambda with FP32 accumulation).
// lo (FP64 products only): also store P as FP32 / BF16 there (the moves' copy).
template <typename T, typename TL = T>
static hipError_t P_build_t(const SysDev& s, const WalkDev& w, int halves, hipStream_t st,
                            const TL* lam, const TL* lamT, void* lo = nullptr, bool lo_bf16 = false, int dirty = 0) {
  const long rowst = (long)s.N * s.Lp;
  const T* phi = (const T*)w.phi;
  T* P = (T*)w.P;
  hipError_t e = hipSuccess;
  const int mask_ld = (s.Lp + kLamTileN - 1) / kLamTileN;
  int* ridx[2] = {nullptr, nullptr};
  int* rcnt[2] = {nullptr, nullptr};
  for (int h = 0; h < 2; ++h)
    if ((halves >> h) & 1) {
      e = launch_moved_rows(s, w, h, (dirty >> h) & 1, &ridx[h], &rcnt[h], st);
      if (e != hipSuccess) return e;
    }
  if (halves & 1) {   // P_up = Phi_up Lambda  (rows 0..nu-1 of every walker)
    GemmArgs g = plain(w.Wk * s.nu, s.Lp, s.Lp);
    g.ridx = ridx[0]; g.rcnt = rcnt[0];
    g.A = phi; g.lda = s.Lp; g.a_grp = s.nu; g.a_gs = rowst;
    g.B = lam; g.ldb = s.Lp;
    g.kmask = s.lam_mask; g.kmask_ld = mask_ld;
    g.C = P; g.ldc = s.Lp; g.c_grp = s.nu; g.c_gs = rowst;
    g.C2 = lo; g.c2_bf16 = lo_bf16 ? 1 : 0;
    e = P_gemm<T, TL>(g, st);
    if (e != hipSuccess) return e;
  }
  if (halves & 2) {   // P_dn = Phi_dn Lambda^T (rows nu..N-1)
    GemmArgs g = plain(w.Wk * s.nd, s.Lp, s.Lp);
    g.ridx = ridx[1]; g.rcnt = rcnt[1];
    g.A = phi + (long)s.nu * s.Lp; g.lda = s.Lp; g.a_grp = s.nd; g.a_gs = rowst;
    g.B = lamT; g.ldb = s.Lp;
    g.kmask = s.lamT_mask; g.kmask_ld = mask_ld;
    g.C = P + (long)s.nu * s.Lp; g.ldc = s.Lp; g.c_grp = s.nd; g.c_gs = rowst;
    if (lo) {
      g.C2 = lo_bf16 ? (void*)((bf16s*)lo + (long)s.nu * s.Lp) : (void*)((float*)lo + (long)s.nu * s.Lp);
      g.c2_bf16 = lo_bf16 ? 1 : 0;
    }
    e = P_gemm<T, TL>(g, st);
  }
  return e;
}

// ---------------------------------------------------------------------------
// BF16 rows (QMC_MIXED_BF16): P = Phi Lambda on the BF16 matrix cores.  Phi is
// stored in BF16 (exact operand); Lambda enters as an unevaluated pair
// hi + lo of BF16 values (lo = bf16(Lambda - hi), Lambda to about 16
// significant bits), two v_mfma_f32_16x16x32_bf16 per block and K step, FP32
// accumulation, and the result rounded once to the BF16 rows.  The operand
// split keeps Lambda's share of the error far below the rows' own BF16
// rounding.  256 threads as 2 x 2 waves over a 64 x 64 tile, 32 x 32 per wave
// as 2 x 2 blocks of 16 x 16; K steps of 32 staged through LDS (rows of 32
// BF16 values, padded to 40), the next step loaded into registers while the
// current one multiplies.  Operand layout of the instruction: lane l holds row
// (column) l % 16 of A (B), k = 8 (l / 16) .. 8 (l / 16) + 7; accumulator
// register r of lane l is row 4 (l / 16) + r, column l % 16.
// ---------------------------------------------------------------------------
typedef __bf16 bfx8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

struct PBf16Args {
  const uint16_t* A; long lda; int a_grp; long a_gs;   // rows m: (m / a_grp) a_gs + (m % a_grp) lda
  const uint16_t* Bh; const uint16_t* Bl; long ldb;    // [N][K] hi and lo
  uint16_t* C; long ldc; int c_grp; long c_gs;
  int M, N, K;
};

__global__ void __launch_bounds__(256) p_bf16_kernel(PBf16Args g, int gx) {
  constexpr int BK = 32, LD = 40;
  __shared__ __align__(16) uint16_t As[64][LD];
  __shared__ __align__(16) uint16_t Bh[64][LD];
  __shared__ __align__(16) uint16_t Bl[64][LD];
  const long L = xcd_remap(blockIdx.x, (long)gridDim.x);
  const int bx = (int)(L % gx), by = (int)(L / gx);
  const int m0 = 64 * by, n0 = 64 * bx;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // staging: thread t moves 8 values (16 bytes) of row / column t / 4, k = 8 (t % 4)
  const int sr = tid >> 2, sk = 8 * (tid & 3);
  const int gm = m0 + sr, gn = n0 + sr;
  const bool aok = gm < g.M, bok = gn < g.N;
  const uint16_t* ap = g.A + (aok ? (long)(gm / g.a_grp) * g.a_gs + (long)(gm % g.a_grp) * g.lda : 0) + sk;
  const uint16_t* bhp = g.Bh + (bok ? (long)gn * g.ldb : 0) + sk;
  const uint16_t* blp = g.Bl + (bok ? (long)gn * g.ldb : 0) + sk;
  const u16x8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
  u16x8 ra, rh, rl;
  auto load = [&](int k0) {
    ra = aok ? *(const u16x8*)(ap + k0) : zero;
    rh = bok ? *(const u16x8*)(bhp + k0) : zero;
    rl = bok ? *(const u16x8*)(blp + k0) : zero;
  };
  fx4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = fx4{0.f, 0.f, 0.f, 0.f};
  load(0);
  const int fr = lane & 15, fk = 8 * (lane >> 4);
  for (int k0 = 0; k0 < g.K; k0 += BK) {
    __syncthreads();   // the previous step's reads are done
    *(u16x8*)&As[sr][sk] = ra;
    *(u16x8*)&Bh[sr][sk] = rh;
    *(u16x8*)&Bl[sr][sk] = rl;
    __syncthreads();
    if (k0 + BK < g.K) load(k0 + BK);
    bfx8 a[2], bh[2], bl[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      a[i] = __builtin_bit_cast(bfx8, *(const u16x8*)&As[32 * wm + 16 * i + fr][fk]);
      bh[i] = __builtin_bit_cast(bfx8, *(const u16x8*)&Bh[32 * wn + 16 * i + fr][fk]);
      bl[i] = __builtin_bit_cast(bfx8, *(const u16x8*)&Bl[32 * wn + 16 * i + fr][fk]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bh[j], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], bl[j], acc[i][j], 0, 0, 0);
      }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + 32 * wm + 16 * i + 4 * (lane >> 4) + r;
        const int n = n0 + 32 * wn + 16 * j + fr;
        if (m < g.M && n < g.N)
          g.C[(long)(m / g.c_grp) * g.c_gs + (long)(m % g.c_grp) * g.ldc + n] = bf16s(acc[i][j][r]).x;
      }
}

static hipError_t P_build_bf16(const SysDev& s, const WalkDev& w, int halves, hipStream_t st) {
  if (!s.lamB || s.Lp % 32 != 0) return hipErrorInvalidValue;
  const long rowst = (long)s.N * s.Lp, pl = (long)s.Lp * s.Lp;
  const uint16_t* phi = (const uint16_t*)w.phi;
  uint16_t* P = (uint16_t*)w.P;
  for (int h = 0; h < 2; ++h) {
    if (!((halves >> h) & 1)) continue;
    const int rows = h == 0 ? s.nu : s.nd;
    if (rows == 0) continue;
    PBf16Args g;
    g.A = phi + (h == 0 ? 0 : (long)s.nu * s.Lp); g.lda = s.Lp; g.a_grp = rows; g.a_gs = rowst;
    g.Bh = s.lamB + 2 * h * pl; g.Bl = s.lamB + (2 * h + 1) * pl; g.ldb = s.Lp;
    g.C = P + (h == 0 ? 0 : (long)s.nu * s.Lp); g.ldc = s.Lp; g.c_grp = rows; g.c_gs = rowst;
    g.M = w.Wk * rows; g.N = s.Lp; g.K = s.Lp;
    const int gx = (g.N + 63) / 64, gy = (g.M + 63) / 64;
    hipLaunchKernelGGL(p_bf16_kernel, dim3((unsigned)((long)gx * gy)), dim3(256), 0, st, g, gx);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_P_build(const SysDev& s, const WalkDev& w, int halves, hipStream_t st, void* lo,
                          bool lo_bf16, int dirty) {
  if (s.bf16()) return dirty ? hipErrorInvalidValue : P_build_bf16(s, w, halves, st);
  if (s.f32()) return P_build_t<float>(s, w, halves, st, s.lam32, s.lamT32, nullptr, false, dirty);
  return P_build_t<double>(s, w, halves, st, s.lam, s.lamT, lo, lo_bf16, dirty);
}

// W[w] = P_up[w] Phi_dn[w]^T  ->  W[i][j] = sum_nu (Phi_up Lambda)[i][nu] psi_nu(r_j),
// and with unpaired orbitals (eq:wfAGPunpaired) the last nk columns
// W[i][n_dn + l] = psi(r_i) . U[:, l] = (Phi_up Uph^T)[i][l].  W is n_up x n_up.
// The geminal matrix of one walker per workgroup, W = P_up Phi_dn^T (n x n,
// K = Lp), for n = n_up = n_dn = 16 RB <= 80, Lp a multiple of 32 and no
// unpaired orbitals.  The batched product reads 16 n Lp bytes per walker for
// 2 n^2 Lp flops, about the FP64 matrix cores' ratio of flops to HBM bytes, so
// the kernel keeps both busy: K advances in chunks of 16 whose rows are read
// with 16-byte loads into registers while the previous chunk's MFMAs run from
// LDS, where both operands sit in fragment order (each K step's 64 lane values
// of a 16-row block contiguous).  Wave rb owns output rows 16 rb .. 16 rb + 15.
// Products accumulate in k order in steps of 4 with the generic kernel's
// instruction, so W is bitwise the same.
template <typename T, int RB>
__global__ void __launch_bounds__(64 * RB, RB == 5 ? 5 : 4) wgem_kernel(const T* __restrict__ Pg, const T* __restrict__ Fg,
                                                          double* __restrict__ Wg, int N, int Lp) {
  constexpr int n = 16 * RB, KC = 16, SC = KC / 4;   // K per chunk, K steps per chunk
  constexpr int HC = KC / 2, PQ = KC / 8;             // column pairs per row, pieces per thread and operand
  __shared__ double La[RB * SC * 64], Lb[RB * SC * 64];   // [row block][K step in chunk][lane]
  const long wk = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const T* Pa = Pg + wk * N * (long)Lp;             // P_up rows
  const T* Fb = Fg + (wk * N + n) * (long)Lp;       // Phi_dn rows
  // each thread copies PQ pieces of 16 bytes (2 columns) of each operand per
  // chunk: piece q is row tid / HC + (64 RB / HC) q, columns 2 (tid % HC) + {0, 1}
  // (a uniform base per piece and one lane offset)
  const int loff = (tid / HC) * Lp + 2 * (tid % HC);
  double2 ra[PQ], rb[PQ];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const long ub = (long)(64 * RB / HC * q) * Lp + k0;
      if constexpr (sizeof(T) == 8) {
        ra[q] = *(const double2*)((Pa + ub) + loff);
        rb[q] = *(const double2*)((Fb + ub) + loff);
      } else {
        const float2 x = *(const float2*)((Pa + ub) + loff);
        const float2 y = *(const float2*)((Fb + ub) + loff);
        ra[q] = double2{(double)x.x, (double)x.y};
        rb[q] = double2{(double)y.x, (double)y.y};
      }
    }
  };
  // fragment order: column k of the chunk goes to K step k / 4, lane (k % 4) 16 + row % 16
  auto store = [&]() {
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
      const int row = tid / HC + 64 * RB / HC * q, k = 2 * (tid % HC);
      const int o = ((row >> 4) * SC + (k >> 2)) * 64 + (k & 3) * 16 + (row & 15);
      La[o] = ra[q].x; La[o + 16] = ra[q].y;
      Lb[o] = rb[q].x; Lb[o + 16] = rb[q].y;
    }
  };
  dx4 acc[RB];
#pragma unroll
  for (int cb = 0; cb < RB; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[cb][r] = 0.0;
  load(0);
  for (int k0 = 0; k0 < Lp; k0 += KC) {
    store();
    __syncthreads();
    if (k0 + KC < Lp) load(k0 + KC);
#pragma unroll
    for (int st = 0; st < SC; ++st) {
      const double a = La[(wave * SC + st) * 64 + lane];
#pragma unroll
      for (int cb = 0; cb < RB; ++cb)
        acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Lb[(cb * SC + st) * 64 + lane], acc[cb], 0, 0, 0);
    }
    __syncthreads();
  }
  // 16 x 16 block layout: lane holds column lane % 16 and rows 4 r + lane / 16
  double* W = Wg + wk * (long)n * n;
#pragma unroll
  for (int cb = 0; cb < RB; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) W[(long)(wave * 16 + 4 * r + (lane >> 4)) * n + cb * 16 + (lane & 15)] = acc[cb][r];
}

template <typename T>
static hipError_t launch_wgem(const SysDev& s, const WalkDev& w, hipStream_t st) {
#define QMC_WG(R)                                                                                               \
  hipLaunchKernelGGL((wgem_kernel<T, R>), dim3((unsigned)w.Wk), dim3(64 * R), 0, st, (const T*)w.P, (const T*)w.phi, \
                     w.W, s.N, s.Lp)
  switch (s.nu / 16) {
    case 1: QMC_WG(1); break;
    case 2: QMC_WG(2); break;
    case 3: QMC_WG(3); break;
    case 4: QMC_WG(4); break;
    default: QMC_WG(5); break;
  }
#undef QMC_WG
  return hipGetLastError();
}

template <typename T>
static hipError_t W_build_t(const SysDev& s, const WalkDev& w, const T* Uph, hipStream_t st) {
  const long rowst = (long)s.N * s.Lp, n = s.nu;
  if (s.nk == 0 && s.nu == s.nd && s.nu % 16 == 0 && s.nu >= 16 && s.nu <= 80 && s.Lp % 32 == 0)
    return launch_wgem<T>(s, w, st);
  GemmArgs g = plain(s.nu, s.nd, s.Lp);
  g.A = (const T*)w.P; g.lda = s.Lp; g.a_bs = rowst;
  g.B = (const T*)w.phi + (long)s.nu * s.Lp; g.ldb = s.Lp; g.b_bs = rowst;
  g.C = w.W; g.ldc = n; g.c_bs = n * n;
  g.batch = w.Wk;
  // FP64 MFMA accumulation whatever the storage type of P and Phi (FP32 values
  // promote exactly): the length-L sums of the geminal entries carry no FP32
  // rounding.
  hipError_t e = run_gemm<32, 32, false, true, T, T, double, double>(g, st);
  if (e != hipSuccess || s.nk == 0) return e;
  GemmArgs u = plain(s.nu, s.nk, s.Lp);
  u.A = (const T*)w.phi; u.lda = s.Lp; u.a_bs = rowst;
  u.B = Uph; u.ldb = s.Lp; u.b_bs = 0;
  u.C = w.W + s.nd; u.ldc = n; u.c_bs = n * n;
  u.batch = w.Wk;
  return run_gemm<32, 32, false, true, T, T, double, double>(u, st);
}

hipError_t launch_W_build(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (s.bf16()) return hipErrorNotSupported;   // BF16 systems evaluate in FP64
  if (s.f32()) return W_build_t<float>(s, w, s.Uph32, st);
  return W_build_t<double>(s, w, s.Uph, st);
}

// Cofactor vectors of the local-energy derivatives:
//   Yt_up[i][mu] = sum_j A[j][i] P_dn[j][mu]   (= (Lambda Phi_dn^T W^{-1})[mu][i])
//   Yt_dn[j][nu] = sum_i A[j][i] P_up[i][nu]   (= (W^{-1} Phi_up Lambda)[j][nu])
// so that grad_i det/det = grad psi(r_i) . Yt[i] for every electron i.  Always
// FP64 arithmetic: A is FP64 and P (FP64 or FP32 storage) is promoted exactly.
// With unpaired orbitals the up electrons' vectors also collect the unpaired
// columns: Yt_up[i] += sum_l A[n_dn + l][i] U[:, l].
// Both spins' cofactor products of one walker per set of workgroups, for
// n_up = n_dn = n = 16 RB <= 96, Lp a multiple of 32 and no unpaired orbitals:
//   Yt_up[i][mu] = sum_j A[j][i] P_dn[j][mu],  Yt_dn[j][mu] = sum_i A[j][i] P_up[i][mu].
// The product is bound by its HBM traffic (P in, Yt out: 16 n Lp bytes per
// spin and walker) as much as by the FP64 matrix rate (K = n is short), and
// the generic tiled kernel spends most of its time staging K through LDS in
// short steps with M = n rounded up to 32-row tiles.  Here a workgroup owns 64
// columns of one spin of one walker: the n x 64 slab of P goes to LDS once, and
// wave rb computes output rows 16 rb .. 16 rb + 15 for the 64 columns as four
// 16 x 16 blocks, taking its A fragments straight from global memory (the
// walker's A is read by all its slabs from L2).  Products accumulate in k order
// in steps of 4 with the same MFMA instruction as the generic kernel, so Yt is
// bitwise the same.
template <typename T, int RB>
__global__ void __launch_bounds__(64 * RB) yt_kernel(const double* __restrict__ Ag, const T* __restrict__ Pg,
                                                     double* __restrict__ Yg, int n, int N, int Lp, int nslab) {
  extern __shared__ double Ps[];   // [n][64]
  // the slabs of one walker on one XCD (they share its A in that L2)
  const long b = xcd_remap(blockIdx.x, gridDim.x);
  const int slab = (int)(b % nslab);
  const int spin = (int)((b / nslab) & 1);   // 0: up rows of Yt (from P_dn), 1: down rows (from P_up)
  const long wk = b / nslab / 2;
  const int c0 = slab * 64;
  const int cw = min(64, Lp - c0);           // columns in this slab: 64, or 32 in the last one
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const double* A = Ag + wk * (long)n * n;
  const T* P = Pg + (wk * N + (spin == 0 ? n : 0)) * (long)Lp + c0;
  double* Y = Yg + (wk * N + (spin == 0 ? 0 : n)) * (long)Lp + c0;
  // this wave's A fragments for every K step, requested first (n is a multiple
  // of 16: no row or k past n).  op(A)[row][k] is A^T for the up rows (A[k][row])
  // and A for the down rows (A[row][k]); each step's loads take a uniform base
  // and one lane offset
  const int row = wave * 16 + (lane & 15), g = lane >> 4;
  const int tstride = spin == 0 ? 4 * n : 4;
  const int loff = spin == 0 ? g * n + row : row * n + g;
  constexpr int KS = 24;   // K steps of 4 for n <= 96
  double af[KS];
#pragma unroll
  for (int t = 0; t < KS; ++t)
    if (4 * t < n) af[t] = (A + (long)t * tstride)[loff];
  // the slab of P, two columns per load, all eight loads of a thread in
  // flight together (n x 32 pairs over 64 RB = 4 n threads; FP32 storage
  // promotes exactly)
  const int h = cw / 2;   // pairs of columns per row
  double2 pv[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int idx = tid + 64 * RB * q, k = idx >> 5, cp = idx & 31;
    pv[q] = double2{};
    if (cp < h) {
      if constexpr (sizeof(T) == 8) {
        pv[q] = *(const double2*)(P + (long)k * Lp + 2 * cp);
      } else {
        const float2 v = *(const float2*)(P + (long)k * Lp + 2 * cp);
        pv[q] = double2{(double)v.x, (double)v.y};
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 8; ++q) *(double2*)(Ps + 2 * (tid + 64 * RB * q)) = pv[q];
  __syncthreads();
  dx4 acc[4];
#pragma unroll
  for (int cb = 0; cb < 4; ++cb)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[cb][r] = 0.0;
#pragma unroll
  for (int t = 0; t < KS; ++t) {
    if (4 * t < n) {
      const double* pr = Ps + (4 * t + g) * 64 + (lane & 15);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[t], pr[16 * cb], acc[cb], 0, 0, 0);
    }
  }
  // 16 x 16 block layout: lane holds column lane % 16 and rows 4 r + lane / 16
#pragma unroll
  for (int cb = 0; cb < 4; ++cb) {
    const int c = cb * 16 + (lane & 15);
    if (c < cw) {
#pragma unroll
      for (int r = 0; r < 4; ++r) Y[(long)(wave * 16 + 4 * r + g) * Lp + c] = acc[cb][r];
    }
  }
}

// The same products for n = 80 or 96 (RB = 5 or 6 row blocks of 16): one
// workgroup of four waves per (walker, spin) walks all column slabs of P.
// With RB > 4 the per-slab kernel above puts RB waves on the four SIMDs, two
// of them on one, which then takes twice as long; here wave w computes row
// block w for all four 16-column blocks of a slab and row blocks 4 .. RB - 1
// for column block w, so that every SIMD runs the same number of MFMA chains
// (RB of the 4 RB of a slab).  The wave's A fragments
// (its row blocks, every K step) are loaded once per walker; the next slab's
// values are loaded into registers while the current slab multiplies out of
// LDS.  Same instruction, same k order: bitwise the per-slab kernel's Yt.
template <typename T, int RB>
__global__ void __launch_bounds__(256) yt_walker_kernel(const double* __restrict__ Ag, const T* __restrict__ Pg,
                                                        double* __restrict__ Yg, int N, int Lp) {
  static_assert(RB == 5 || RB == 6, "n = 80 or 96");
  constexpr int n = 16 * RB, KS = n / 4, NX = RB - 4;   // K steps; extra row blocks per wave
  constexpr int PAIRS = n * 32 / 256;                    // column pairs of a slab per thread
  __shared__ double Ps[n * 64];
  const long b = xcd_remap(blockIdx.x, gridDim.x);
  const int spin = (int)(b & 1);   // 0: up rows of Yt (from P_dn), 1: down rows (from P_up)
  const long wk = b >> 1;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nslab = (Lp + 63) / 64;
  const double* A = Ag + wk * (long)n * n;
  const T* P = Pg + (wk * N + (spin == 0 ? n : 0)) * (long)Lp;
  double* Y = Yg + (wk * N + (spin == 0 ? 0 : n)) * (long)Lp;
  // A fragments of row blocks wave and 4 .. RB - 1: op(A)[row][k] is A^T
  // (A[k][row]) for the up rows and A (A[row][k]) for the down rows
  const int g = lane >> 4;
  const int tstride = spin == 0 ? 4 * n : 4;
  double am[KS], ax[NX > 0 ? NX : 1][KS];
  {
    const int row = wave * 16 + (lane & 15);
    const int loff = spin == 0 ? g * n + row : row * n + g;
#pragma unroll
    for (int t = 0; t < KS; ++t) am[t] = (A + (long)t * tstride)[loff];
  }
#pragma unroll
  for (int j = 0; j < NX; ++j) {
    const int row = (4 + j) * 16 + (lane & 15);
    const int loff = spin == 0 ? g * n + row : row * n + g;
#pragma unroll
    for (int t = 0; t < KS; ++t) ax[j][t] = (A + (long)t * tstride)[loff];
  }
  // slab staging: thread tid moves column pairs idx = tid + 256 q (row idx / 32, pair idx % 32)
  double2 pv[PAIRS];
  auto load = [&](int c0) {
    const int h = min(64, Lp - c0) / 2;
#pragma unroll
    for (int q = 0; q < PAIRS; ++q) {
      const int idx = tid + 256 * q, k = idx >> 5, cp = idx & 31;
      pv[q] = double2{};
      if (cp < h) {
        if constexpr (sizeof(T) == 8) {
          pv[q] = *(const double2*)(P + (long)k * Lp + c0 + 2 * cp);
        } else {
          const float2 v = *(const float2*)(P + (long)k * Lp + c0 + 2 * cp);
          pv[q] = double2{(double)v.x, (double)v.y};
        }
      }
    }
  };
  load(0);
  for (int sl = 0; sl < nslab; ++sl) {
    const int c0 = sl * 64, cw = min(64, Lp - c0);
#pragma unroll
    for (int q = 0; q < PAIRS; ++q) *(double2*)(Ps + 2 * (tid + 256 * q)) = pv[q];
    __syncthreads();
    if (sl + 1 < nslab) load(c0 + 64);
    dx4 acc[4], accx[NX > 0 ? NX : 1];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[cb][r] = 0.0;
#pragma unroll
    for (int j = 0; j < NX; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) accx[j][r] = 0.0;
#pragma unroll
    for (int t = 0; t < KS; ++t) {
      const double* pr = Ps + (4 * t + g) * 64 + (lane & 15);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) acc[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(am[t], pr[16 * cb], acc[cb], 0, 0, 0);
#pragma unroll
      for (int j = 0; j < NX; ++j)
        accx[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[j][t], pr[16 * wave], accx[j], 0, 0, 0);
    }
    // 16 x 16 block layout: lane holds column lane % 16 and rows 4 r + lane / 16
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int c = cb * 16 + (lane & 15);
      if (c < cw) {
#pragma unroll
        for (int r = 0; r < 4; ++r) Y[(long)(wave * 16 + 4 * r + g) * Lp + c0 + c] = acc[cb][r];
      }
    }
    {
      const int c = wave * 16 + (lane & 15);
      if (c < cw) {
#pragma unroll
        for (int j = 0; j < NX; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) Y[(long)((4 + j) * 16 + 4 * r + g) * Lp + c0 + c] = accx[j][r];
      }
    }
    __syncthreads();   // every wave has read the slab before the next one is written
  }
}

template <typename T>
static hipError_t launch_yt(const SysDev& s, const WalkDev& w, hipStream_t st) {
  const int n = s.nu, nslab = (s.Lp + 63) / 64;
  if (n == 80 || n == 96) {   // four balanced waves per walker and spin
    if ((long)w.Wk * 2 > 0x7fffffffL) return hipErrorInvalidValue;
    if (n == 80)
      hipLaunchKernelGGL((yt_walker_kernel<T, 5>), dim3((unsigned)(w.Wk * 2)), dim3(256), 0, st, w.A, (const T*)w.P,
                         w.Yt, s.N, s.Lp);
    else
      hipLaunchKernelGGL((yt_walker_kernel<T, 6>), dim3((unsigned)(w.Wk * 2)), dim3(256), 0, st, w.A, (const T*)w.P,
                         w.Yt, s.N, s.Lp);
    return hipGetLastError();
  }
  const long total = (long)w.Wk * 2 * nslab;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  const size_t lds = sizeof(double) * (size_t)n * 64;
#define QMC_YT(R)                                                                                         \
  hipLaunchKernelGGL((yt_kernel<T, R>), dim3((unsigned)total), dim3(64 * R), lds, st, w.A, (const T*)w.P, w.Yt, n, \
                     s.N, s.Lp, nslab)
  switch (n / 16) {
    case 1: QMC_YT(1); break;
    case 2: QMC_YT(2); break;
    case 3: QMC_YT(3); break;
    case 4: QMC_YT(4); break;
    case 5: QMC_YT(5); break;
    default: QMC_YT(6); break;
  }
#undef QMC_YT
  return hipGetLastError();
}

template <typename T>
static hipError_t Y_build_t(const SysDev& s, const WalkDev& w, const T* Uph, hipStream_t st) {
  const long rowst = (long)s.N * s.Lp, n = s.nu;
  if (s.nk == 0 && s.nu == s.nd && s.nu % 16 == 0 && s.nu >= 16 && s.nu <= 96 && s.Lp % 32 == 0)
    return launch_yt<T>(s, w, st);
  hipError_t e;
  {
    GemmArgs g = plain(s.nu, s.Lp, s.nd);
    g.A = w.A; g.lda = n; g.a_bs = n * n;
    g.B = (const T*)w.P + (long)s.nu * s.Lp; g.ldb = s.Lp; g.b_bs = rowst;
    g.C = w.Yt; g.ldc = s.Lp; g.c_bs = rowst;
    g.batch = w.Wk;
    e = run_gemm<32, 64, true, false, double, T, double, double, 16>(g, st);
    if (e != hipSuccess) return e;
  }
  if (s.nk > 0) {
    GemmArgs g = plain(s.nu, s.Lp, s.nk);
    g.A = w.A + (long)s.nd * n; g.lda = n; g.a_bs = n * n;
    g.B = Uph; g.ldb = s.Lp; g.b_bs = 0;
    g.C = w.Yt; g.ldc = s.Lp; g.c_bs = rowst;
    g.batch = w.Wk;
    g.accumulate = 1;
    e = run_gemm<32, 64, true, false, double, T, double, double, 16>(g, st);
    if (e != hipSuccess) return e;
  }
  {
    GemmArgs g = plain(s.nd, s.Lp, s.nu);
    g.A = w.A; g.lda = n; g.a_bs = n * n;
    g.B = (const T*)w.P; g.ldb = s.Lp; g.b_bs = rowst;
    g.C = w.Yt + (long)s.nu * s.Lp; g.ldc = s.Lp; g.c_bs = rowst;
    g.batch = w.Wk;
    e = run_gemm<32, 64, false, false, double, T, double, double, 16>(g, st);
  }
  return e;
}

hipError_t launch_Y_build(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (s.bf16()) return hipErrorNotSupported;
  if (s.f32()) return Y_build_t<float>(s, w, s.Uph32, st);
  return Y_build_t<double>(s, w, s.Uph, st);
}

}  // namespace qmc
