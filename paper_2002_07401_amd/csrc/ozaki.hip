// The geminal products P = Phi Lambda (rows of the up electrons) and
// P = Phi Lambda^T (down electrons), agp_expansion / eq:wfAGPs, on the int8
// matrix cores of gfx950 without rounding error in the accumulation.
//
// Every FP64 row x of Phi (and every column of Lambda) is split into S int8
// digits with one power-of-two scale per row:
//     x = 2^(E-5) * sum_{a<S} d_a 2^(-7a) + rest,   |d_a| <= 64,
//     E = floor(log2 max|x|),  |rest| <= 2^(E-6-7(S-1)).
// The digit products d_a . g_b of a row of Phi and a column of Lambda are sums
// of K terms of magnitude <= 2^12, so their int32 accumulation on the matrix
// cores is exact for K < 2^19.  The product keeps every pair with a + b < S
// (the leading "diagonals" q = a + b of the digit expansion), adds them in FP64
// and scales once:
//     P = 2^(Ex + Ey - 10) * sum_{q<S} 2^(-7q) sum_{a+b=q} d_a . g_b.
// The leading digit pair alone is a product of 7-bit inputs (the reduced-
// precision build); each further diagonal is one correction term.  The error
// left after S diagonals is below (S + 3) 2^(2-7S) max|x| max|y| K, and every
// step in between is exact, so the result is the FP64 product to that bound
// (S = 7: 7e-14 of max|x| max|y| K).
//
// Digit layout ("fragment tiles"): for plane a, group g of 32 rows and K step
// j (32 digits), one 1 KB block in the lane order of a v_mfma_i32_32x32x32_i8
// operand: lane l holds row 32 g + l % 32, digits 32 j + 16 (l / 32) .. +16, at
// byte 16 l; block (a, g, j) at ((a G + g) J + j) KiB, G = ceil(rows / 32),
// J = Kp / 32.  A wave copies one block with one contiguous 1 KB load.
#include "internal.h"

namespace qmc {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int kOzMaxKSteps = 256;   // K <= 8192 (one K step per thread of a workgroup)
constexpr int kNoRow = -2147483647 - 1;   // exponent of a row or column with no output

// ---------------------------------------------------------------------------
// digits
// ---------------------------------------------------------------------------
// One workgroup per group of 32 rows.  Row m of the input starts at
// X + (m / grp) * gs + (m % grp) * ld and has K values (zeros up to Kp); rows
// m >= rows of the last group get zero digits.  Exponents to expo[m].  K is
// read in chunks of 64 values, 8 threads per row reading 64 contiguous bytes
// each; the chunk passes through LDS so that each thread then turns 8 values
// of one row into digits and the 32 rows' pieces of a tile go out together.
// With ridx, row m of the tiles is row ridx[m] of X (m < *rcnt; the rest of
// the rows up to `rows` are not written) and the exponents go to expo_c in
// that order (copied from expo[ridx[m]] with have_expo).
__global__ void __launch_bounds__(256)
slice_tiles_kernel(const double* __restrict__ X, long rows, int K, int Kp, int grp, long gs, long ld, int S,
                   int8_t* __restrict__ out, long plane, int* __restrict__ expo, int have_expo,
                   const int* __restrict__ ridx, const int* __restrict__ rcnt, int* __restrict__ expo_c) {
  __shared__ double xs[32][65];
  __shared__ double red[32][9];
  __shared__ int se[32];
  const long g = blockIdx.x;
  const int tid = threadIdx.x;
  const int J = Kp / 32;
  const long nrow = ridx ? min(rows, (long)*rcnt) : rows;
  if (32 * g >= nrow) return;   // (uniform) tiles past the compacted rows are not read
  const int lr = tid >> 3, lc = tid & 7;          // load mapping: row, 8-value piece
  const long lm = 32 * g + lr;
  const long src = lm < nrow ? (ridx ? (long)ridx[lm] : lm) : -1;
  const double* xrow = src >= 0 ? X + (src / grp) * gs + (src % grp) * ld : nullptr;
  int* eout = ridx ? expo_c : expo;
  // pass 1: row maxima (unless the producer of X gave the exponents)
  if (have_expo) {
    if (tid < 32) {
      const long m = 32 * g + tid;
      se[tid] = m < nrow ? expo[ridx ? (long)ridx[m] : m] : 0;
      if (ridx && m < nrow) expo_c[m] = se[tid];
    }
  } else {
    double mx = 0.0;
    if (xrow)
      for (int k = 8 * lc; k < K; k += 64)
#pragma unroll
        for (int v = 0; v < 8; ++v)
          if (k + v < K) mx = fmax(mx, fabs(xrow[k + v]));
    red[lr][lc] = mx;
    __syncthreads();
    if (tid < 32) {
      double m = 0.0;
      for (int c = 0; c < 8; ++c) m = fmax(m, red[tid][c]);
      const int E = m > 0.0 ? ilogb(m) : 0;
      se[tid] = E;
      if (32 * g + tid < nrow) eout[32 * g + tid] = E;
    }
  }
  __syncthreads();
  // pass 2: digits, 64 values of every row at a time
  const int r = tid & 31, p = tid >> 5;           // digit mapping: row, 8-value piece
  const int E = se[r];
  for (int k0 = 0; k0 < Kp; k0 += 64) {
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int k = k0 + 8 * lc + v;
      xs[lr][8 * lc + v] = (xrow && k < K) ? xrow[k] : 0.0;
    }
    __syncthreads();
    const int k = k0 + 8 * p;                     // this thread's 8 values: row r, k .. k + 7
    if (k < Kp) {
      double t[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) t[v] = ldexp(xs[r][8 * p + v], 5 - E);
      // tile position: K step k / 32, lane 32 ((k % 32) / 16) + r, byte k % 16
      int8_t* dst = out + (g * J + k / 32) * 1024 + 16 * (32 * ((k % 32) / 16) + r) + (k % 16);
      for (int a = 0; a < S; ++a) {
        uint32_t w0 = 0u, w1 = 0u;
#pragma unroll
        for (int v = 0; v < 8; ++v) {
          const double d = rint(t[v]);
          t[v] = (t[v] - d) * 128.0;
          const uint32_t b = (uint32_t)(uint8_t)(int8_t)(int)d;
          if (v < 4) w0 |= b << (8 * v); else w1 |= b << (8 * (v - 4));
        }
        *reinterpret_cast<uint2*>(dst + a * plane) = make_uint2(w0, w1);
      }
    }
    __syncthreads();
  }
}

// bytes of one digit plane of `rows` rows in fragment tiles
long oz_plane_bytes(long rows, int Kp) { return (rows + 31) / 32 * 32 * (long)Kp; }

// Digits of `rows` rows into fragment tiles (plane: bytes per digit plane).
hipError_t launch_slice_tiles(const double* X, long rows, int K, int Kp, int grp, long gs, long ld, int S, int8_t* out,
                              long plane, int* expo, hipStream_t st, bool have_expo, const int* ridx, const int* rcnt,
                              int* expo_c) {
  if (rows <= 0) return hipSuccess;
  if (Kp % 32 != 0 || K > Kp || S < 1 || S > kOzMaxSlices) return hipErrorInvalidValue;
  if (plane < oz_plane_bytes(rows, Kp)) return hipErrorInvalidValue;
  const long G = (rows + 31) / 32;
  if (ridx && (!rcnt || !expo_c)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(slice_tiles_kernel, dim3((unsigned)G), dim3(256), 0, st, X, rows, K, Kp, grp, gs, ld, S, out,
                     plane, expo, have_expo ? 1 : 0, ridx, rcnt, expo_c);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// products
// ---------------------------------------------------------------------------
// C[m][n] = sum_k A[m][k] B[n][k] from the digit tiles of A (rows of Phi) and
// of B (rows of Lambda^T for P_up, of Lambda for P_dn).
struct OzArgs {
  int M, N, Kp;
  const int8_t* A; long a_plane; const int* ea;                       // A tiles, exponents [M]
  const int8_t* B; long b_plane; const int* eb;                       // B tiles, exponents [N]
  double* C; int c_grp; long c_gs; long ldc;                          // C row m at (m/grp)*gs + (m%grp)*ldc
  void* C2; int c2_bf16;                                              // optional FP32 / BF16 copy
  double* CT; long ct_gs; long ct_ld;                                 // optional transposed FP64 copy:
                                                                      // C[m][n] at (m/grp)*ct_gs + n*ct_ld + m%grp
  const uint8_t* kmask; int kmask_ld;                                 // nonzero 16 x 64 tiles of B^T
  const int* ridx; const int* rcnt;   // optional: output row m is row ridx[m] of C (and CT), m < *rcnt
};

__device__ __forceinline__ long oz_xcd_remap(long id, long total) {
  const long per = total / 8, rem = total % 8;
  const long x = id % 8, slot = id / 8;
  return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + slot;
}

// 256 threads (4 waves, one per SIMD) over a 128 x 64 tile of C; wave w owns
// rows 32 w .. 32 w + 31 and all 64 columns, i.e. two 32 x 32 blocks and one
// v_mfma_i32_32x32x32_i8 accumulator per block and diagonal q < S (up to 512
// registers per wave at this occupancy).  Per K step the block needs 4 S blocks
// of A tiles and 2 S of B tiles; they are copied from global memory straight
// into LDS (global_load_lds, no register staging) through a ring of three
// stages, and each wave reads its fragments one step ahead into a second set of
// registers, so that LDS reads, copies and products of neighbouring steps
// overlap; within a step the copies and fragment reads are spread between the
// products (scheduling groups), so that neither queue holds the matrix core
// back.  Every wave issues the same number of copies per step (slots past the
// last block copy into `spare`, steps past the end repeat the last one), so
// the count of copies in flight is the same on every path and a fixed vmcnt
// tells when a step has landed.  Rows past M or N read the last tile group
// (their products land in outputs that are not stored).  The exponents and
// output offsets of the tile's rows and columns are loaded once, ahead of the
// first copies, and kept in LDS for the epilogue, which then needs no global
// load and no division per output.
template <int S>
__global__ void __launch_bounds__(256) ozaki_gemm_kernel(OzArgs g, int gx, int gy) {
  constexpr int NA = S * 4, NB = S * 2;          // fragment blocks per stage: A (4 row groups), B (2)
  constexpr int NBLK = NA + NB;
  constexpr int PW = (NBLK + 3) / 4;             // copies per wave and step
  // three separate arrays (not one indexed by stage): with each access naming a
  // fixed array the compiler can tell that the copies in flight write a stage
  // other than the one being read, and does not wait for them
  __shared__ __attribute__((aligned(16))) int8_t st0[NBLK][1024];
  __shared__ __attribute__((aligned(16))) int8_t st1[NBLK][1024];
  __shared__ __attribute__((aligned(16))) int8_t st2[NBLK][1024];
  __shared__ __attribute__((aligned(16))) int8_t spare[1024];
  __shared__ short steps[kOzMaxKSteps];          // K steps with a nonzero B^T tile, in order
  __shared__ int nsteps, wcnt[4];
  __shared__ long rows_c[128], rows_t[128];      // offsets of the tile's output rows in C and CT
  __shared__ int rows_e[128], cols_e[64];        // exponents of its rows and columns (kNoRow: no output)
  // with a row list, only its tiles are spread over the XCDs (the grid is
  // sized for every row; the workgroups past the list's tiles leave at once)
  const int Mr = g.ridx ? min(g.M, *g.rcnt) : g.M;   // rows with an output
  const long nt = g.ridx ? (long)((Mr + 127) / 128) * gx : (long)gx * gy;
  if ((long)blockIdx.x >= nt) return;                  // (uniform, before any copy or barrier)
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int J = g.Kp / 32;
  const int GA = (g.M + 31) / 32, GB = (g.N + 31) / 32;
  int m0 = 0, n0 = 0, ns = J;
  // per copy slot: the tile's base address (uniform over the wave: scalar
  // registers) and the stage block it fills (-1: the spare block)
  const int wvs = __builtin_amdgcn_readfirstlane(wave);
  const int8_t* src[PW];
  int dst[PW];
  int ld_e = kNoRow, ld_r = 0;
  // K offset of step t (the step list's entries; past the end the last one)
  auto koff = [&](int t) -> long { return ns > 0 ? 1024L * steps[min(t, ns - 1)] : 0; };
  auto issue_k = [&](long k, int8_t (&buf)[NBLK][1024]) {
#pragma unroll
    for (int j = 0; j < PW; ++j) {
      int8_t* d = dst[j] >= 0 ? &buf[dst[j]][0] : &spare[0];
      __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)(src[j] + (k + 16 * lane)),
                                       (__attribute__((address_space(3))) void*)d, 16, 0, 0);
    }
  };
  v16i acc[S][2];

  // Fragments of step t sit in registers (set 0 / set 1 by parity) while step
  // t + 1's are read from LDS, and the copies of steps t + 2 and t + 3 are in
  // flight.  Step t: wait for this wave's reads of step t's fragments (lgkmcnt)
  // and for its copies of step t + 1 (vmcnt: only the PW copies of step t + 2
  // may still be outstanding, copies complete in issue order); one barrier
  // (every wave's copies of t + 1 have landed and every wave has read step t's
  // stage, which the copies of step t + 3 then reuse); issue step t + 3; read
  // step t + 1's fragments; the products of step t.
  v4i fa0[S], fb0[S][2], fa1[S], fb1[S][2];
  auto frags = [&](int8_t (&buf)[NBLK][1024], v4i (&fa)[S], v4i (&fb)[S][2]) {
#pragma unroll
    for (int q = 0; q < S; ++q) {
      fa[q] = *reinterpret_cast<const v4i*>(&buf[q * 4 + wave][16 * lane]);
      fb[q][0] = *reinterpret_cast<const v4i*>(&buf[NA + q * 2][16 * lane]);
      fb[q][1] = *reinterpret_cast<const v4i*>(&buf[NA + q * 2 + 1][16 * lane]);
    }
  };
  auto mma = [&](const v4i (&fa)[S], const v4i (&fb)[S][2]) {
#pragma unroll
    for (int a = 0; a < S; ++a)
#pragma unroll
      for (int b = 0; a + b < S; ++b)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[a + b][c] = __builtin_amdgcn_mfma_i32_32x32x32_i8(fa[a], fb[b][c], acc[a + b][c], 0, 0, 0);
  };
  // (past the last step the fragment reads fetch a repeated stage; unused)
  auto step = [&](int t, int8_t (&cur)[NBLK][1024], int8_t (&nx1)[NBLK][1024], const v4i (&fa)[S],
                  const v4i (&fb)[S][2], v4i (&na)[S], v4i (&nb)[S][2]) {
    const long k3 = koff(t + 3);
    __builtin_amdgcn_s_waitcnt(0x0070 | PW);   // vmcnt(PW), lgkmcnt(0); expcnt: no wait
    __builtin_amdgcn_s_barrier();
    issue_k(k3, cur);
    frags(nx1, na, nb);
    mma(fa, fb);
    // order within the step: each copy, then each fragment read, followed by
    // one product; the remaining products last
    constexpr int NR = 3 * S, NM = S * (S + 1);
    static_assert(NM >= NR + PW, "fewer products than memory operations to spread");
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x0020, 1, 0);   // one VMEM read (the copy)
      __builtin_amdgcn_sched_group_barrier(0x0008, 1, 0);   // one MFMA
    }
#pragma unroll
    for (int i = 0; i < NR; ++i) {
      __builtin_amdgcn_sched_group_barrier(0x0100, 1, 0);   // one DS read
      __builtin_amdgcn_sched_group_barrier(0x0008, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x0008, NM - NR - PW, 0);
  };
  // The epilogue.  32 x 32 accumulator layout: lane holds column lane % 32
  // and, in register r, row 8 (r / 4) + 4 (lane / 32) + r % 4.
  auto epilogue = [&]() {
    const bool full = m0 + 128 <= Mr && n0 + 64 <= g.N;
    int en[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) en[c] = cols_e[32 * c + (lane & 31)];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int lr = wave * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
      const int er = rows_e[lr];
      const long oc = rows_c[lr], ot = rows_t[lr];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const int gn = n0 + 32 * c + (lane & 31);
        if (full || (er != kNoRow && gn < g.N)) {
          double v = 0.0;
#pragma unroll
          for (int q = S - 1; q >= 0; --q) v = v * (1.0 / 128.0) + (double)acc[q][c][r];
          v = ldexp(v, er + en[c] - 10);
          g.C[oc + gn] = v;
          if (g.C2) {
            if (g.c2_bf16) ((bf16s*)g.C2)[oc + gn] = bf16s(v);
            else ((float*)g.C2)[oc + gn] = (float)v;
          }
          if (g.CT) g.CT[ot + (long)gn * g.ct_ld] = v;
        }
      }
    }
  };

  // the tile's place, its step list, the copy sources of this wave's PW
  // slots (lane l copies the 16 bytes at 16 l of a block), the exponents and
  // row indices of its rows (threads 0..127) and columns (128..191), then the
  // copies of its first three steps.  The exponent loads go out before the
  // copies: they complete first, so the copy counts of the main loop hold.
  {
    const long Lb = oz_xcd_remap(blockIdx.x, nt);
    m0 = (int)((Lb / gx) % gy) * 128;
    n0 = (int)(Lb % gx) * 64;
  }
  {
    // thread t < J flags K step t (a nonzero B^T tile); the flagged steps are
    // compacted in order by wave ballots (J <= 256)
    bool nz = tid < J;
    if (nz && g.kmask) {
      const int nb = n0 / kLamTileN;
      nz = g.kmask[(long)(2 * tid) * g.kmask_ld + nb] || g.kmask[(long)(2 * tid + 1) * g.kmask_ld + nb];
    }
    const unsigned long long bal = __ballot(nz);
    if (lane == 0) wcnt[wave] = __popcll(bal);
    __syncthreads();
    int pos = __popcll(bal & ((1ull << lane) - 1ull));
    for (int k = 0; k < wave; ++k) pos += wcnt[k];
    if (nz) steps[pos] = (short)tid;
    if (tid == 0) nsteps = wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
    ns = nsteps;
  }
#pragma unroll
  for (int j = 0; j < PW; ++j) {
    const int b = wvs * PW + j;
    dst[j] = b < NBLK ? b : -1;
    if (b < NA) {
      const int q = b / 4, grp = min(m0 / 32 + b % 4, GA - 1);
      src[j] = g.A + (long)q * g.a_plane + (long)grp * J * 1024;
    } else if (b < NBLK) {
      const int q = (b - NA) / 2, grp = min(n0 / 32 + (b - NA) % 2, GB - 1);
      src[j] = g.B + (long)q * g.b_plane + (long)grp * J * 1024;
    } else {
      src[j] = g.B;   // any valid address: the copy lands in `spare`
    }
  }
  if (tid < 128) {
    const int gm = m0 + tid;
    if (gm < Mr) { ld_e = g.ea[gm]; ld_r = g.ridx ? g.ridx[gm] : gm; }
  } else if (tid < 192) {
    const int gn = n0 + tid - 128;
    if (gn < g.N) ld_e = g.eb[gn];
  }
  issue_k(koff(0), st0);
  issue_k(koff(1), st1);
  issue_k(koff(2), st2);
  __builtin_amdgcn_s_waitcnt(0x0F70 | (2 * PW));   // vmcnt(2 PW): step 0 landed
  __builtin_amdgcn_s_barrier();
  if (tid < 128) {   // row r of C sits at (r / grp) gs + (r % grp) ldc, of CT at (r / grp) ct_gs + r % grp
    rows_e[tid] = ld_e;
    const long q = ld_r / g.c_grp, rm = ld_r - q * g.c_grp;
    rows_c[tid] = q * g.c_gs + rm * g.ldc;
    rows_t[tid] = q * g.ct_gs + rm;
  } else if (tid < 192) {
    cols_e[tid - 128] = ld_e;
  }
#pragma unroll
  for (int q = 0; q < S; ++q)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[q][c][r] = 0;
  frags(st0, fa0, fb0);
  for (int t = 0; t < ns; t += 6) {
    step(t, st0, st1, fa0, fb0, fa1, fb1);
    if (t + 1 < ns) step(t + 1, st1, st2, fa1, fb1, fa0, fb0);
    if (t + 2 < ns) step(t + 2, st2, st0, fa0, fb0, fa1, fb1);
    if (t + 3 < ns) step(t + 3, st0, st1, fa1, fb1, fa0, fb0);
    if (t + 4 < ns) step(t + 4, st1, st2, fa0, fb0, fa1, fb1);
    if (t + 5 < ns) step(t + 5, st2, st0, fa1, fb1, fa0, fb0);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): no copy outlives the workgroup
  __syncthreads();                       // the row and column data are visible (also when no K step ran)
  epilogue();
}

template <int S>
static hipError_t run_ozaki(const OzArgs& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.Kp % 32 != 0 || g.Kp / 32 > kOzMaxKSteps) return hipErrorInvalidValue;
  const int gx = (g.N + 63) / 64, gy = (g.M + 127) / 128;
  const long total = (long)gx * gy;
  if (total > 0x7fffffffL) return hipErrorInvalidValue;
  hipLaunchKernelGGL((ozaki_gemm_kernel<S>), dim3((unsigned)total), dim3(256), 0, st, g, gx, gy);
  return hipGetLastError();
}

static hipError_t run_ozaki_s(int S, const OzArgs& g, hipStream_t st) {
  switch (S) {
    case 6: return run_ozaki<6>(g, st);
    case 7: return run_ozaki<7>(g, st);
    case 8: return run_ozaki<8>(g, st);
    default: return hipErrorInvalidValue;
  }
}

// Digits of Lambda's columns (rows of Lambda^T, the B operand of P_up) and of
// its rows (the B operand of P_dn): tiles [2][oz_s][plane], exponents [2][Lp].
hipError_t launch_oz_lambda(const SysDev& s, hipStream_t st) {
  const long plane = oz_plane_bytes(s.Lp, s.Lp);
  hipError_t e = launch_slice_tiles(s.lamT, s.Lp, s.Lp, s.Lp, 1 << 30, 0, s.Lp, s.oz_s, s.oz_lam, plane, s.oz_elam,
                                    st);
  if (e != hipSuccess) return e;
  return launch_slice_tiles(s.lam, s.Lp, s.Lp, s.Lp, 1 << 30, 0, s.Lp, s.oz_s, s.oz_lam + (long)s.oz_s * plane, plane,
                            s.oz_elam + s.Lp, st);
}

// Bytes of the walkers' digit tiles: up rows, then down rows.
long oz_phi_bytes(const SysDev& s, long Wk) {
  return (long)s.oz_s * (oz_plane_bytes(Wk * s.nu, s.Lp) + oz_plane_bytes(Wk * s.nd, s.Lp));
}

// The rows of one P half (rows i0 .. i0 + n - 1 of every walker) whose
// electron has moved since its row was last built, listed in increasing order
// of their index walker * n + i (so that a block of compacted rows still
// writes P and its transpose in nearly contiguous runs): per block of 256 rows
// the count of moved ones, an exclusive scan of the counts, then the list,
// with the positions recorded.  ALL (a full build): positions only.
__device__ __forceinline__ bool row_moved(const double* __restrict__ r, const double* __restrict__ rP, long o) {
  return !(r[o] == rP[o] && r[o + 1] == rP[o + 1] && r[o + 2] == rP[o + 2]);
}

__global__ void __launch_bounds__(256)
p_dirty_count_kernel(const double* __restrict__ r, const double* __restrict__ rP, int Wk, int N, int i0, int n,
                     int* __restrict__ bcnt) {
  __shared__ int wc[4];
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool moved = t < (long)Wk * n && row_moved(r, rP, ((t / n) * N + i0 + t % n) * 3);
  const unsigned long long b = __ballot(moved);
  if (lane == 0) wc[wave] = __popcll(b);
  __syncthreads();
  if (threadIdx.x == 0) bcnt[blockIdx.x] = wc[0] + wc[1] + wc[2] + wc[3];
}

// one workgroup of 1024 threads: bcnt[0 .. nb) -> exclusive offsets in place,
// the total to *cnt
__global__ void __launch_bounds__(1024) p_dirty_scan_kernel(int* __restrict__ bcnt, int nb, int* __restrict__ cnt) {
  __shared__ int part[1024];
  int carry = 0;
  for (int c0 = 0; c0 < nb; c0 += 1024) {
    const int i = c0 + (int)threadIdx.x;
    const int v = i < nb ? bcnt[i] : 0;
    part[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
      const int x = threadIdx.x >= (unsigned)o ? part[threadIdx.x - o] : 0;
      __syncthreads();
      part[threadIdx.x] += x;
      __syncthreads();
    }
    if (i < nb) bcnt[i] = carry + part[threadIdx.x] - v;
    carry += part[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *cnt = carry;
}

template <bool ALL>
__global__ void __launch_bounds__(256)
p_dirty_write_kernel(const double* __restrict__ r, double* __restrict__ rP, int Wk, int N, int i0, int n,
                     const int* __restrict__ boff, int* __restrict__ idx) {
  __shared__ int wc[4];
  const long t = (long)blockIdx.x * 256 + threadIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long o = ((t / n) * N + i0 + t % n) * 3;
  const bool moved = t < (long)Wk * n && (ALL || row_moved(r, rP, o));
  if (!ALL) {
    const unsigned long long b = __ballot(moved);
    if (lane == 0) wc[wave] = __popcll(b);
    __syncthreads();
    int at = boff[blockIdx.x] + __popcll(b & ((1ull << lane) - 1ull));
    for (int k = 0; k < wave; ++k) at += wc[k];
    if (moved) idx[at] = (int)t;
  }
  if (moved) { rP[o] = r[o]; rP[o + 1] = r[o + 1]; rP[o + 2] = r[o + 2]; }
}

hipError_t launch_moved_rows(const SysDev& s, const WalkDev& w, int h, bool moved_only, int** ridx, int** rcnt,
                             hipStream_t st) {
  *ridx = nullptr;
  *rcnt = nullptr;
  if (!w.rpos_P) return moved_only ? hipErrorInvalidValue : hipSuccess;
  const int n = h == 0 ? s.nu : s.nd, i0 = h == 0 ? 0 : s.nu;
  const long rows = (long)w.Wk * n;
  if (rows <= 0) return hipSuccess;
  const int nb = (int)((rows + 255) / 256);
  if (moved_only) {
    *ridx = w.dirty_idx + (h == 0 ? 0 : (long)w.Wk * s.nu);
    *rcnt = w.dirty_cnt + h;
    int* boff = w.dirty_blk;
    hipLaunchKernelGGL(p_dirty_count_kernel, dim3(nb), dim3(256), 0, st, w.r, w.rpos_P, w.Wk, s.N, i0, n, boff);
    hipLaunchKernelGGL(p_dirty_scan_kernel, dim3(1), dim3(1024), 0, st, boff, nb, *rcnt);
    hipLaunchKernelGGL(p_dirty_write_kernel<false>, dim3(nb), dim3(256), 0, st, w.r, w.rpos_P, w.Wk, s.N, i0, n,
                       boff, *ridx);
  } else {
    hipLaunchKernelGGL(p_dirty_write_kernel<true>, dim3(nb), dim3(256), 0, st, w.r, w.rpos_P, w.Wk, s.N, i0, n,
                       nullptr, nullptr);
  }
  return hipGetLastError();
}

// P halves (bit 0: up rows, bit 1: down rows) from the FP64 basis rows in
// phi64: digits of those rows first (oz_phi: up tiles, then down tiles; with
// have_expo the rows' exponents in oz_ephi are already set), then the
// products; P64 gets the FP64 result, lo (if given) its FP32 / BF16 copy and PT
// (if given) its transpose per walker, PT[w][mu][i].
hipError_t launch_P_build_oz(const SysDev& s, const WalkDev& w, int halves, const double* phi64, double* P64,
                             void* lo, bool lo_bf16, hipStream_t st, bool have_expo, double* PT, int dirty) {
  const long rowst = (long)s.N * s.Lp;
  const long planeB = oz_plane_bytes(s.Lp, s.Lp);
  const int mask_ld = (s.Lp + kLamTileN - 1) / kLamTileN;
  const long up_bytes = (long)s.oz_s * oz_plane_bytes((long)w.Wk * s.nu, s.Lp);
  for (int h = 0; h < 2; ++h) {
    if (!(halves & (1 << h))) continue;
    const int n = h == 0 ? s.nu : s.nd;
    if (n == 0) continue;
    const long r0 = h == 0 ? 0 : (long)s.nu * s.Lp;
    const long rows = (long)w.Wk * n;
    const long planeA = oz_plane_bytes(rows, s.Lp);
    int8_t* tiles = w.oz_phi + (h == 0 ? 0 : up_bytes);
    int* ex = w.oz_ephi + (h == 0 ? 0 : (long)w.Wk * s.nu);
    // rows of this half that need a product (all, or those whose electron has
    // moved: the positions of the rows built are recorded either way)
    const bool dirt = (dirty >> h) & 1;
    int* ridx = nullptr;
    int* rcnt = nullptr;
    int* exc = nullptr;
    hipError_t e = launch_moved_rows(s, w, h, dirt, &ridx, &rcnt, st);
    if (e != hipSuccess) return e;
    if (ridx) exc = w.oz_ephi_c + (h == 0 ? 0 : (long)w.Wk * s.nu);
    // rows m of this half: walker m / n, electron m % n of the spin
    e = launch_slice_tiles(phi64 + r0, rows, s.L, s.Lp, n, rowst, s.Lp, s.oz_s, tiles, planeA, ex, st, have_expo,
                           ridx, rcnt, exc);
    if (e != hipSuccess) return e;
    OzArgs g{};
    g.M = (int)rows; g.N = s.Lp; g.Kp = s.Lp;
    g.A = tiles; g.a_plane = planeA; g.ea = ridx ? exc : ex;
    g.ridx = ridx; g.rcnt = rcnt;
    g.B = s.oz_lam + (long)h * s.oz_s * planeB; g.b_plane = planeB; g.eb = s.oz_elam + (long)h * s.Lp;
    g.C = P64 + r0; g.c_grp = n; g.c_gs = rowst; g.ldc = s.Lp;
    if (lo) {
      g.C2 = lo_bf16 ? (void*)((bf16s*)lo + r0) : (void*)((float*)lo + r0);
      g.c2_bf16 = lo_bf16 ? 1 : 0;
    }
    if (PT) {   // PT[w][mu][i] for every electron i of walker w (this half: i = i0 + m % n)
      g.CT = PT + (h == 0 ? 0 : s.nu);
      g.ct_gs = (long)s.Lp * s.pt_ld();
      g.ct_ld = s.pt_ld();
    }
    g.kmask = h == 0 ? s.lam_mask : s.lamT_mask;
    g.kmask_ld = mask_ld;
    e = run_ozaki_s(s.oz_s, g, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Pfaffian B rows (QMC_REFINED): B^s_j = psi(r_j)^T K^{s s_j} as the same
// error-free digit products, B operand = the rows of K^T.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) oz_transpose_kernel(const double* __restrict__ K, double* __restrict__ T,
                                                           int Lp) {
  __shared__ double t[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
  for (int r = ty; r < 32; r += 8)
    t[r][tx] = (by + r < Lp && bx + tx < Lp) ? K[(long)(by + r) * Lp + bx + tx] : 0.0;
  __syncthreads();
  for (int r = ty; r < 32; r += 8)
    if (bx + r < Lp && by + tx < Lp) T[(long)(bx + r) * Lp + by + tx] = t[tx][r];
}

hipError_t launch_oz_pf_K(const SysDev& s, hipStream_t st) {
  if (!s.pf_refined() || !s.oz_lam || !s.oz_tmp) return hipErrorInvalidValue;
  const long plane = oz_plane_bytes(s.Lp, s.Lp);
  const double* K[4] = {s.Kuu, s.Kud, s.Kdu, s.Kdd};
  const dim3 grid((s.Lp + 31) / 32, (s.Lp + 31) / 32);
  for (int q = 0; q < 4; ++q) {
    hipLaunchKernelGGL(oz_transpose_kernel, grid, dim3(256), 0, st, K[q], s.oz_tmp, s.Lp);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
      e = launch_slice_tiles(s.oz_tmp, s.Lp, s.Lp, s.Lp, 1 << 30, 0, s.Lp, s.oz_s, s.oz_lam + (long)q * s.oz_s * plane,
                             plane, s.oz_elam + (long)q * s.Lp, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_pf_B_build_oz(const SysDev& s, const WalkDev& w, hipStream_t st) {
  if (!s.pf_refined() || !w.oz_phi || !w.oz_ephi) return hipErrorInvalidValue;
  const long rowst = (long)s.N * s.Lp;
  const long planeB = oz_plane_bytes(s.Lp, s.Lp);
  const long up_bytes = (long)s.oz_s * oz_plane_bytes((long)w.Wk * s.nu, s.Lp);
  const double* phi = (const double*)w.phi;   // FP64 rows in this mode
  // digits of the up rows, then the down rows (rows m: walker m / n, electron m % n of the spin)
  for (int h = 0; h < 2; ++h) {
    const int n = h == 0 ? s.nu : s.nd;
    if (n == 0) continue;
    const long rows = (long)w.Wk * n;
    hipError_t e = launch_slice_tiles(phi + (h == 0 ? 0 : (long)s.nu * s.Lp), rows, s.L, s.Lp, n, rowst, s.Lp,
                                      s.oz_s, w.oz_phi + (h == 0 ? 0 : up_bytes), oz_plane_bytes(rows, s.Lp),
                                      w.oz_ephi + (h == 0 ? 0 : (long)w.Wk * s.nu), st);
    if (e != hipSuccess) return e;
  }
  // B^u = [Phi_u K^{uu}; Phi_d K^{ud}] in P, B^d = [Phi_u K^{du}; Phi_d K^{dd}] in Bd
  struct Part { int q, h; double* out; };
  const Part parts[4] = {{0, 0, (double*)w.P}, {1, 1, (double*)w.P}, {2, 0, w.Bd}, {3, 1, w.Bd}};
  for (const Part& x : parts) {
    const int n = x.h == 0 ? s.nu : s.nd;
    if (n == 0) continue;
    const long rows = (long)w.Wk * n;
    OzArgs g{};
    g.M = (int)rows; g.N = s.Lp; g.Kp = s.Lp;
    g.A = w.oz_phi + (x.h == 0 ? 0 : up_bytes); g.a_plane = oz_plane_bytes(rows, s.Lp);
    g.ea = w.oz_ephi + (x.h == 0 ? 0 : (long)w.Wk * s.nu);
    g.B = s.oz_lam + (long)x.q * s.oz_s * planeB; g.b_plane = planeB; g.eb = s.oz_elam + (long)x.q * s.Lp;
    g.C = x.out + (x.h == 0 ? 0 : (long)s.nu * s.Lp); g.c_grp = n; g.c_gs = rowst; g.ldc = s.Lp;
    const hipError_t e = run_ozaki_s(s.oz_s, g, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace qmc
