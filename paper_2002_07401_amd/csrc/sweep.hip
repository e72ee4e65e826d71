// The persistent sweep (k moves of every walker in one launch).  Compiled on
// its own without machine loop-invariant code motion: hoisting the two
// phases' constants and addresses out of the move loop would hold them in
// registers across the loop, past the 128 VGPRs of four waves per SIMD.
#include <hip/hip_ext.h>

#include "move_staged.h"
#include <algorithm>

namespace qmc {

// ---------------------------------------------------------------------------
// Persistent sweep: k consecutive proposals of every walker and the k - 1
// fused accepts between them in one launch, one workgroup per walker, for a
// run of moves with no refresh, change of spin or P rebuild inside (the host
// accepts the last proposal).  Each move does the streaming proposal's work
// and the staged accept's work unchanged, so the chain is bitwise that of the
// per-move launches.  In one launch a walker's accept (latency-bound) can
// overlap the streaming of the other walkers of its compute unit
// (bandwidth-bound), which separate launches serialise, and the launch gaps
// between the moves go.  (Spreading the workgroups' starts over up to one
// move's time with s_sleep measured no faster: they fall out of step by
// themselves.)  LDS: one layout of mcl staged rows for every move (at most
// 38 KiB: four workgroups per compute unit hold the 1024 walkers of a large
// batch at once).
// ---------------------------------------------------------------------------
constexpr size_t kSweepMaxLds = 37 * 1024;

// All S row blocks of walker wk's proposal in one workgroup, FP64 rows, two
// rows per wave and block (R = 8 = 2 x 4 waves): block sb's rows j0 + v and
// j0 + v + 4 go to wave v as in rows_body.  Every sum runs in rows_body's
// order and each block's partial ratio adds the waves' sums in wave order as
// block_partial does, so the new W line and the S partial ratios equal the
// proposal kernel's bit for bit.  With from_lds, psi(r') and the inverse
// line are taken from the LDS (psl, cvl: the set-up ran in the same
// workgroup); the new W line and the partial ratios also go to hand.
template <int NC>
__device__ void rows_stream_walker(const SysDev& s, const WalkDev& w, int wk, int e, int S, SweepHand* hand,
                                   const double* psl, const double* cvl, bool from_lds) {
  __shared__ double red2[kStageMaxSplits * 4];
  constexpr int VN = 2, STEP = 64 * VN, NW = 4, R = 2 * NW;
  const int tid = phase_tid(), lane = tid & 63, wave = tid >> 6;
  const bool up = e < s.nu;
  const int row0 = up ? s.nu : 0;
  const int nrow = s.nu;
  const double* Pw = (const double*)w.P + ((long)wk * s.N + row0) * s.Lp;
  auto rowp = [&](int j) -> const double* {
    return (up && j >= s.nd) ? (const double*)s.UphS + (long)(j - s.nd) * s.Lp : Pw + (long)j * s.Lp;
  };
  const double* cv = from_lds ? cvl : w.cvec + (long)wk * s.nu;
  double* wn_g = w.w_new + (long)wk * s.nu;
  const double* psi = from_lds ? psl : w.psi_new + (long)wk * s.Lp;
  double ps[NC][VN];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int i0 = c * STEP + lane * VN;
#pragma unroll
    for (int v = 0; v < VN; ++v) ps[c][v] = (i0 < s.Lp) ? psi[i0 + v] : 0.0;
  }
  for (int sb = 0; sb < S; ++sb) {
    const int ja = sb * R + wave, jb = ja + NW, j1 = min(sb * R + R, nrow);
    const bool oka = ja < j1, okb = jb < j1;   // uniform over the wave
    const double aa = oka ? cv[ja] : 0.0, ab = okb ? cv[jb] : 0.0;
    const double* pa = rowp(oka ? ja : 0);
    const double* pb = rowp(okb ? jb : 0);
    double2 va[NC], vb[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int i0 = c * STEP + lane * VN;
      va[c] = (oka && i0 < s.Lp) ? load16_nt<double2>(pa + i0) : double2{};
      vb[c] = (okb && i0 < s.Lp) ? load16_nt<double2>(pb + i0) : double2{};
    }
    double xa = 0.0, xb = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int v = 0; v < VN; ++v) {
        xa += vget(va[c], v) * ps[c][v];
        xb += vget(vb[c], v) * ps[c][v];
      }
    xa = wave_sum(xa);
    xb = wave_sum(xb);
    if (lane == 0) {
      double part = 0.0;
      if (oka) {
        wn_g[ja] = xa;
        hand->wn[ja] = xa;
        part += xa * aa;
        if (okb) {
          wn_g[jb] = xb;
          hand->wn[jb] = xb;
          part += xb * ab;
        }
      }
      red2[sb * NW + wave] = part;
    }
  }
  __syncthreads();
  if (tid < S) {
    double t = 0.0;
    for (int k = 0; k < NW; ++k) t += red2[tid * NW + k];
    w.rdet_part[(long)wk * S + tid] = t;
    hand->part[tid] = t;
  }
}

// Wave priorities.  Instruction issue on a SIMD favours the oldest wave, so
// with no hint the walkers dispatched first stream fastest and the launch waits
// for the last ones (over a 160-move sweep at 1024 walkers the walkers' busy
// time grew from 9.9 ms in the first quarter of the grid to 12.5 ms in the
// last).  The accept (a chain of dependent steps) runs at the upper two levels
// and the stream (bandwidth-bound) at the lower two; within each pair the level
// alternates with the move and the walker's quarter of the grid, so the four
// workgroups of a compute unit take turns (FP64 sweep 12.95 -> 12.77 ms,
// refined 4.86 -> 4.77 ms).
__device__ __forceinline__ void sweep_prio(int level) {
  switch (level & 3) {
    case 0: __builtin_amdgcn_s_setprio(0); break;
    case 1: __builtin_amdgcn_s_setprio(1); break;
    case 2: __builtin_amdgcn_s_setprio(2); break;
    default: __builtin_amdgcn_s_setprio(3); break;
  }
}

template <int QL, int NC, int IPB>
__global__ void __launch_bounds__(256, 4)   // four waves per SIMD: 128 VGPRs
sweep_segment_kernel(SysDev s, WalkDev w, int e0, int k, const double* __restrict__ disp,
                     const double* __restrict__ unif, int32_t* __restrict__ accept_count, int S, int FB, int since0,
                     int mcl, int vec_min) {
  extern __shared__ __align__(16) char lds[];
  __shared__ SweepHand hand;
  // the inverse line the set-up leaves in the vector area (after d and v0)
  const double* cvl = (const double*)(lds + stage_layout(s.nu, w.kb, mcl, vec_min).vec) + 2 * s.nu;
  const int N = s.N;
  const long Wk = w.Wk;
  const int quarter = (int)(((long)blockIdx.x * 4) / gridDim.x);
  for (int j = 0; j < k; ++j) {
    const int e = (e0 + j) % N;
    sweep_prio((j + quarter) & 1);
    // the walker index through an opaque move as well: the per-walker
    // addresses are recomputed in each phase (scalar work) instead of being
    // held in registers across the loop
    int wk;
    asm volatile("s_mov_b32 %0, %1" : "=s"(wk) : "s"(blockIdx.x));
    if constexpr (IPB > 0) screened_stream_walker<IPB, true>(s, w, wk, e, S, FB, lds, &hand, cvl, j > 0);
    else rows_stream_walker<NC>(s, w, wk, e, S, &hand, (const double*)lds, cvl, j > 0);
    if (j + 1 == k) break;
    __syncthreads();
    sweep_prio(2 + ((j + quarter) & 1));
    const int mc = min(since0 + j, mcl);
    accept_prep_staged_phase<double, QL, true>(s, w, wk, e, unif + (long)j * Wk, accept_count, S,
                                               (e0 + j + 1) % N, disp + (long)(j + 1) * Wk * 3, mc, mcl, lds, &hand,
                                               (size_t)vec_min);
    __syncthreads();
  }
}

// The launch shape of a sweep of proposals of e0's spin: false where the
// persistent kernel is not built for the system (the per-move launches run).
struct SweepShape {
  int S, QL, NC, IPB, FB;
  size_t lds_stream, vec_min;
};
static bool sweep_shape(const SysDev& s, const WalkDev& w, int e0, SweepShape& o) {
  if (s.store() != 0 || s.pairing || s.LJ > 0 || s.Lq > 0 || s.Lp > kFuseMaxLp || !w.wv || s.nu > kStageMaxN ||
      s.N > kStageMaxNe || s.n_nuc > kStageMaxNuc || s.L > 1024 || s.L < 1)
    return false;
  o.S = propose_splits(s);
  const int n = s.nu, kb = w.kb;
  const bool aligned = ((uintptr_t)w.wv | (uintptr_t)w.wd | (uintptr_t)w.wS) % 16 == 0 &&
                       ((long)kb * n) % 2 == 0 && kb % 2 == 0;
  if (o.S <= 0 || o.S > kStageMaxSplits || !aligned) return false;
  o.QL = (s.L + 255) / 256;
  o.IPB = o.FB = o.NC = 0;
  o.lds_stream = 0;
  if (s.screened()) {
    if (!w.PT || !w.muk || !screened_blk_config(s, w, e0, o.IPB, o.FB, o.lds_stream)) return false;
  } else {
    o.NC = (s.Lp + 127) / 128;
    if (s.prop_rows() != 8 || (o.NC != 2 * o.QL && o.NC != 2 * o.QL - 1)) return false;
  }
  // the hand-off region at the bottom of the LDS: the screened stream's kept
  // list and partial sums, or psi(r') for the row stream; the set-up's vectors
  // above it
  o.vec_min = s.screened() ? o.lds_stream : pad1k(sizeof(double) * (size_t)s.Lp);
  return stage_layout(n, kb, 0, o.vec_min).total <= kSweepMaxLds;
}

bool sweep_segment_ok(const SysDev& s, const WalkDev& w, int e0) {
  SweepShape o;
  return sweep_shape(s, w, e0, o);
}

hipError_t launch_sweep_segment(const SysDev& s, const WalkDev& w, int e0, int k, const double* disp,
                                const double* unif, int32_t* accept_count, int since0, hipStream_t st,
                                hipEvent_t ev_start, hipEvent_t ev_stop) {
  if (k < 2 || since0 < 0) return hipErrorInvalidValue;
  SweepShape o;
  if (!sweep_shape(s, w, e0, o)) return hipErrorNotSupported;
  const int S = o.S, QL = o.QL, NC = o.NC, IPB = o.IPB, FB = o.FB;
  const int n = s.nu, kb = w.kb;
  // staged rows: the most any move of the run can hold that the LDS allows
  int mcl = std::max(0, std::min(since0 + k - 2, kb - 1));
  while (mcl > 0 && stage_layout(n, kb, mcl, o.vec_min).total > kSweepMaxLds) --mcl;
  const size_t lds = stage_layout(n, kb, mcl, o.vec_min).total;   // >= vec_min >= the stream's region
  const dim3 grid(w.Wk), blk(256);
#define QMC_SWEEP(Q, C, I)                                                                                      hipExtLaunchKernelGGL((sweep_segment_kernel<Q, C, I>), grid, blk, lds, st, ev_start, ev_stop, 0, s, w, e0, k,                         disp, unif, accept_count, S, FB, since0, mcl, (int)o.vec_min)
#define QMC_SWEEP_IPB(Q)                                                                switch (IPB) {                                                                          case 1: QMC_SWEEP(Q, 0, 1); break; case 2: QMC_SWEEP(Q, 0, 2); break;                 case 3: QMC_SWEEP(Q, 0, 3); break; case 4: QMC_SWEEP(Q, 0, 4); break;                 case 5: QMC_SWEEP(Q, 0, 5); break; case 6: QMC_SWEEP(Q, 0, 6); break;                 case 7: QMC_SWEEP(Q, 0, 7); break; default: QMC_SWEEP(Q, 0, 8); break;             }
  if (IPB > 0) {
    switch (QL) {
      case 1: QMC_SWEEP_IPB(1) break;
      case 2: QMC_SWEEP_IPB(2) break;
      case 3: QMC_SWEEP_IPB(3) break;
      default: QMC_SWEEP_IPB(4) break;
    }
  } else {
    switch (NC) {
      case 1: QMC_SWEEP(1, 1, 0); break; case 2: QMC_SWEEP(1, 2, 0); break;
      case 3: QMC_SWEEP(2, 3, 0); break; case 4: QMC_SWEEP(2, 4, 0); break;
      case 5: QMC_SWEEP(3, 5, 0); break; case 6: QMC_SWEEP(3, 6, 0); break;
      case 7: QMC_SWEEP(4, 7, 0); break; default: QMC_SWEEP(4, 8, 0); break;
    }
  }
#undef QMC_SWEEP_IPB
#undef QMC_SWEEP
  return hipGetLastError();
}

}  // namespace qmc
