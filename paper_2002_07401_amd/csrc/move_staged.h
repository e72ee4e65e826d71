// Device code shared by the move kernels (move.hip) and the persistent sweep
// (sweep.hip): the screened proposal's streaming phase and the Metropolis
// accept fused with the next proposal's set-up, staged through LDS.
#pragma once
#include "move_dev.h"

namespace qmc {

constexpr int kStageQL = (kFuseMaxLp + 255) / 256;   // per-thread slots over Lp <= kFuseMaxLp
__host__ __device__ inline size_t pad1k(size_t b) { return (b + 1023) & ~(size_t)1023; }
typedef double dbl2 __attribute__((ext_vector_type(2)));

// threadIdx.x through an opaque move: values computed from it stay inside the
// phase that computes them.  In the persistent sweep's loop the compiler would
// otherwise hoist each phase's per-lane addresses and loads out of the loop and
// keep them live across the other phase, past 128 VGPRs.
__device__ __forceinline__ int phase_tid() {
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  return (int)threadIdx.x + z;
}

// Blocked form of the same sum, for an even row count n: the kept functions
// are taken FB at a time (FB n a multiple of 128, IPB = FB n / 128 <= 8), and
// a wave reads a block's FB columns (FB n doubles) with IPB 16-byte loads of
// all 64 lanes: lane l of load i holds the two rows j, j + 1 of function f
// with 2 (64 i + l) = f n + j, fixed over the blocks.  The kept list and the
// inverse line come first (one round), then every wave issues about eight
// loads at once (8 / IPB blocks), some 32 KiB in flight per walker.  The
// per-lane sums go to LDS and row j adds its FB x 4 partial sums in a fixed
// order (waves outer, functions inner).
constexpr int kStageMaxN = 128;    // n <= 128 (one W entry per thread)
constexpr int kStageMaxNe = 256;   // electrons
constexpr int kStageMaxNuc = 256;  // nuclei (one per thread)
constexpr int kStageMaxSplits = (kStageMaxN + kPropRowsMin - 1) / kPropRowsMin;   // partial ratios
constexpr size_t kStageMaxLds = 63 * 1024;   // dynamic LDS (the static arrays take the rest of 64 KiB)

struct StageLayout {
  size_t V, D, S, vec, total;   // byte offsets of the regions and the size
};
// vec_min: the vector area starts at vec_min or later (the persistent sweep
// keeps its hand-off arrays below it)
__host__ __device__ inline StageLayout stage_layout(int n, int kb, int mc, size_t vec_min = 0) {
  StageLayout o;
  o.V = 0;
  o.D = o.V + pad1k(sizeof(double) * (size_t)(mc + 1) * n);
  o.S = o.D + pad1k(sizeof(double) * (size_t)(mc + 1) * n);
  o.vec = o.S + pad1k(sizeof(double) * (size_t)(mc + 1) * kb);
  if (o.vec < vec_min) o.vec = vec_min;
  o.total = o.vec + sizeof(double) * (3 * (size_t)n + 5 * (size_t)kb);
  return o;
}

// The persistent sweep hands values from one phase of a move to the next
// through LDS rather than global memory (a load of a value the workgroup has
// just stored waits for the store): the new W line and the partial ratios of a
// proposal (to the accept), the kept count of a screened set-up (to the next
// proposal; the kept list itself and psi(r') go to the bottom of the dynamic
// LDS, the inverse line stays in the vector area).
struct SweepHand {
  double wn[kStageMaxN];
  double part[kStageMaxSplits];
  int cnt;
};


// HAND (persistent sweep): with from_lds the kept list is already at the
// bottom of lds, its count in hand->cnt and the inverse line in cvl (the set-up
// ran in the same workgroup); the new W line and the partial ratios also go to
// hand.
template <int IPB, bool HAND = false>
__device__ void screened_stream_walker(const SysDev& s, const WalkDev& w, int wk, int e, int S, int FB, char* lds,
                                       SweepHand* hand = nullptr, const double* cvl = nullptr,
                                       bool from_lds = false) {
  __shared__ double red[8];
  const int tid = phase_tid(), lane = tid & 63, wave = tid >> 6;
  const bool up = e < s.nu;
  const int i0 = up ? s.nu : 0;
  const int n = up ? s.nd + s.nk : s.nu;   // = n_up either way (unpaired orbitals after the down rows)
  const int Lp = s.Lp, ld = s.pt_ld();
  const double* base = w.PT + (long)wk * Lp * ld + i0;
  int* lmu = (int*)lds;
  double* lv = (double*)(lds + pad1k(sizeof(int) * (size_t)Lp));
  dbl2* part = (dbl2*)((char*)lv + pad1k(sizeof(double) * (size_t)Lp));
  int cnt;
  double cj;
  if (HAND && from_lds) {
    cnt = hand->cnt;
    cj = cvl[tid < n ? tid : 0];
  } else {
    // the kept list (the whole Lp-long arrays: no wait on the count), c
    const int* mk = w.muk + (long)wk * Lp;
    const double* pk = w.psk + (long)wk * Lp;
    int xm[kStageQL];
    double xv[kStageQL];
#pragma unroll
    for (int k = 0; k < kStageQL; ++k) {
      const int q = tid + 256 * k, qc = q < Lp ? q : 0;
      xm[k] = mk[qc];
      xv[k] = pk[qc];
    }
    cnt = w.nkeep[wk];
    cj = w.cvec[(long)wk * s.nu + (tid < n ? tid : 0)];
#pragma unroll
    for (int k = 0; k < kStageQL; ++k) {
      const int q = tid + 256 * k;
      if (q < Lp) { lmu[q] = xm[k]; lv[q] = xv[k]; }
    }
  }
  __syncthreads();
  // this lane's (function, row) of each of its IPB loads
  int fi[IPB], ji[IPB];
#pragma unroll
  for (int i = 0; i < IPB; ++i) {
    const int el = 2 * (64 * i + lane);
    fi[i] = el / n;
    ji[i] = el - fi[i] * n;
  }
  dbl2 acc[IPB];
#pragma unroll
  for (int i = 0; i < IPB; ++i) acc[i] = dbl2{0.0, 0.0};
  const int nblk = (cnt + FB - 1) / FB;
  constexpr int UB = 8 / IPB > 1 ? 8 / IPB : 1;   // blocks per wave in flight (8 loads)
  for (int b0 = wave; b0 < nblk; b0 += 4 * UB) {
    dbl2 x[UB][IPB];
    double vv[UB][IPB];
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int i = 0; i < IPB; ++i) {
        const int kk = (b0 + 4 * u) * FB + fi[i];
        const bool ok = kk < cnt;
        const int mu = lmu[ok ? kk : 0];
        vv[u][i] = ok ? lv[kk] : 0.0;
        x[u][i] = __builtin_nontemporal_load((const dbl2*)(base + (long)mu * ld + ji[i]));
      }
#pragma unroll
    for (int u = 0; u < UB; ++u)
#pragma unroll
      for (int i = 0; i < IPB; ++i) {
        acc[i].x += vv[u][i] * x[u][i].x;
        acc[i].y += vv[u][i] * x[u][i].y;
      }
  }
#pragma unroll
  for (int i = 0; i < IPB; ++i) part[wave * 64 * IPB + 64 * i + lane] = acc[i];
  __syncthreads();
  const double* pd = (const double*)part;
  double* wn = w.w_new + (long)wk * s.nu;
  double rp = 0.0;
  if (tid < n) {
    double t = 0.0;
    for (int v = 0; v < 4; ++v)
      for (int f = 0; f < FB; ++f) t += pd[v * 128 * IPB + f * n + tid];
    wn[tid] = t;
    if (HAND) hand->wn[tid] = t;
    rp = t * cj;
  }
  const double R = block_sum_mv(rp, red);
  for (int q = tid; q < S; q += blockDim.x) {
    w.rdet_part[(long)wk * S + q] = q == 0 ? R : 0.0;
    if (HAND) hand->part[q] = q == 0 ? R : 0.0;
  }
}

// The plain screened stream of one walker (any row count), one workgroup of
// 256 threads: wave v takes kept functions v, v + 4, ..., four at a time, lane
// l the rows l, l + 64, ...; the waves' partial rows are added in a fixed order
// through LDS, then the ratio sum_j w'_j c_j, which goes to the first of the
// walker's S partial slots (the others are zeroed).
template <int NB>
__device__ void screened_rows_walker(const SysDev& s, const WalkDev& w, int wk, int e, int S) {
  __shared__ double part[4][64 * NB];
  __shared__ double red[8];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool up = e < s.nu;
  const int i0 = up ? s.nu : 0;
  const int n = up ? s.nd + s.nk : s.nu;   // = n_up either way
  const int ld = s.pt_ld();
  const double* base = w.PT + (long)wk * s.Lp * ld + i0;
  const int cnt = w.nkeep[wk];
  const int* mk = w.muk + (long)wk * s.Lp;
  const double* pk = w.psk + (long)wk * s.Lp;
  double acc[NB];
#pragma unroll
  for (int b = 0; b < NB; ++b) acc[b] = 0.0;
  int k = wave;
  for (; k + 12 < cnt; k += 16) {   // four functions in flight per wave
    int mu[4];
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) { mu[q] = mk[k + 4 * q]; v[q] = pk[k + 4 * q]; }
    double x[4][NB];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int j = lane + 64 * b;
        x[q][b] = j < n ? __builtin_nontemporal_load(base + (long)mu[q] * ld + j) : 0.0;
      }
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int b = 0; b < NB; ++b) acc[b] += v[q] * x[q][b];
  }
  for (; k < cnt; k += 4) {
    const int mu = mk[k];
    const double v = pk[k];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int j = lane + 64 * b;
      if (j < n) acc[b] += v * base[(long)mu * ld + j];
    }
  }
#pragma unroll
  for (int b = 0; b < NB; ++b) part[wave][lane + 64 * b] = acc[b];
  __syncthreads();
  const double* cv = w.cvec + (long)wk * s.nu;
  double* wn = w.w_new + (long)wk * s.nu;
  double rp = 0.0;
  for (int j = tid; j < n; j += blockDim.x) {
    const double x = ((part[0][j] + part[1][j]) + part[2][j]) + part[3][j];
    wn[j] = x;
    rp += x * cv[j];
  }
  const double R = block_sum_mv(rp, red);
  for (int q = tid; q < S; q += blockDim.x) w.rdet_part[(long)wk * S + q] = q == 0 ? R : 0.0;
}

// The blocked screened stream for proposals of e: n even, FB = 128 /
// gcd(n, 128) functions per block, IPB = FB n / 128 loads per lane and block,
// at most 8; n <= 256 (one row per thread in the final sums), Lp <=
// kFuseMaxLp (the kept list in LDS).  False: the plain screened kernel.
__host__ __device__ inline bool screened_blk_config(const SysDev& s, const WalkDev& w, int e, int& IPB, int& FB,
                                                   size_t& lds) {
  const int n = e < s.nu ? s.nd + s.nk : s.nu;
  int g = 128;
  while (n % g) g >>= 1;
  FB = 128 / g;
  IPB = FB * n / 128;
  lds = pad1k(sizeof(int) * (size_t)s.Lp) + pad1k(sizeof(double) * (size_t)s.Lp) +
        sizeof(dbl2) * 4 * 64 * (size_t)IPB;
  return n % 2 == 0 && n <= 256 && IPB >= 1 && IPB <= 8 && s.Lp <= kFuseMaxLp && (uintptr_t)w.PT % 16 == 0 &&
         s.pt_ld() % 2 == 0 && (e < s.nu ? s.nu : 0) % 2 == 0;
}

// ---------------------------------------------------------------------------
// Metropolis accept of e fused with the set-up of e2, staged through LDS.
// The same arithmetic in the same order as accept_prep_body (so chains are
// bitwise those of the unstaged kernel and of the multi-system launches), but
// every input the workgroup reads is requested at once at the start: the
// delayed-update buffers V and D (rows below mc), S^{-1} and the positions go
// global -> LDS by direct copies (no registers held), while the basis records
// of psi(r'), the nuclei of the one-body Jastrow, the new and old W line, v0
// and z of the pending proposal, A0's line of e2, psi(r') of the pending
// proposal and the column maxima of the screened proposals go to registers.
// psi(r') of e2 is computed while the copies are in flight.  The unstaged
// kernel walks a chain of some fifteen dependent global round trips per
// walker; this one, one.
// mc bounds the buffered moves: at the accept of an attempt, wm <= the
// attempts since the last refresh (both restart together, wm grows by at
// most one per attempt), which the host passes.  A walker with more (not
// reachable through the move calls) reads the buffers from global memory.
// LDS: V, D [(mc+1) n], S^{-1} [(mc+1) kb], r [3 N] (each padded to 1 KiB,
// the copy granule), psi(r') of e2 [Lp], three n-vectors, five kb-vectors.
// ---------------------------------------------------------------------------
// bytes (a multiple of 8) from global src to LDS dst in 1 KiB granules, 16
// bytes per lane (global_load_lds): granule j by wave j mod the wave count.
// Lanes past the end re-read src's first 16 bytes into dst's padding.
__device__ __forceinline__ void lds_copy_async(void* dst, const void* src, int bytes) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const char* s = (const char*)src;
  char* d = (char*)dst;
  const int nch = (bytes + 1023) >> 10;
  for (int j = wave; j < nch; j += nw) {
    const int off = (j << 10) + 16 * lane;
    const char* p = off < bytes ? s + off : s;
    __builtin_amdgcn_global_load_lds((const __attribute__((address_space(1))) void*)p,
                                     (__attribute__((address_space(3))) void*)(d + (j << 10)), 16, 0, 0);
  }
}

// Prefetched per-thread inputs of the staged kernel.
struct StagePre {
  double4 bf[kStageQL];   // basis records of mu = tid + 256 q
  int bk[kStageQL];
  double xp[kStageQL];    // psi(r') of the pending proposal (the accepted row)
  double xc[kStageQL];    // column maxima of the rows e2's proposal streams (screened)
  double sv[kStageQL];    // psi(r') of e2 (computed)
  double nx, ny, nz, nZ, nb;   // nucleus tid (one-body Jastrow)
  double ex, ey, ez;           // electron tid's position (two-body Jastrow)
  double wn, Wo, v0, a0, z;    // new W entry, old one, v0, A0's line of e2, z (thread = index)
};

// jastrow_one for N <= the block size: nucleus tid's record and electron
// tid's position (xj, yj, zj) in registers, the two-body parameters (j2p, the
// eight of s.j2d) in LDS.
__device__ __forceinline__ double jastrow_staged(const SysDev& s, int e, double px, double py, double pz,
                                                 const StagePre& q, double xj, double yj, double zj,
                                                 const double* j2p) {
  double val = 0.0;
  const int tid = threadIdx.x;
  if (s.j1_form) {
    if (tid < s.n_nuc) {
      const double dx = px - q.nx, dy = py - q.ny, dz = pz - q.nz;
      const double ria = sqrt(dx * dx + dy * dy + dz * dz);
      double f, f1, f2;
      j1_radial(s.j1_form, q.nZ, q.nb, ria, f, f1, f2);
      val += f;
    }
  }
  if (s.j2_form) {
    const bool up_e = e < s.nu;
    const int j = tid;
    if (j < s.N && j != e) {
      const double dx = px - xj, dy = py - yj, dz = pz - zj;
      const double rij = sqrt(dx * dx + dy * dy + dz * dz);
      double v, v1, v2;
      j2_radial(s.j2_form, j2p, up_e == (j < s.nu), rij, v, v1, v2);
      val += v;
    }
  }
  return val;
}

template <typename T, bool STAGED, int QL, bool HAND = false>
__device__ void accept_prep_staged_body(const SysDev& s, const WalkDev& w, int wk, int e, double u,
                                        int32_t* __restrict__ cnt, int cnt0, int S, int e2, double px, double py,
                                        double pz, double R, double dJ, int m, int mc, char* lds, const StagePre& q,
                                        const double* j2p, double la, double sg, double jv, double rx, double ry,
                                        double rz, double ox, double oy, double oz, SweepHand* hand = nullptr,
                                        size_t vec_min = 0) {
  __shared__ double red[16];
  __shared__ double gam_s;
  __shared__ int wcnt[QL][4];
  const int tid = phase_tid(), lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
  const int n = s.nu, kb = w.kb, N = s.N, L = s.L, Lp = s.Lp;
  const bool up = e < n;
  const int ie = up ? e : e - n;
  const StageLayout ly = stage_layout(n, kb, mc, vec_min);
  double* Vl = (double*)(lds + ly.V);
  double* Dl = (double*)(lds + ly.D);
  double* Sl = (double*)(lds + ly.S);
  double* sd = (double*)(lds + ly.vec);
  double* sv0 = sd + n;
  double* cvl = sv0 + n;
  double* zo = cvl + n;
  double* sr = zo + kb;
  double* sy = sr + kb;
  double* st = sy + kb;
  double* sz = st + kb;
  double* Vg = w.wv + (long)wk * kb * n;
  double* Dg = w.wd + (long)wk * kb * n;
  double* Sg = w.wS + (long)wk * kb * kb;
  const double* Vr = STAGED ? Vl : Vg;
  const double* Dr = STAGED ? Dl : Dg;
  double* Sr = STAGED ? Sl : Sg;

  // the accept of e (accept_body, Metropolis mode)
  const double ratio = R * exp(dJ);
  const bool acc = m < kb && u < ratio * ratio;
  if (tid == 0) {
    w.rdet[wk] = R;
    w.ratio[wk] = ratio;
    w.acc[wk] = acc ? 1 : 0;
  }
  if (acc) {
    double p0 = 0.0;
    if (tid < n) {
      const double d = q.wn - q.Wo;
      sd[tid] = d;
      p0 += d * q.v0;
      Dg[(long)m * n + tid] = d;
      Vg[(long)m * n + tid] = q.v0;
      if (STAGED) { Dl[(long)m * n + tid] = d; Vl[(long)m * n + tid] = q.v0; }
    }
    p0 = wave_sum(p0);
    if (lane == 0) red[wave] = p0;
    __syncthreads();
    rows_dot_lds(Vr, n, m, n, sd, sr);           // r_i = delta . v_i
    __syncthreads();
    if (tid == 0) {
      double dv = 0.0;
      for (int k = 0; k < nw; ++k) dv += red[k];
      double rzs = 0.0;
      for (int i = 0; i < m; ++i) rzs += sr[i] * zo[i];
      gam_s = 1.0 + dv - rzs;
    }
    for (int k = tid; k < m; k += blockDim.x) {
      double y = 0.0;
      for (int i = 0; i < m; ++i) y += Sr[i * kb + k] * sr[i];
      sy[k] = y;
    }
    __syncthreads();
    const double ig = 1.0 / gam_s;
    for (int idx = tid; idx < (m + 1) * (m + 1); idx += blockDim.x) {
      const int i = idx / (m + 1), k = idx % (m + 1);
      double v;
      if (i < m && k < m) v = Sr[i * kb + k] + zo[i] * sy[k] * ig;
      else if (i < m) v = -zo[i] * ig;
      else if (k < m) v = -sy[k] * ig;
      else v = ig;
      Sr[i * kb + k] = v;
      if (STAGED) Sg[i * kb + k] = v;
    }
    if (tid < n) {
      double* Ww = w.W + (long)wk * n * n;
      if (up) Ww[(long)ie * n + tid] = q.wn;
      else Ww[(long)tid * n + ie] = q.wn;
    }
    T* prow = (T*)w.phi + ((long)wk * N + e) * Lp;
#pragma unroll
    for (int k = 0; k < QL; ++k) {
      const int mu = tid + 256 * k;
      if (mu < L) prow[mu] = (T)q.xp[k];
    }
    if (tid == 0) {
      w.wm[wk] = m + 1;
      double* re = w.r + ((long)wk * N + e) * 3;
      re[0] = rx; re[1] = ry; re[2] = rz;
      w.logabs[wk] = la + (log(fabs(R)) + dJ);
      if (R < 0.0) w.sign[wk] = -sg;
      w.J[wk] = jv + dJ;
      if (cnt) cnt[0] = cnt0 + 1;
    }
  }
  __syncthreads();

  // the set-up of e2: psi(r'), r', the Jastrow change (with e at its new
  // position when accepted)
  double* psi = w.psi_new + (long)wk * Lp;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = tid + 256 * k;
    if (mu < Lp) psi[mu] = mu < L ? q.sv[k] : 0.0;
  }
  if (tid < 3) w.r_new[3 * wk + tid] = tid == 0 ? px : (tid == 1 ? py : pz);
  const bool me = acc && tid == e;
  const double xj = me ? rx : q.ex, yj = me ? ry : q.ey, zj = me ? rz : q.ez;
  const double jn = jastrow_staged(s, e2, px, py, pz, q, xj, yj, zj, j2p);
  const double jo = jastrow_staged(s, e2, ox, oy, oz, q, xj, yj, zj, j2p);
  const double dJ2 = block_sum_mv(jn - jo, red);
  if (tid == 0) w.dJ[wk] = dJ2;

  // the current inverse's line of e2 (inverse_line_body)
  double* v0g = w.v0 + (long)wk * n;
  double* cv = w.cvec + (long)wk * n;
  if (tid < n) v0g[tid] = sv0[tid];
  const int m2 = acc ? m + 1 : m;
  if (m2 == 0) {
    if (tid < n) { cv[tid] = sv0[tid]; cvl[tid] = sv0[tid]; }
  } else {
    double* tz = w.tz + (long)wk * 2 * kb;
    rows_dot_lds(Dr, n, m2, n, sv0, st);        // t = D^T v0
    __syncthreads();
    rows_dot_lds(Sr, kb, m2, m2, st, sz);       // z = S^{-1} t
    __syncthreads();
    for (int i = tid; i < m2; i += blockDim.x) {
      tz[i] = st[i];
      tz[kb + i] = sz[i];
    }
    if (tid < n) {
      double c = sv0[tid];
      for (int i = 0; i < m2; ++i) c -= sz[i] * Vr[(long)i * n + tid];
      cv[tid] = c;
      cvl[tid] = c;
    }
  }
  if (!s.screened()) {
    if (HAND) {
      // psi(r') of e2 for the next proposal's stream, at the bottom of the LDS
      // (the staged rows there are no longer read)
      __syncthreads();
      double* psl = (double*)lds;
#pragma unroll
      for (int k = 0; k < QL; ++k) {
        const int mu = tid + 256 * k;
        if (mu < Lp) psl[mu] = mu < L ? q.sv[k] : 0.0;
      }
    }
    return;
  }

  // screened proposals of e2 (screen_list_body)
  __syncthreads();
  double c1 = 0.0;
  for (int j = tid; j < n; j += blockDim.x) c1 += fabs(cvl[j]);
  c1 = block_sum_mv(c1, red);
  const double thr = (c1 > 0.0) ? kScreenTol / ((double)L * c1) : 0.0;
  int* mk = w.muk + (long)wk * Lp;
  double* pk = w.psk + (long)wk * Lp;
  // the kept functions in increasing mu: every slot's ballot first, one
  // barrier, then each kept lane's place from the counts before it
  unsigned long long bal[QL];
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = 256 * k + tid;
    const bool keep = mu < L && fabs(q.sv[k]) * q.xc[k] > thr;
    bal[k] = __ballot(keep);
    if (lane == 0) wcnt[k][wave] = __popcll(bal[k]);
  }
  __syncthreads();
  int off = 0;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    int before = off;   // kept in earlier slots, then earlier waves of this slot
    for (int k2 = 0; k2 < wave; ++k2) before += wcnt[k][k2];
    if ((bal[k] >> lane) & 1ull) {
      const int at = before + __popcll(bal[k] & ((1ull << lane) - 1ull));
      if (HAND) {   // the list where the screened stream keeps it (the staged rows are no longer read)
        ((int*)lds)[at] = 256 * k + tid;
        ((double*)(lds + pad1k(sizeof(int) * (size_t)Lp)))[at] = q.sv[k];
      } else {
        mk[at] = 256 * k + tid;
        pk[at] = q.sv[k];
      }
    }
    for (int k2 = 0; k2 < nw; ++k2) off += wcnt[k][k2];
  }
  if (tid == 0) {
    w.nkeep[wk] = off;
    if (HAND) hand->cnt = off;
  }
}

// One walker's fused accept and set-up (the staged kernel's work for walker
// wk): rows below mc of V and D are staged; the LDS regions are laid out for
// mcl >= mc rows (the persistent sweep keeps one layout for all its moves).
template <typename T, int QL, bool HAND = false>
__device__ void accept_prep_staged_phase(const SysDev& s, const WalkDev& w, int wk, int e,
                                         const double* __restrict__ unif, int32_t* __restrict__ accept_count,
                                         int S, int e2, const double* __restrict__ disp2, int mc, int mcl,
                                         char* lds, SweepHand* hand = nullptr, size_t vec_min = 0) {
  __shared__ double scal[kStageMaxSplits + 22];
  __shared__ int ints_s[2];
  const int tid = phase_tid();
  const int n = s.nu, kb = w.kb, N = s.N, L = s.L, Lp = s.Lp;
  const bool up = e < n, up2 = e2 < n;
  const int ie = up ? e : e - n, ie2 = up2 ? e2 : e2 - n;
  const StageLayout ly = stage_layout(n, kb, mcl, vec_min);
  // bulk copies first
  lds_copy_async(lds + ly.V, w.wv + (long)wk * kb * n, 8 * mc * n);
  lds_copy_async(lds + ly.D, w.wd + (long)wk * kb * n, 8 * mc * n);
  lds_copy_async(lds + ly.S, w.wS + (long)wk * kb * kb, 8 * mc * kb);
  // per-thread loads, every address valid (indices past the ends read element 0)
  StagePre q;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = tid + 256 * k, mc0 = mu < L ? mu : 0;
    q.bf[k] = s.bfn[mc0];
    q.bk[k] = s.kind[mc0];
  }
  {
    const int a = tid < s.n_nuc ? tid : 0;
    q.nx = s.R[3 * a]; q.ny = s.R[3 * a + 1]; q.nz = s.R[3 * a + 2];
    q.nZ = s.Z[a];
    q.nb = s.j1_b[a];
    const double* rj = w.r + ((long)wk * N + (tid < N ? tid : 0)) * 3;
    q.ex = rj[0]; q.ey = rj[1]; q.ez = rj[2];
  }
  {
    const int j = tid < n ? tid : 0;
    const double* Ww = w.W + (long)wk * n * n;
    const double* A0 = w.A + (long)wk * n * n;
    q.wn = HAND ? hand->wn[j] : w.w_new[(long)wk * n + j];
    q.Wo = up ? Ww[(long)ie * n + j] : Ww[(long)j * n + ie];
    q.v0 = w.v0[(long)wk * n + j];
    q.a0 = up2 ? A0[(long)j * n + ie2] : A0[(long)ie2 * n + j];
    q.z = w.tz[(long)wk * 2 * kb + kb + (tid < kb ? tid : 0)];
  }
  const double* pn = w.psi_new + (long)wk * Lp;
  const double* cm = s.screened() ? w.cmax + ((long)wk * 2 + (up2 ? 1 : 0)) * Lp : pn;
#pragma unroll
  for (int k = 0; k < QL; ++k) {
    const int mu = tid + 256 * k, mc0 = mu < L ? mu : 0;
    q.xp[k] = pn[mc0];
    q.xc[k] = cm[mc0];
  }
  // the walker's scalars, one per thread, through LDS: the S partial ratios
  // (threads 0..S-1), then dJ, log|Psi|, sign, J, u, the displacement of e2,
  // r' of e and r of e2 and the eight two-body parameters (wave 1), the
  // buffered-move and accept counts.  Loads first, unconditionally (every
  // address valid), stores after.
  const double pv = HAND ? hand->part[tid < S ? tid : 0] : w.rdet_part[(long)wk * S + (tid < S ? tid : 0)];
  const int t2 = tid - 64;
  const double* sp;
  switch (t2) {
    case 0: sp = w.dJ + wk; break;
    case 1: sp = w.logabs + wk; break;
    case 2: sp = w.sign + wk; break;
    case 3: sp = w.J + wk; break;
    case 4: sp = unif + wk; break;
    case 5: case 6: case 7: sp = disp2 + 3 * (long)wk + (t2 - 5); break;
    case 8: case 9: case 10: sp = w.r_new + 3 * (long)wk + (t2 - 8); break;
    case 11: case 12: case 13: sp = w.r + ((long)wk * N + e2) * 3 + (t2 - 11); break;
    case 14: case 15: case 16: case 17: case 18: case 19: case 20: case 21: sp = s.j2d + (t2 - 14); break;
    default: sp = w.dJ + wk; break;
  }
  const double sv_ = *sp;
  const int mv = w.wm[wk];
  const int cv_ = accept_count ? accept_count[wk] : 0;
  if (tid < S) scal[tid] = pv;
  if (t2 >= 0 && t2 < 22) scal[kStageMaxSplits + t2] = sv_;
  if (tid == 128) { ints_s[0] = mv; ints_s[1] = cv_; }
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's copies landed
  __syncthreads();
  double R = 0.0;
  for (int k = 0; k < S; ++k) R += scal[k];
  const double* sc = scal + kStageMaxSplits;
  const double dJ = sc[0], la = sc[1], sg = sc[2], jv = sc[3], u = sc[4];
  const double rx = sc[8], ry = sc[9], rz = sc[10];
  const double px = sc[11] + sc[5], py = sc[12] + sc[6], pz = sc[13] + sc[7];
  const int m = ints_s[0];
  double* sv0 = (double*)(lds + ly.vec) + n;
  double* zo = sv0 + 2 * n;
  // psi(r') of e2
#pragma unroll
  for (int k = 0; k < QL; ++k) q.sv[k] = basis_value_rec(q.bf[k], q.bk[k], px, py, pz);
  if (tid < n) sv0[tid] = q.a0;
  if (tid < kb) zo[tid] = q.z;
  __syncthreads();
  int32_t* cnt = accept_count ? accept_count + wk : nullptr;
  if (m <= mc)
    accept_prep_staged_body<T, true, QL, HAND>(s, w, wk, e, u, cnt, ints_s[1], S, e2, px, py, pz, R, dJ, m, mcl,
                                               lds, q, sc + 14, la, sg, jv, rx, ry, rz, sc[11], sc[12], sc[13],
                                               hand, vec_min);
  else
    accept_prep_staged_body<T, false, QL, HAND>(s, w, wk, e, u, cnt, ints_s[1], S, e2, px, py, pz, R, dJ, m, mcl,
                                                lds, q, sc + 14, la, sg, jv, rx, ry, rz, sc[11], sc[12], sc[13],
                                                hand, vec_min);
}

}  // namespace qmc
