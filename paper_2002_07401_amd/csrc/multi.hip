// Several systems of uneven electron count moved together: each phase of a
// Metropolis step (proposal set-up, streaming rows, accept/update) is one
// persistent launch whose workgroups walk a table of (system, walker[, row
// chunk]) work items ordered by decreasing cost.  The per-item work is the same
// device code as the one-system kernels (move_dev.h), so every member evolves
// exactly as it would alone.  Random numbers come from Philox4x32-10 (counter =
// the member's move count, the walker and the member; key = the seed), which
// lets a captured graph of many steps be replayed without host involvement.
#include "move_staged.h"

namespace qmc {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Metropolis draws
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k.x += 0x9E3779B9u; k.y += 0xBB67AE85u; }
    const unsigned long long p0 = (unsigned long long)0xD2511F53u * c.x;
    const unsigned long long p1 = (unsigned long long)0xCD9E8D57u * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
  }
  return c;
}

__device__ __forceinline__ double words_to_uniform(uint32_t hi, uint32_t lo) {
  const unsigned long long v = (((unsigned long long)hi << 32) | lo) >> 11;
  return (double)v * 0x1.0p-53;
}

// Displacement (N(0, sigma^2) per component, Box-Muller) and acceptance uniform
// of one walker at one step.
__device__ void metropolis_draw(unsigned long long seed, int member, int walker, unsigned long long step,
                                double sigma, double disp[3], double* u) {
  const uint2 key = make_uint2((uint32_t)seed, (uint32_t)(seed >> 32));
  uint4 o[3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
    o[b] = philox4x32_10(make_uint4((uint32_t)step, (uint32_t)(step >> 32), (uint32_t)walker,
                                    ((uint32_t)member << 16) | (uint32_t)b), key);
  const double u0 = words_to_uniform(o[0].x, o[0].y), v0 = words_to_uniform(o[0].z, o[0].w);
  const double u1 = words_to_uniform(o[1].x, o[1].y), v1 = words_to_uniform(o[1].z, o[1].w);
  const double r0 = sqrt(-2.0 * log1p(-u0)), r1 = sqrt(-2.0 * log1p(-u1));
  const double two_pi = 6.283185307179586476925286766559;
  disp[0] = sigma * r0 * cos(two_pi * v0);
  disp[1] = sigma * r0 * sin(two_pi * v0);
  disp[2] = sigma * r1 * cos(two_pi * v1);
  *u = words_to_uniform(o[2].x, o[2].y);
}

// Per-member draws for tests: disp [Wk][3], unif [Wk] at a given step.
__global__ void philox_draws_kernel(unsigned long long seed, int member, int Wk, unsigned long long step,
                                    double sigma, double* __restrict__ disp, double* __restrict__ unif) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= Wk) return;
  double d[3], u;
  metropolis_draw(seed, member, w, step, sigma, d, &u);
  disp[3 * w] = d[0]; disp[3 * w + 1] = d[1]; disp[3 * w + 2] = d[2];
  unif[w] = u;
}

hipError_t launch_philox_draws(unsigned long long seed, int member, int Wk, unsigned long long step, double sigma,
                               double* disp, double* unif, hipStream_t st) {
  hipLaunchKernelGGL(philox_draws_kernel, dim3((Wk + 255) / 256), dim3(256), 0, st, seed, member, Wk, step, sigma,
                     disp, unif);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// persistent phase kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ void member_draw(const MultiArgs& a, int k, int w, int Wk, double d[3], double* u) {
  if (a.disp) {
    const double* p = a.disp[k] + ((long)a.t * Wk + w) * 3;
    d[0] = p[0]; d[1] = p[1]; d[2] = p[2];
    *u = a.unif[k][(long)a.t * Wk + w];
  } else {
    metropolis_draw(a.seed, k, w, (unsigned long long)a.steps[k], a.sigma, d, u);
  }
}

__global__ void __launch_bounds__(256) multi_prep_kernel(MultiArgs a, const int2* __restrict__ items, int n_items) {
  __shared__ double dv[3];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();
    const int k = items[it].x, w = items[it].y;
    const SysDev& s = a.sysv[k];
    const WalkDev& wd = a.wkv[k];
    const int e = (int)(a.steps[k] % s.N);
    if (threadIdx.x == 0) {
      double d[3], u;
      member_draw(a, k, w, wd.Wk, d, &u);
      dv[0] = d[0]; dv[1] = d[1]; dv[2] = d[2];
    }
    __syncthreads();
    prep_body<false>(s, wd, w, e, nullptr, dv);
  }
}

template <typename T, int NC>
__global__ void __launch_bounds__(256) multi_rows_kernel(MultiArgs a, const int4* __restrict__ items, int n_items) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();
    const int4 q = items[it];   // member, walker, chunk, chunks
    const SysDev& s = a.sysv[q.x];
    const int e = (int)(a.steps[q.x] % s.N);
    rows_body<T, NC>(s, a.wkv[q.x], q.y, q.z, q.w, e, a.rows[q.x]);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) multi_accept_kernel(MultiArgs a, const int2* __restrict__ items, int n_items) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();
    const int k = items[it].x, w = items[it].y;
    const SysDev& s = a.sysv[k];
    const WalkDev& wd = a.wkv[k];
    const int e = (int)(a.steps[k] % s.N);
    double d[3], u;
    member_draw(a, k, w, wd.Wk, d, &u);
    // the rows phase wrote ceil(n_up / rows) partial ratios for every walker
    // (the count the rows table was built with), whichever spin moved
    accept_body<T>(s, wd, w, e, 1, nullptr, u, nullptr, (s.nu + a.rows[k] - 1) / a.rows[k]);
  }
}

// QMC_REFINED members: one item per walker, the screened stream the lone
// proposal would run (blocked with its LDS where screened_blk_config allows,
// else the plain one), writing the S partial slots the accept sums.
__global__ void __launch_bounds__(256) multi_screened_rows_kernel(MultiArgs a, const int4* __restrict__ items,
                                                                  int n_items) {
  extern __shared__ __align__(16) char dyn[];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    __syncthreads();
    const int4 q = items[it];   // member, walker, 0, 1
    const SysDev& s = a.sysv[q.x];
    const WalkDev& wd = a.wkv[q.x];
    const int e = (int)(a.steps[q.x] % s.N);
    const int S = (s.nu + a.rows[q.x] - 1) / a.rows[q.x];
    int IPB = 0, FB = 0;
    size_t lds = 0;
    if (screened_blk_config(s, wd, e, IPB, FB, lds)) {
      switch (IPB) {
        case 1: screened_stream_walker<1>(s, wd, q.y, e, S, FB, dyn); break;
        case 2: screened_stream_walker<2>(s, wd, q.y, e, S, FB, dyn); break;
        case 3: screened_stream_walker<3>(s, wd, q.y, e, S, FB, dyn); break;
        case 4: screened_stream_walker<4>(s, wd, q.y, e, S, FB, dyn); break;
        case 5: screened_stream_walker<5>(s, wd, q.y, e, S, FB, dyn); break;
        case 6: screened_stream_walker<6>(s, wd, q.y, e, S, FB, dyn); break;
        case 7: screened_stream_walker<7>(s, wd, q.y, e, S, FB, dyn); break;
        default: screened_stream_walker<8>(s, wd, q.y, e, S, FB, dyn); break;
      }
    } else if (s.nu <= 64) {
      screened_rows_walker<1>(s, wd, q.y, e, S);
    } else {
      screened_rows_walker<2>(s, wd, q.y, e, S);   // members have n_up <= 128
    }
  }
}

__global__ void multi_advance_kernel(long long* steps, int n) {
  const int k = threadIdx.x;
  if (k < n) steps[k] += 1;
}

template <typename T, int NC>
static hipError_t rows_launch(const MultiArgs& a, const int4* items, int n_items, int grid, hipStream_t st) {
  hipLaunchKernelGGL((multi_rows_kernel<T, NC>), dim3(grid), dim3(256), 0, st, a, items, n_items);
  return hipGetLastError();
}

hipError_t launch_multi_prep(const MultiArgs& a, const int2* items, int n_items, int grid, hipStream_t st) {
  hipLaunchKernelGGL(multi_prep_kernel, dim3(grid), dim3(256), 0, st, a, items, n_items);
  return hipGetLastError();
}

hipError_t launch_multi_rows(const MultiArgs& a, int store, int nc, const int4* items, int n_items, int grid,
                             hipStream_t st, size_t screened_lds) {
  if (screened_lds > 0) {
    hipLaunchKernelGGL(multi_screened_rows_kernel, dim3(grid), dim3(256), screened_lds, st, a, items, n_items);
    return hipGetLastError();
  }
#define QMC_MR(T, NC) case NC: return rows_launch<T, NC>(a, items, n_items, grid, st);
  if (store == 2) {
    switch (nc) { QMC_MR(bf16s, 1) QMC_MR(bf16s, 2) QMC_MR(bf16s, 3) QMC_MR(bf16s, 4)
                  QMC_MR(bf16s, 5) QMC_MR(bf16s, 6) QMC_MR(bf16s, 7) QMC_MR(bf16s, 8) }
  } else if (store == 1) {
    switch (nc) { QMC_MR(float, 1) QMC_MR(float, 2) QMC_MR(float, 3) QMC_MR(float, 4)
                  QMC_MR(float, 5) QMC_MR(float, 6) QMC_MR(float, 7) QMC_MR(float, 8) }
  } else {
    switch (nc) { QMC_MR(double, 1) QMC_MR(double, 2) QMC_MR(double, 3) QMC_MR(double, 4)
                  QMC_MR(double, 5) QMC_MR(double, 6) QMC_MR(double, 7) QMC_MR(double, 8) }
  }
#undef QMC_MR
  return hipErrorInvalidValue;
}

hipError_t launch_multi_accept(const MultiArgs& a, int store, const int2* items, int n_items, int grid,
                               hipStream_t st) {
  if (store == 2) hipLaunchKernelGGL(multi_accept_kernel<bf16s>, dim3(grid), dim3(256), 0, st, a, items, n_items);
  else if (store == 1) hipLaunchKernelGGL(multi_accept_kernel<float>, dim3(grid), dim3(256), 0, st, a, items, n_items);
  else hipLaunchKernelGGL(multi_accept_kernel<double>, dim3(grid), dim3(256), 0, st, a, items, n_items);
  return hipGetLastError();
}

hipError_t launch_multi_advance(long long* steps, int n, hipStream_t st) {
  hipLaunchKernelGGL(multi_advance_kernel, dim3(1), dim3(64), 0, st, steps, n);
  return hipGetLastError();
}

}  // namespace qmc
