// Small device helpers: wavefront/block reductions and the pivot comparison.
#pragma once

#include <hip/hip_runtime.h>

#include "mpid_internal.h"

namespace mpid {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum over the 256 threads of a block; the result is returned to every thread.
// "scratch" must hold 4 doubles; the call contains two barriers.
__device__ __forceinline__ double block_sum(double v, double* scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) scratch[wave] = v;
  __syncthreads();
  double t = scratch[0] + scratch[1] + scratch[2] + scratch[3];
  __syncthreads();
  return t;
}

// sum over t = start, start + step, ... < end of p[t * stride], keeping eight
// independent loads in flight; fixed summation order (deterministic).
__device__ __forceinline__ double strided_sum(const double* __restrict__ p, int64_t stride,
                                              int64_t start, int64_t end, int step) {
  double s[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) s[u] = 0.0;
  int64_t t = start;
  for (; t + 7 * (int64_t)step < end; t += 8 * (int64_t)step) {
#pragma unroll
    for (int u = 0; u < 8; ++u) s[u] += p[(t + (int64_t)u * step) * stride];
  }
  for (; t < end; t += step) s[0] += p[t * stride];
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Pivot order: larger norm first; equal norms go to the smaller swap-order key.
__device__ __forceinline__ bool amax_better(double va, int ka, double vb, int kb) {
  return va > vb || (va == vb && ka < kb);
}

struct AmaxVal {
  double v, s2;
  int pos, key;
};

__device__ __forceinline__ AmaxVal amax_combine(AmaxVal a, AmaxVal b) {
  AmaxVal r = amax_better(a.v, a.key, b.v, b.key) ? a : b;
  r.s2 = a.s2 + b.s2;
  return r;
}

__device__ __forceinline__ AmaxVal wave_amax(AmaxVal a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    AmaxVal b;
    b.v = __shfl_xor(a.v, off, 64);
    b.s2 = __shfl_xor(a.s2, off, 64);
    b.pos = __shfl_xor(a.pos, off, 64);
    b.key = __shfl_xor(a.key, off, 64);
    a = amax_combine(a, b);
  }
  return a;
}

// Block-wide pivot reduction; result returned to every thread (two barriers).
__device__ __forceinline__ AmaxVal block_amax(AmaxVal a, AmaxVal* scratch) {
  a = wave_amax(a);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) scratch[wave] = a;
  __syncthreads();
  AmaxVal r = scratch[0];
  r = amax_combine(r, scratch[1]);
  r = amax_combine(r, scratch[2]);
  r = amax_combine(r, scratch[3]);
  __syncthreads();
  return r;
}

__device__ __forceinline__ AmaxVal amax_none() {
  AmaxVal a;
  a.v = -1.0;
  a.s2 = 0.0;
  a.pos = -1;
  a.key = 0x7fffffff;
  return a;
}

}  // namespace mpid
