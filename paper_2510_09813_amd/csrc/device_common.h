// Device helpers shared by the librsv kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rsv_internal.h"

namespace rsv {

template <class R> struct CxT;
template <> struct CxT<double> { using T = double2; };
template <> struct CxT<float> { using T = float2; };
template <class R> using Cx = typename CxT<R>::T;

// The hardware hands workgroup w to XCD w % 8.  Give every XCD one contiguous range of tile
// indices, so that neighbouring tiles (which share cache lines in the strided passes) are
// scheduled back to back on the same XCD and its L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t bid, uint32_t nblk) {
  if (nblk < 8 || (nblk & 7u) != 0) return bid;
  return (bid & 7u) * (nblk >> 3) + (bid >> 3);
}

// Sum of a double over a 256-thread workgroup; the result is valid in thread 0.  Fixed
// reduction tree, so the result is bitwise reproducible.
__device__ __forceinline__ double block_sum_256(double v, double* red /* >= 4 doubles */) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return r;
}

// acc + (x^2 + y^2) with every product and sum rounded separately, so that every kernel
// that accumulates a squared norm of the same values gets the same bits.  The pragma keeps
// the operations out of FMA contraction after inlining (the _rn intrinsics alone do not).
__device__ __forceinline__ double norm_add(double acc, double x, double y) {
#pragma clang fp contract(off)
  return acc + (x * x + y * y);
}

// Fixed grid for the streaming vector kernels: 8 workgroups per CU on 256 CUs at most.
inline uint32_t stream_grid(size_t count, int per_thread) {
  size_t per_wg = (size_t)kBlock * per_thread;
  size_t g = (count + per_wg - 1) / per_wg;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return (uint32_t)g;
}

}  // namespace rsv
