// Streaming vector kernels: norms, reductions and the Krylov
// combination psi_{k+1} = |psi_k| V_m exp(-i dt T_m) e_1 (eq. 6).
//
// All are HBM-bound single sweeps.  Every reduction is two-stage and deterministic: each
// workgroup writes one FP64 partial in a fixed grid-stride order, then one workgroup sums
// the partials in a fixed order (no floating-point atomics), so a result does not depend on
// what else runs on the device.
#include "device_common.h"

namespace rsv {
namespace {

constexpr int kPerThread = 8;

template <class R>
__global__ __launch_bounds__(kBlock) void combine_kernel(const CombineCoef c,
                                                         Cx<R>* __restrict__ out,
                                                         double* __restrict__ partial,
                                                         const size_t count) {
  __shared__ double red[4];
  __shared__ const Cx<R>* ptr[kMaxCombine];
  if (threadIdx.x < c.m) ptr[threadIdx.x] = (const Cx<R>*)c.x[threadIdx.x];
  __syncthreads();
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
    double re = 0.0, im = 0.0;
    for (int l = 0; l < c.m; ++l) {
      const Cx<R> xi = ptr[l][i];
      re += c.re[l] * (double)xi.x - c.im[l] * (double)xi.y;
      im += c.re[l] * (double)xi.y + c.im[l] * (double)xi.x;
    }
    Cx<R> r;
    r.x = (R)re;
    r.y = (R)im;
    out[i] = r;
    acc = norm_add(acc, (double)r.x, (double)r.y);
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

template <class R>
__global__ __launch_bounds__(kBlock) void norm2_kernel(const Cx<R>* __restrict__ x,
                                                       double* __restrict__ partial,
                                                       const size_t count) {
  __shared__ double red[4];
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
    const Cx<R> xi = x[i];
    acc = norm_add(acc, (double)xi.x, (double)xi.y);
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
}

// Conjugate inner products of up to kDotGroup vectors with y, FP64 accumulation.
template <class R>
__global__ __launch_bounds__(kBlock) void multi_dot_kernel(const DotGroup d,
                                                           const Cx<R>* __restrict__ y,
                                                           double* __restrict__ partial,
                                                           const size_t count) {
  __shared__ double red[4];
  double acc[2 * kDotGroup];
#pragma unroll
  for (int j = 0; j < 2 * kDotGroup; ++j) acc[j] = 0.0;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
    const Cx<R> yi = y[i];
#pragma unroll
    for (int g = 0; g < kDotGroup; ++g) {
      if (g < d.g) {
        const Cx<R> xi = ((const Cx<R>*)d.x[g])[i];
        acc[2 * g] += (double)xi.x * (double)yi.x + (double)xi.y * (double)yi.y;
        acc[2 * g + 1] += (double)xi.x * (double)yi.y - (double)xi.y * (double)yi.x;
      }
    }
  }
#pragma unroll
  for (int j = 0; j < 2 * kDotGroup; ++j) {
    if (j < 2 * d.g) {
      const double t = block_sum_256(acc[j], red);
      if (threadIdx.x == 0) partial[(size_t)j * gridDim.x + blockIdx.x] = t;
    }
  }
}

// One workgroup of 1024 threads per row: thread t sums partial[t], partial[t + 1024], ... in
// order (coalesced loads, four independent chains), then a fixed tree over the workgroup.
constexpr int kFinalizeThreads = 1024;
__global__ __launch_bounds__(kFinalizeThreads) void finalize_kernel(const double* __restrict__ all,
                                                                    const int64_t count,
                                                                    double* __restrict__ dst_all) {
  __shared__ double red[kFinalizeThreads / 64];
  const double* partial = all + (size_t)blockIdx.x * count;
  double* dst = dst_all + blockIdx.x;
  constexpr int64_t S = kFinalizeThreads;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t i = threadIdx.x;
  for (; i + 3 * S < count; i += 4 * S) {
    a0 += partial[i];
    a1 += partial[i + S];
    a2 += partial[i + 2 * S];
    a3 += partial[i + 3 * S];
  }
  for (; i < count; i += S) a0 += partial[i];
  double v = (a0 + a1) + (a2 + a3);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kFinalizeThreads / 64; ++w) t += red[w];
    dst[0] = t;
  }
}

template <class RS, class RD>
__global__ __launch_bounds__(kBlock) void convert_kernel(const Cx<RS>* __restrict__ src,
                                                         Cx<RD>* __restrict__ dst,
                                                         const size_t count) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride) {
    const Cx<RS> v = src[i];
    Cx<RD> r;
    r.x = (RD)v.x;
    r.y = (RD)v.y;
    dst[i] = r;
  }
}

}  // namespace

int64_t vec_num_partials(int prec, int n) {
  (void)prec;
  return stream_grid(size_t(1) << n, kPerThread);
}

hipError_t krylov_combine(int prec, int n, const CombineCoef& c, void* out, double* partial,
                          hipStream_t s) {
  const size_t count = size_t(1) << n;
  const uint32_t g = stream_grid(count, kPerThread);
  if (prec == kC128)
    hipLaunchKernelGGL(combine_kernel<double>, dim3(g), dim3(kBlock), 0, s, c, (double2*)out,
                       partial, count);
  else
    hipLaunchKernelGGL(combine_kernel<float>, dim3(g), dim3(kBlock), 0, s, c, (float2*)out,
                       partial, count);
  return hipGetLastError();
}

hipError_t norm2_partial(int prec, int n, const void* x, double* partial, hipStream_t s) {
  const size_t count = size_t(1) << n;
  const uint32_t g = stream_grid(count, kPerThread);
  if (prec == kC128)
    hipLaunchKernelGGL(norm2_kernel<double>, dim3(g), dim3(kBlock), 0, s, (const double2*)x,
                       partial, count);
  else
    hipLaunchKernelGGL(norm2_kernel<float>, dim3(g), dim3(kBlock), 0, s, (const float2*)x,
                       partial, count);
  return hipGetLastError();
}

hipError_t finalize_sum(const double* partial, int64_t count, double* dst, hipStream_t s) {
  return finalize_rows(partial, count, 1, dst, s);
}

hipError_t finalize_rows(const double* partial, int64_t count, int rows, double* dst,
                         hipStream_t s) {
  if (rows <= 0) return hipSuccess;
  hipLaunchKernelGGL(finalize_kernel, dim3(rows), dim3(kFinalizeThreads), 0, s, partial, count,
                     dst);
  return hipGetLastError();
}

hipError_t multi_dot(int prec, int n, const DotGroup& d, const void* y, double* partial,
                     hipStream_t s) {
  const size_t count = size_t(1) << n;
  const uint32_t g = stream_grid(count, kPerThread);
  if (prec == kC128)
    hipLaunchKernelGGL(multi_dot_kernel<double>, dim3(g), dim3(kBlock), 0, s, d,
                       (const double2*)y, partial, count);
  else
    hipLaunchKernelGGL(multi_dot_kernel<float>, dim3(g), dim3(kBlock), 0, s, d,
                       (const float2*)y, partial, count);
  return hipGetLastError();
}

hipError_t convert_from_c128(int prec, int n, const void* src, void* dst, hipStream_t s) {
  const size_t count = size_t(1) << n;
  const uint32_t g = stream_grid(count, kPerThread);
  if (prec == kC128)
    hipLaunchKernelGGL((convert_kernel<double, double>), dim3(g), dim3(kBlock), 0, s,
                       (const double2*)src, (double2*)dst, count);
  else
    hipLaunchKernelGGL((convert_kernel<double, float>), dim3(g), dim3(kBlock), 0, s,
                       (const double2*)src, (float2*)dst, count);
  return hipGetLastError();
}

hipError_t convert_to_c128(int prec, int n, const void* src, void* dst, hipStream_t s) {
  const size_t count = size_t(1) << n;
  const uint32_t g = stream_grid(count, kPerThread);
  if (prec == kC128)
    hipLaunchKernelGGL((convert_kernel<double, double>), dim3(g), dim3(kBlock), 0, s,
                       (const double2*)src, (double2*)dst, count);
  else
    hipLaunchKernelGGL((convert_kernel<float, double>), dim3(g), dim3(kBlock), 0, s,
                       (const float2*)src, (double2*)dst, count);
  return hipGetLastError();
}

}  // namespace rsv
