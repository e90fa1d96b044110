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
// loop bits of the fused occupation sums: at most n - 19 (30 atoms, 2048 workgroups)
constexpr int kOccLoopBits = 11;
constexpr int kOccCombSlots = 1 + 8 + kOccLoopBits;

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

// The combination with the occupation sums of the new state fused in (observables at
// intermediate times, read from the same pass that writes the state).  With the grid of
// stream_grid, thread t of workgroup w visits i = w * 256 + t + k * stride (stride = grid * 256,
// a power of two SB = log2(stride) bits): bits [0, 8) of i are the thread's, bits [8, SB) the
// workgroup's, bits above SB the loop counter's.  Per workgroup it writes, at
// partial[w * kOccCombSlots + ...]: [0] sum |x|^2, [1 + b] the sum over thread bit b, [9 + q]
// the sum over loop bit q; the workgroup bits are resolved when finalising.
template <class R>
__global__ __launch_bounds__(kBlock) void combine_occ_kernel(const CombineCoef c,
                                                             Cx<R>* __restrict__ out,
                                                             double* __restrict__ partial,
                                                             double* __restrict__ occ_partial,
                                                             const size_t count, const int sb) {
  __shared__ double red[4];
  __shared__ const Cx<R>* ptr[kMaxCombine];
  if (threadIdx.x < c.m) ptr[threadIdx.x] = (const Cx<R>*)c.x[threadIdx.x];
  __syncthreads();
  double acc = 0.0, tot = 0.0, loop[kOccLoopBits];
#pragma unroll
  for (int q = 0; q < kOccLoopBits; ++q) loop[q] = 0.0;
  const size_t stride = (size_t)gridDim.x * kBlock;
  size_t k = 0;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < count; i += stride, ++k) {
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
    // the probability of the stored (rounded) amplitude, as the occupation kernel forms it
    const double pr = norm_add(0.0, (double)r.x, (double)r.y);
    tot += pr;
#pragma unroll
    for (int q = 0; q < kOccLoopBits; ++q)
      if ((k >> q) & 1) loop[q] += pr;
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = t;
  double* o = occ_partial + (size_t)blockIdx.x * kOccCombSlots;
  const double all = block_sum_256(tot, red);
  if (threadIdx.x == 0) o[0] = all;
  for (int b = 0; b < 8; ++b) {
    const double v = block_sum_256(((threadIdx.x >> b) & 1) ? tot : 0.0, red);
    if (threadIdx.x == 0) o[1 + b] = v;
  }
  const int nloop = (int)(64 - __clzll((unsigned long long)((count - 1) | 1))) - sb;  // bits above SB
  for (int q = 0; q < kOccLoopBits; ++q) {
    if (q >= nloop) break;
    const double v = block_sum_256(loop[q], red);
    if (threadIdx.x == 0) o[9 + q] = v;
  }
}

// <n> numerators of combine_occ_kernel's partials: out[0] = total, out[1 + p] = sum over
// amplitudes with bit p set, p < n.  Fixed order: thread t sums workgroups t, t + 256, ...
__global__ __launch_bounds__(kBlock) void combine_occ_finalize(const double* __restrict__ part,
                                                               const int64_t nwg, const int n,
                                                               const int sb,
                                                               double* __restrict__ out) {
  __shared__ double red[4];
  for (int p = -1; p < n; ++p) {
    double a = 0.0;
    for (int64_t w = threadIdx.x; w < nwg; w += kBlock) {
      const double* o = part + w * kOccCombSlots;
      if (p < 0) a += o[0];
      else if (p < 8) a += o[1 + p];
      else if (p < sb) a += ((w >> (p - 8)) & 1) ? o[0] : 0.0;
      else a += o[9 + (p - sb)];
    }
    const double t = block_sum_256(a, red);
    if (threadIdx.x == 0) out[1 + p] = t;
  }
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

int ilog2_u64(uint64_t v) {
  int r = 0;
  while (v > 1) {
    v >>= 1;
    ++r;
  }
  return r;
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

int64_t combine_occ_partial_doubles(int n) {
  return (int64_t)stream_grid(size_t(1) << n, kPerThread) * kOccCombSlots;
}

hipError_t krylov_combine_occ(int prec, int n, const CombineCoef& c, void* out, double* partial,
                              double* occ_partial, double* occ_out, hipStream_t s) {
  const size_t count = size_t(1) << n;
  const uint32_t g = stream_grid(count, kPerThread);
  const int sb = ilog2_u64((uint64_t)g * kBlock);
  if (n - sb > kOccLoopBits || n > kMaxAtoms) return hipErrorInvalidValue;
  if (prec == kC128)
    hipLaunchKernelGGL(combine_occ_kernel<double>, dim3(g), dim3(kBlock), 0, s, c,
                       (double2*)out, partial, occ_partial, count, sb);
  else
    hipLaunchKernelGGL(combine_occ_kernel<float>, dim3(g), dim3(kBlock), 0, s, c,
                       (float2*)out, partial, occ_partial, count, sb);
  hipLaunchKernelGGL(combine_occ_finalize, dim3(1), dim3(kBlock), 0, s, occ_partial,
                     (int64_t)g, n, sb, occ_out);
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
