// Outputs of an evolved state: occupations <n_i> and bitstring samples.
//
// Occupations: <n_i> = sum_b |psi_b|^2 b_p / sum_b |psi_b|^2 with p = n-1-i, FP64.  A
// workgroup owns 2^C contiguous amplitudes (C = min(n, 12)): thread-index bits and the
// register-loop bits are accumulated locally, bits above C are constant per workgroup and
// resolved in the second stage from the workgroup index.
//
// Sampling: shot s draws u_s from a SplitMix64 stream (Steele, Lea & Flood 2014; the Weyl
// increment 0x9E3779B97F4A7C15 and the variant-13 finaliser) seeded with `seed`, and returns
// the smallest b with CDF(b) > u_s * CDF(last); without such a b (rounding), the largest b
// with nonzero probability.  CDF is evaluated as a prefix sum in three levels: per-block
// sums of |psi|^2 (FP64), one exclusive scan over the blocks, then a scan inside the
// selected block.
#include <mutex>

#include "device_common.h"

namespace rsv {
namespace {

constexpr int kChunkBits = 12;
constexpr int kOccStride = 1 + kChunkBits;  // per chunk: total, then one sum per low bit

template <class R>
__device__ __forceinline__ double prob(const Cx<R>& v) {
  return norm_add(0.0, (double)v.x, (double)v.y);
}

template <class R>
__global__ __launch_bounds__(kBlock) void occ_partial_kernel(const Cx<R>* __restrict__ x,
                                                             const int cbits,
                                                             double* __restrict__ partial) {
  __shared__ double red[4];
  const uint32_t tid = threadIdx.x;
  const uint32_t chunk = 1u << cbits;
  const size_t base = (size_t)blockIdx.x << cbits;
  double tot = 0.0, reg[4] = {0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < 16; ++s) {
    const uint32_t e = tid + kBlock * s;
    if (e >= chunk) break;
    const double p = prob<R>(x[base + e]);
    tot += p;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if ((s >> q) & 1) reg[q] += p;
  }
  double* out = partial + (size_t)blockIdx.x * kOccStride;
  const double t_all = block_sum_256(tot, red);
  if (tid == 0) out[0] = t_all;
  for (int p = 0; p < 8; ++p) {
    const double t = block_sum_256(((tid >> p) & 1) ? tot : 0.0, red);
    if (tid == 0) out[1 + p] = t;
  }
  for (int q = 0; q < 4; ++q) {
    const double t = block_sum_256(reg[q], red);
    if (tid == 0) out[9 + q] = t;
  }
}

// Second stage: thread t sums chunks [t*per, (t+1)*per) for every output, then a fixed tree.
__global__ __launch_bounds__(kBlock) void occ_finalize_kernel(const double* __restrict__ partial,
                                                              const int64_t nchunk,
                                                              const int n, const int cbits,
                                                              double* __restrict__ out) {
  __shared__ double red[4];
  const int64_t per = (nchunk + kBlock - 1) / kBlock;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nchunk ? lo + per : nchunk;
  for (int p = -1; p < n; ++p) {  // p = -1: the total
    double acc = 0.0;
    for (int64_t ch = lo; ch < hi; ++ch) {
      const double* c = partial + ch * kOccStride;
      if (p < 0) acc += c[0];
      else if (p < cbits) acc += c[1 + p];
      else if ((ch >> (p - cbits)) & 1) acc += c[0];
    }
    const double t = block_sum_256(acc, red);
    if (threadIdx.x == 0) out[1 + p] = t;
  }
}

// --------------------------------------------------------------------------- correlations
// <n_i n_j> numerators.  Per chunk of 2^C amplitudes (C = min(n, 12)) the low C bits vary and
// the bits above are constant, so a chunk contributes its total T, its single-bit sums S_p
// (p < C) and its pair sums P_pq (p < q < C); pairs involving high bits follow from T and
// S_p and the chunk index.  Thread t holds 16 amplitudes e = t + 256 s: bits 0..7 of e are
// t's, bits 8..11 are s's.  Each thread keeps its total, its sums over the s bits and over
// pairs of s bits; the 79 chunk values are then sums over threads in a fixed order.
constexpr int kCorrSlots = 1 + 12 + 66;

__device__ __forceinline__ int corr_pair_slot(int p, int q) {  // p < q < 12
  return 13 + p * 12 - p * (p + 1) / 2 + (q - p - 1);
}

template <class R>
__global__ __launch_bounds__(kBlock) void corr_partial_kernel(const Cx<R>* __restrict__ x,
                                                              const int cbits,
                                                              double* __restrict__ partial) {
  __shared__ double th[11][kBlock];  // total, 4 s-bit sums, 6 s-bit pair sums per thread
  const uint32_t tid = threadIdx.x;
  const uint32_t chunk = 1u << cbits;
  const size_t base = (size_t)blockIdx.x << cbits;
  double v[11];
#pragma unroll
  for (int j = 0; j < 11; ++j) v[j] = 0.0;
  for (int s = 0; s < 16; ++s) {
    const uint32_t e = tid + kBlock * s;
    if (e >= chunk) break;
    const double p = prob<R>(x[base + e]);
    v[0] += p;
    int j = 5;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if ((s >> q) & 1) v[1 + q] += p;
#pragma unroll
      for (int r = q + 1; r < 4; ++r, ++j)
        if (((s >> q) & 1) && ((s >> r) & 1)) v[j] += p;
    }
  }
#pragma unroll
  for (int j = 0; j < 11; ++j) th[j][tid] = v[j];
  __syncthreads();
  if (tid < kCorrSlots) {
    // which per-thread value, and which thread bits must be set, for slot tid
    int src = 0, ta = -1, tb = -1;
    const int slot = (int)tid;
    if (slot == 0) {
      src = 0;
    } else if (slot < 13) {  // single bit p
      const int p = slot - 1;
      if (p < 8) ta = p;
      else src = 1 + (p - 8);
    } else {  // pair p < q
      int p = 0, q = 1;
      for (int a = 0; a < 12; ++a)
        for (int b = a + 1; b < 12; ++b)
          if (corr_pair_slot(a, b) == slot) p = a, q = b;
      if (q < 8) {
        ta = p, tb = q;
      } else if (p < 8) {
        ta = p, src = 1 + (q - 8);
      } else {
        const int a = p - 8, b = q - 8;  // s-bit pair index in the order the loop above used
        int j = 5;
        for (int qq = 0; qq < 4; ++qq)
          for (int rr = qq + 1; rr < 4; ++rr, ++j)
            if (qq == a && rr == b) src = j;
      }
    }
    double acc = 0.0;
    for (int t = 0; t < kBlock; ++t) {
      if (ta >= 0 && !((t >> ta) & 1)) continue;
      if (tb >= 0 && !((t >> tb) & 1)) continue;
      acc += th[src][t];
    }
    partial[(size_t)blockIdx.x * kCorrSlots + slot] = acc;
  }
}

// out[0] = total; out[1 + p * n + q] (p <= q, bit positions) = sum |x_b|^2 b_p b_q.  One
// workgroup per output; thread t sums chunks t, t + 256, ... then a fixed tree.
__global__ __launch_bounds__(kBlock) void corr_finalize_kernel(const double* __restrict__ partial,
                                                               const int64_t nchunk, const int n,
                                                               const int cbits,
                                                               double* __restrict__ out) {
  __shared__ double red[4];
  int p = -1, q = -1;  // workgroup 0: the total
  if (blockIdx.x > 0) {
    int w = (int)blockIdx.x - 1;
    for (int a = 0; a < n && p < 0; ++a)
      for (int b = a; b < n; ++b, --w)
        if (w == 0) {
          p = a, q = b;
          break;
        }
  }
  double acc = 0.0;
  for (int64_t ch = threadIdx.x; ch < nchunk; ch += kBlock) {
    const double* c = partial + ch * kCorrSlots;
    double v;
    if (p < 0) {
      v = c[0];
    } else if (p == q) {
      v = p < cbits ? c[1 + p] : (((ch >> (p - cbits)) & 1) ? c[0] : 0.0);
    } else if (q < cbits) {
      v = c[corr_pair_slot(p, q)];
    } else if (p < cbits) {
      v = ((ch >> (q - cbits)) & 1) ? c[1 + p] : 0.0;
    } else {
      v = (((ch >> (p - cbits)) & 1) && ((ch >> (q - cbits)) & 1)) ? c[0] : 0.0;
    }
    acc += v;
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) {
    if (p < 0) out[0] = t;
    else out[1 + p * n + q] = t;
  }
}

// ------------------------------------------------------------------------------- sampling
__device__ __forceinline__ uint64_t splitmix64_at(uint64_t seed, uint64_t s) {
  uint64_t z = seed + (s + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

template <class R>
__global__ __launch_bounds__(kBlock) void block_prob_kernel(const Cx<R>* __restrict__ x,
                                                            const int cbits,
                                                            double* __restrict__ bsum) {
  __shared__ double red[4];
  const uint32_t chunk = 1u << cbits;
  const size_t base = (size_t)blockIdx.x << cbits;
  double acc = 0.0;
  // the same per-thread order as the in-block scan of sample_kernel
  for (uint32_t j = 0; j < 16; ++j) {
    const uint32_t e = threadIdx.x * 16 + j;
    if (e < chunk) acc += prob<R>(x[base + e]);
  }
  const double t = block_sum_256(acc, red);
  if (threadIdx.x == 0) bsum[blockIdx.x] = t;
}

// Exclusive scan of nb block sums into pre[0..nb], pre[nb] = total.  One workgroup.
__global__ __launch_bounds__(kBlock) void block_scan_kernel(const double* __restrict__ bsum,
                                                            const int64_t nb,
                                                            double* __restrict__ pre) {
  __shared__ double tsum[kBlock];
  const int64_t per = (nb + kBlock - 1) / kBlock;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = lo + per < nb ? lo + per : nb;
  double acc = 0.0;
  for (int64_t i = lo; i < hi; ++i) acc += bsum[i];
  tsum[threadIdx.x] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double run = 0.0;
    for (int t = 0; t < kBlock; ++t) {
      const double v = tsum[t];
      tsum[t] = run;
      run += v;
    }
    pre[nb] = run;
  }
  __syncthreads();
  double run = tsum[threadIdx.x];
  for (int64_t i = lo; i < hi; ++i) {
    pre[i] = run;
    run += bsum[i];
  }
}

template <class R>
__global__ __launch_bounds__(kBlock) void sample_kernel(const Cx<R>* __restrict__ x,
                                                        const int cbits, const int64_t nb,
                                                        const double* __restrict__ pre,
                                                        const double* __restrict__ bsum,
                                                        const uint64_t seed,
                                                        uint64_t* __restrict__ idx) {
  __shared__ double tsum[kBlock];
  __shared__ int64_t blk_sh;
  __shared__ double target_sh;
  __shared__ int fallback_sh;
  __shared__ unsigned int cand, last_sh;
  const uint32_t tid = threadIdx.x;
  const uint32_t chunk = 1u << cbits;
  if (tid == 0) {
    const uint64_t r = splitmix64_at(seed, blockIdx.x);
    const double u = (double)(r >> 11) * 0x1.0p-53;
    const double total = pre[nb];
    const double target = u * total;
    // smallest block whose inclusive prefix exceeds the target
    int64_t lo = 0, hi = nb;  // answer in [lo, hi]; hi == nb means none
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (pre[mid + 1] > target) hi = mid;
      else lo = mid + 1;
    }
    int fb = 0;
    if (lo == nb) {  // no block: fall back to the last block with mass
      fb = 1;
      lo = nb - 1;
      while (lo > 0 && !(bsum[lo] > 0.0)) --lo;
    }
    blk_sh = lo;
    target_sh = target;
    fallback_sh = fb;
    cand = 0xFFFFFFFFu;
    last_sh = 0u;
  }
  __syncthreads();
  const int64_t blk = blk_sh;
  const double target = target_sh;
  const size_t base = (size_t)blk << cbits;
  double p[16];
  double own = 0.0;
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const uint32_t e = tid * 16 + j;
    p[j] = e < chunk ? prob<R>(x[base + e]) : 0.0;
    own += p[j];
  }
  tsum[tid] = own;
  __syncthreads();
  if (tid == 0) {
    double run = pre[blk];
    for (int t = 0; t < kBlock; ++t) {
      const double v = tsum[t];
      tsum[t] = run;
      run += v;
    }
  }
  __syncthreads();
  if (!fallback_sh) {
    double c = tsum[tid];
    for (int j = 0; j < 16; ++j) {
      c += p[j];
      if (c > target && p[j] > 0.0) {
        atomicMin(&cand, tid * 16 + j);
        break;
      }
    }
  }
  __syncthreads();
  const unsigned int found = cand;  // every thread reads before anyone writes last_sh
  if (found == 0xFFFFFFFFu) {       // rounding left no index: take the last one with mass
    for (int j = 15; j >= 0; --j) {
      if (p[j] > 0.0) {
        atomicMax(&last_sh, tid * 16 + j + 1);  // +1: zero means "no mass in this block"
        break;
      }
    }
    __syncthreads();
    if (tid == 0) idx[blockIdx.x] = (uint64_t)base + (last_sh > 0 ? last_sh - 1 : 0);
    return;
  }
  if (tid == 0) idx[blockIdx.x] = (uint64_t)base + found;
}

// Scratch of the allocation-free sampling entry point: the block sums and their exclusive
// scan for up to kMaxAtoms atoms, then the drawn indices of up to kStaticMaxShots shots
// (4.7 MB, held by every device the library runs on until the process ends).
constexpr int64_t kStaticBlocks = int64_t(1) << (kMaxAtoms - kChunkBits);
constexpr size_t kStaticIdxOffset = (size_t)(2 * kStaticBlocks + 1 + 31) / 32 * 32;  // doubles
constexpr size_t kStaticDoubles = kStaticIdxOffset + kStaticMaxShots;
static __device__ __align__(256) double scratch[kStaticDoubles];

}  // namespace

int static_sample_scratch(int device, void** out) {
  // The array's host-side name is not a device address: its address on each device comes
  // from the runtime, once per device, with that device current.
  static std::mutex mu;
  static void* addr[64] = {};
  if (device < 0 || device >= 64) return -1;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return -1;
    addr[device] = p;
  }
  *out = addr[device];
  return 0;
}

size_t static_sample_idx_offset_bytes() { return kStaticIdxOffset * sizeof(double); }

int64_t occ_num_partials(int n) {
  const int cbits = n < kChunkBits ? n : kChunkBits;
  return (int64_t(1) << (n - cbits)) * kOccStride;
}

hipError_t occupations(int prec, int n, const void* x, double* partial, double* out,
                       hipStream_t s) {
  const int cbits = n < kChunkBits ? n : kChunkBits;
  const uint32_t nchunk = 1u << (n - cbits);
  if (prec == kC128)
    hipLaunchKernelGGL(occ_partial_kernel<double>, dim3(nchunk), dim3(kBlock), 0, s,
                       (const double2*)x, cbits, partial);
  else
    hipLaunchKernelGGL(occ_partial_kernel<float>, dim3(nchunk), dim3(kBlock), 0, s,
                       (const float2*)x, cbits, partial);
  hipLaunchKernelGGL(occ_finalize_kernel, dim3(1), dim3(kBlock), 0, s, partial,
                     (int64_t)nchunk, n, cbits, out);
  return hipGetLastError();
}

int64_t corr_scratch_doubles(int n) {
  const int cbits = n < kChunkBits ? n : kChunkBits;
  return (int64_t(1) << (n - cbits)) * kCorrSlots + 1 + (int64_t)n * n;
}

hipError_t correlations(int prec, int n, const void* x, double* scratch, double** out_dev,
                        hipStream_t s) {
  const int cbits = n < kChunkBits ? n : kChunkBits;
  const uint32_t nchunk = 1u << (n - cbits);
  double* out = scratch + (size_t)nchunk * kCorrSlots;
  if (prec == kC128)
    hipLaunchKernelGGL(corr_partial_kernel<double>, dim3(nchunk), dim3(kBlock), 0, s,
                       (const double2*)x, cbits, scratch);
  else
    hipLaunchKernelGGL(corr_partial_kernel<float>, dim3(nchunk), dim3(kBlock), 0, s,
                       (const float2*)x, cbits, scratch);
  hipLaunchKernelGGL(corr_finalize_kernel, dim3(1 + n * (n + 1) / 2), dim3(kBlock), 0, s, scratch,
                     (int64_t)nchunk, n, cbits, out);
  *out_dev = out;
  return hipGetLastError();
}

int64_t sample_scratch_doubles(int n) {
  const int cbits = n < kChunkBits ? n : kChunkBits;
  const int64_t nb = int64_t(1) << (n - cbits);
  return 2 * nb + 1;
}

hipError_t sample(int prec, int n, const void* x, uint64_t seed, int shots, double* scratch,
                  uint64_t* idx, hipStream_t s) {
  const int cbits = n < kChunkBits ? n : kChunkBits;
  const int64_t nb = int64_t(1) << (n - cbits);
  double* bsum = scratch;
  double* pre = scratch + nb;
  if (prec == kC128)
    hipLaunchKernelGGL(block_prob_kernel<double>, dim3((uint32_t)nb), dim3(kBlock), 0, s,
                       (const double2*)x, cbits, bsum);
  else
    hipLaunchKernelGGL(block_prob_kernel<float>, dim3((uint32_t)nb), dim3(kBlock), 0, s,
                       (const float2*)x, cbits, bsum);
  hipLaunchKernelGGL(block_scan_kernel, dim3(1), dim3(kBlock), 0, s, bsum, nb, pre);
  if (shots > 0) {
    if (prec == kC128)
      hipLaunchKernelGGL(sample_kernel<double>, dim3((uint32_t)shots), dim3(kBlock), 0, s,
                         (const double2*)x, cbits, nb, pre, bsum, seed, idx);
    else
      hipLaunchKernelGGL(sample_kernel<float>, dim3((uint32_t)shots), dim3(kBlock), 0, s,
                         (const float2*)x, cbits, nb, pre, bsum, seed, idx);
  }
  return hipGetLastError();
}

}  // namespace rsv
