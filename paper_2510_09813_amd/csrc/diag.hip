// Interaction diagonal E_b = sum_{i>j} C/|r_ij|^6 n_i n_j of eq. (3), built once per register.
//
// Sec. III.A keeps only the diagonal of H (plus the drive samples) instead of a sparse
// matrix.  The detuning part of the diagonal changes every step and is added on the fly by
// the H|psi> kernels from the bit pattern, so only the interaction part is stored.
//
// diag_build writes the whole diagonal (for callers that want E itself, and for the packed
// small-job path); the H|psi> passes use the much smaller tables of diag_tables_build.
//
// A workgroup owns 2^C amplitudes with equal high bits (C = min(n, 12)).  In LDS it keeps
// the bit-indexed U, the energy of the high bits alone and, per low bit p, the coupling
// F_p = sum over set high bits q of U_pq; an amplitude then needs only its low-bit pairs:
//   E_b = E_hi + sum_{p in lo(b)} (F_p + sum_{q in lo(b), q < p} U_pq).
#include "device_common.h"

namespace rsv {
namespace {

template <class R>
__global__ __launch_bounds__(kBlock) void diag_kernel(const int n, const int cbits,
                                                      const double* __restrict__ ub,
                                                      R* __restrict__ diag) {
  __shared__ double u[32][32];
  __shared__ double f[32];
  __shared__ double ehi;
  const uint32_t tid = threadIdx.x;
  for (int i = tid; i < 32 * 32; i += kBlock) u[i >> 5][i & 31] = ub[i];
  __syncthreads();
  const uint32_t hi = blockIdx.x;  // bits [cbits, n) of every index in this workgroup
  if (tid < 32) {
    double s = 0.0;
    if ((int)tid < cbits) {
      for (int q = cbits; q < n; ++q)
        if ((hi >> (q - cbits)) & 1u) s += u[tid][q];
    }
    f[tid] = s;
  }
  if (tid == 64) {
    double s = 0.0;
    for (int q = cbits; q < n; ++q) {
      if (!((hi >> (q - cbits)) & 1u)) continue;
      for (int p = cbits; p < q; ++p)
        if ((hi >> (p - cbits)) & 1u) s += u[p][q];
    }
    ehi = s;
  }
  __syncthreads();
  const uint32_t chunk = 1u << cbits;
  const size_t base = (size_t)hi << cbits;
  for (uint32_t e = tid; e < chunk; e += kBlock) {
    double acc = ehi;
    uint32_t m = e;
    while (m) {
      const int p = __ffs(m) - 1;
      m &= m - 1;
      acc += f[p];
      uint32_t below = e & ((1u << p) - 1u);
      while (below) {
        const int q = __ffs(below) - 1;
        below &= below - 1;
        acc += u[p][q];
      }
    }
    diag[base + e] = (R)acc;
  }
}

// Tables of E_b for the low pass (see diag_tables_build): entries [0, 2^L) are elo, the
// rest are etile rows of L + 1 values.  One thread per entry; n <= 30, so the pair sums
// are short.
__global__ __launch_bounds__(kBlock) void diag_tables_kernel(const int n, const int lbits,
                                                             const double* __restrict__ ub,
                                                             double* __restrict__ dtab,
                                                             const int64_t count) {
  __shared__ double u[32][32];
  for (int i = threadIdx.x; i < 32 * 32; i += kBlock) u[i >> 5][i & 31] = ub[i];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i >= count) return;
  const int64_t nlo = int64_t(1) << lbits;
  double s = 0.0;
  if (i < nlo) {  // pairs inside the low bits of e = i
    const uint32_t e = (uint32_t)i;
    for (int q = 1; q < lbits; ++q) {
      if (!((e >> q) & 1u)) continue;
      for (int p = 0; p < q; ++p)
        if ((e >> p) & 1u) s += u[p][q];
    }
  } else {
    const int64_t j = i - nlo;
    const uint32_t t = (uint32_t)(j / (lbits + 1));
    const int k = (int)(j % (lbits + 1));
    if (k == 0) {  // pairs among the tile's high bits
      for (int q = lbits + 1; q < n; ++q) {
        if (!((t >> (q - lbits)) & 1u)) continue;
        for (int p = lbits; p < q; ++p)
          if ((t >> (p - lbits)) & 1u) s += u[p][q];
      }
    } else {  // coupling of low bit k - 1 to the tile's set high bits
      const int p = k - 1;
      for (int q = lbits; q < n; ++q)
        if ((t >> (q - lbits)) & 1u) s += u[p][q];
    }
  }
  dtab[i] = s;
}

}  // namespace

size_t diag_table_doubles(int prec, int n) {
  const int L = make_tile_plan(prec, n).lo_bits;
  return (size_t(1) << L) + (size_t(1) << (n - L)) * (size_t)(L + 1);
}

hipError_t diag_tables_build(int prec, int n, const double* d_ub, double* dtab, hipStream_t s) {
  const int L = make_tile_plan(prec, n).lo_bits;
  const int64_t count = (int64_t)diag_table_doubles(prec, n);
  const uint32_t nblk = (uint32_t)((count + kBlock - 1) / kBlock);
  hipLaunchKernelGGL(diag_tables_kernel, dim3(nblk), dim3(kBlock), 0, s, n, L, d_ub, dtab, count);
  return hipGetLastError();
}

hipError_t diag_build(int prec, int n, const double* d_ub, void* diag, hipStream_t s) {
  const int cbits = n < 12 ? n : 12;
  const uint32_t nblk = 1u << (n - cbits);
  if (prec == kC128)
    hipLaunchKernelGGL(diag_kernel<double>, dim3(nblk), dim3(kBlock), 0, s, n, cbits, d_ub,
                       (double*)diag);
  else
    hipLaunchKernelGGL(diag_kernel<float>, dim3(nblk), dim3(kBlock), 0, s, n, cbits, d_ub,
                       (float*)diag);
  return hipGetLastError();
}

}  // namespace rsv
