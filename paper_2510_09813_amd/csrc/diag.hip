// Interaction diagonal E_b = sum_{i>j} C/|r_ij|^6 n_i n_j of eq. (3), built once per register.
//
// Sec. III.A keeps only the diagonal of H (plus the drive samples) instead of a sparse
// matrix.  The detuning part of the diagonal changes every step and is added on the fly by
// the H|psi> kernels from the bit pattern, so only the interaction part is stored.
//
// A workgroup owns 2^C amplitudes with equal high bits (C = min(n, 12)).  In LDS it keeps
// the bit-indexed U, the energy of the high bits alone and, per low bit p, the coupling
// F_p = sum over set high bits q of U_pq; an amplitude then needs only its low-bit pairs:
//   E_b = E_hi + sum_{p in lo(b)} (F_p + sum_{q in lo(b), q < p} U_pq).
#include "common.cuh"

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

}  // namespace

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
