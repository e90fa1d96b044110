// Matrix-free H|psi> for the Rydberg Hamiltonian (eq. 3 with the drive phase).
//
// Sec. III.A applies H in two steps: the diagonal, then for every atom the amplitudes with
// that atom's level swapped, scaled by the drive.  On gfx950 this is a bandwidth-bound
// stencil on the n-dimensional hypercube, done in passes over LDS tiles:
//
//  * low pass:  a tile of 2^L contiguous amplitudes (L = 12 for complex128, 13 for
//    complex64, 64 KiB of LDS) covers the L least significant bits.  Each thread keeps 2^(L-8)
//    amplitudes in registers: flips of those bits never touch LDS; flips of the 8 thread-index
//    bits read the tile.  This pass also applies the diagonal E_b read from HBM plus the
//    detuning term, computed from the bit pattern, and the fused Lanczos terms
//    (-c * prev, and Re<x, out> partial sums in FP64).
//  * high passes (n > L): a tile of 2^r contiguous amplitudes (r = 2 or 3, one 64-byte run)
//    times 2^(L-r) combinations of up to L-r high bits; flips of those high bits.  The first
//    high pass writes t, later ones accumulate; the low pass adds t.
//
// No MFMA: the operator has no dense contraction.
#include "common.cuh"

namespace rsv {
namespace {

template <class R> struct Geo;
template <> struct Geo<double> { static constexpr int L = 12, H = 12, RL = 2; };
template <> struct Geo<float> { static constexpr int L = 13, H = 13, RL = 3; };

// Detuning lookup: lut[256 q + v] = -sum_j delta[8q + j] over the set bits j of byte v.
template <class R>
__device__ __forceinline__ void build_delta_lut(const StepCoef& c, R* lut) {
  for (int i = threadIdx.x; i < 4 * 256; i += kBlock) {
    const int q = i >> 8, v = i & 255;
    double s = 0.0;
    for (int j = 0; j < 8; ++j) {
      const int p = 8 * q + j;
      if (p < c.n && ((v >> j) & 1)) s -= c.delta[p];
    }
    lut[i] = (R)s;
  }
}

template <class R, bool SITE>
__device__ __forceinline__ R detuning(const StepCoef& c, const R* lut, uint32_t b) {
  if (SITE) {
    return (lut[b & 255u] + lut[256 + ((b >> 8) & 255u)]) +
           (lut[512 + ((b >> 16) & 255u)] + lut[768 + ((b >> 24) & 255u)]);
  } else {
    return (R)(-c.delta[0] * (double)__popc(b));
  }
}

// acc += coef(bit) * v, coefficients of bit position p.
template <class R>
__device__ __forceinline__ void cmad(Cx<R>& acc, const StepCoef& c, int p, bool bit, Cx<R> v) {
  const R cr = (R)(bit ? c.up_re[p] : c.dn_re[p]);
  const R ci = (R)(bit ? c.up_im[p] : c.dn_im[p]);
  acc.x += cr * v.x - ci * v.y;
  acc.y += cr * v.y + ci * v.x;
}

template <class R>
__device__ __forceinline__ void cadd(Cx<R>& a, Cx<R> v) { a.x += v.x; a.y += v.y; }

// ----------------------------------------------------------------------------- low pass
template <class R, int LB, bool SITE>
__global__ __launch_bounds__(kBlock) void hpsi_lo_kernel(
    const StepCoef c, const R* __restrict__ diag, const Cx<R>* __restrict__ x, const double sx,
    Cx<R>* __restrict__ out, const Cx<R>* __restrict__ tb, const Cx<R>* __restrict__ prev,
    const double cprev, double* __restrict__ partial, const uint32_t nblk) {
  using C = Cx<R>;
  static_assert(LB >= 8, "low pass needs at least 256 amplitudes per tile");
  constexpr int A = 1 << (LB - 8);  // amplitudes per thread
  constexpr int RB = LB - 8;        // bits held in registers
  __shared__ C tile[1 << LB];
  __shared__ R lut[SITE ? 1024 : 1];
  __shared__ double red[4];

  const uint32_t tid = threadIdx.x;
  const uint32_t blk = xcd_remap(blockIdx.x, nblk);
  const uint32_t base = blk << LB;
  if (SITE) build_delta_lut<R>(c, lut);

  const R s_in = (R)sx;
  C v[A];
#pragma unroll
  for (int s = 0; s < A; ++s) {
    const uint32_t e = tid + kBlock * s;
    C a = x[base + e];
    a.x *= s_in;
    a.y *= s_in;
    v[s] = a;
    tile[e] = a;
  }
  __syncthreads();

  const R cp = (R)cprev;
  double dot = 0.0;
#pragma unroll
  for (int s = 0; s < A; ++s) {
    const uint32_t e = tid + kBlock * s;
    const uint32_t b = base + e;
    const R d = diag[b] + detuning<R, SITE>(c, lut, b);
    C acc;
    acc.x = d * v[s].x;
    acc.y = d * v[s].y;
    if (SITE) {
#pragma unroll
      for (int p = 0; p < 8; ++p) cmad<R>(acc, c, p, (tid >> p) & 1, tile[e ^ (1u << p)]);
#pragma unroll
      for (int q = 0; q < RB; ++q) cmad<R>(acc, c, 8 + q, (s >> q) & 1, v[s ^ (1 << q)]);
    } else {
      C all = {0, 0}, one = {0, 0};
#pragma unroll
      for (int p = 0; p < 8; ++p) {
        const C nb = tile[e ^ (1u << p)];
        cadd<R>(all, nb);
        if ((tid >> p) & 1) cadd<R>(one, nb);
      }
#pragma unroll
      for (int q = 0; q < RB; ++q) {
        const C nb = v[s ^ (1 << q)];
        cadd<R>(all, nb);
        if ((s >> q) & 1) cadd<R>(one, nb);
      }
      C zero = {all.x - one.x, all.y - one.y};
      cmad<R>(acc, c, 0, true, one);
      cmad<R>(acc, c, 0, false, zero);
    }
    if (tb) cadd<R>(acc, tb[b]);
    if (prev) {
      const C pv = prev[b];
      acc.x -= cp * pv.x;
      acc.y -= cp * pv.y;
    }
    out[b] = acc;
    if (partial) dot += (double)v[s].x * (double)acc.x + (double)v[s].y * (double)acc.y;
  }
  if (partial) {
    const double t = block_sum_256(dot, red);
    if (tid == 0) partial[blockIdx.x] = t;
  }
}

// ----------------------------------------------------------------------------- small n
// n < 8: one workgroup, one amplitude per thread, every flip through LDS.
template <class R, bool SITE>
__global__ __launch_bounds__(kBlock) void hpsi_small_kernel(
    const StepCoef c, const R* __restrict__ diag, const Cx<R>* __restrict__ x, const double sx,
    Cx<R>* __restrict__ out, const Cx<R>* __restrict__ prev, const double cprev,
    double* __restrict__ partial) {
  using C = Cx<R>;
  __shared__ C tile[128];
  __shared__ R lut[SITE ? 1024 : 1];
  __shared__ double red[4];
  const uint32_t tid = threadIdx.x;
  const uint32_t dim = 1u << c.n;
  if (SITE) build_delta_lut<R>(c, lut);
  C v = {0, 0};
  if (tid < dim) {
    v = x[tid];
    v.x *= (R)sx;
    v.y *= (R)sx;
    tile[tid] = v;
  }
  __syncthreads();
  double dot = 0.0;
  if (tid < dim) {
    const R d = diag[tid] + detuning<R, SITE>(c, lut, tid);
    C acc = {d * v.x, d * v.y};
    for (int p = 0; p < c.n; ++p) cmad<R>(acc, c, SITE ? p : 0, (tid >> p) & 1, tile[tid ^ (1u << p)]);
    if (prev) {
      acc.x -= (R)cprev * prev[tid].x;
      acc.y -= (R)cprev * prev[tid].y;
    }
    out[tid] = acc;
    dot = (double)v.x * (double)acc.x + (double)v.y * (double)acc.y;
  }
  if (partial) {
    const double t = block_sum_256(dot, red);
    if (tid == 0) partial[0] = t;
  }
}

// ----------------------------------------------------------------------------- high pass
// Tile: bits [0, RL) and [a, a + HB - RL) of the index; flips bits in [f0, f1) only.
template <class R, bool SITE>
__global__ __launch_bounds__(kBlock) void hpsi_hi_kernel(
    const StepCoef c, const Cx<R>* __restrict__ x, const double sx, Cx<R>* __restrict__ tb,
    const int accumulate, const int a, const int f0, const int f1, const uint32_t nblk) {
  using C = Cx<R>;
  constexpr int HB = Geo<R>::H, RL = Geo<R>::RL, G = HB - RL;
  constexpr int A = 1 << (HB - 8);
  __shared__ C tile[1 << HB];

  const uint32_t tid = threadIdx.x;
  const uint32_t blk = xcd_remap(blockIdx.x, nblk);
  const int gap = a - RL;  // outside bits between the contiguous run and the tile's high bits
  const uint32_t obase = ((blk & ((1u << gap) - 1u)) << RL) | ((blk >> gap) << (a + G));

  const R s_in = (R)sx;
  C v[A];
  uint32_t gi[A];
#pragma unroll
  for (int s = 0; s < A; ++s) {
    const uint32_t e = tid + kBlock * s;
    gi[s] = obase | (e & ((1u << RL) - 1u)) | ((e >> RL) << a);
    C val = x[gi[s]];
    val.x *= s_in;
    val.y *= s_in;
    v[s] = val;
    tile[e] = val;
  }
  __syncthreads();

#pragma unroll
  for (int s = 0; s < A; ++s) {
    const uint32_t e = tid + kBlock * s;
    C acc = {0, 0};
    C all = {0, 0}, one = {0, 0};
#pragma unroll
    for (int eb = RL; eb < HB; ++eb) {
      const int p = a + eb - RL;
      if (p < f0 || p >= f1) continue;
      C nb;
      if (eb < 8) nb = tile[e ^ (1u << eb)];
      else nb = v[s ^ (1 << (eb - 8))];
      const bool bit = (e >> eb) & 1u;
      if (SITE) {
        cmad<R>(acc, c, p, bit, nb);
      } else {
        cadd<R>(all, nb);
        if (bit) cadd<R>(one, nb);
      }
    }
    if (!SITE) {
      C zero = {all.x - one.x, all.y - one.y};
      cmad<R>(acc, c, 0, true, one);
      cmad<R>(acc, c, 0, false, zero);
    }
    if (accumulate) cadd<R>(acc, tb[gi[s]]);
    tb[gi[s]] = acc;
  }
}

template <class R, int LB, bool SITE>
void launch_lo(const StepCoef& c, const void* diag, const void* x, double sx, void* out,
               const void* tb, const void* prev, double cprev, double* partial, int n,
               hipStream_t s) {
  const uint32_t nblk = 1u << (n - LB);
  hipLaunchKernelGGL((hpsi_lo_kernel<R, LB, SITE>), dim3(nblk), dim3(kBlock), 0, s, c,
                     (const R*)diag, (const Cx<R>*)x, sx, (Cx<R>*)out, (const Cx<R>*)tb,
                     (const Cx<R>*)prev, cprev, partial, nblk);
}

template <class R, bool SITE>
void launch_lo_any(int lb, const StepCoef& c, const void* diag, const void* x, double sx,
                   void* out, const void* tb, const void* prev, double cprev, double* partial,
                   int n, hipStream_t s) {
  switch (lb) {
    case 8: launch_lo<R, 8, SITE>(c, diag, x, sx, out, tb, prev, cprev, partial, n, s); break;
    case 9: launch_lo<R, 9, SITE>(c, diag, x, sx, out, tb, prev, cprev, partial, n, s); break;
    case 10: launch_lo<R, 10, SITE>(c, diag, x, sx, out, tb, prev, cprev, partial, n, s); break;
    case 11: launch_lo<R, 11, SITE>(c, diag, x, sx, out, tb, prev, cprev, partial, n, s); break;
    case 12: launch_lo<R, 12, SITE>(c, diag, x, sx, out, tb, prev, cprev, partial, n, s); break;
    default:
      if constexpr (Geo<R>::L >= 13) {
        launch_lo<R, 13, SITE>(c, diag, x, sx, out, tb, prev, cprev, partial, n, s);
      }
      break;
  }
}

template <class R, bool SITE>
hipError_t apply_t(int n, const StepCoef& c, const void* diag, const void* x, double sx,
                   void* out, const void* prev, double cprev, void* tbuf, double* partial,
                   hipStream_t s) {
  if (n < 8) {
    hipLaunchKernelGGL((hpsi_small_kernel<R, SITE>), dim3(1), dim3(kBlock), 0, s, c,
                       (const R*)diag, (const Cx<R>*)x, sx, (Cx<R>*)out, (const Cx<R>*)prev,
                       cprev, partial);
    return hipGetLastError();
  }
  const TilePlan plan = make_tile_plan(sizeof(R) == 8 ? kC128 : kC64, n);
  for (int i = 0; i < plan.n_hi_passes; ++i) {
    const uint32_t nblk = 1u << (n - plan.hi_bits);
    hipLaunchKernelGGL((hpsi_hi_kernel<R, SITE>), dim3(nblk), dim3(kBlock), 0, s, c,
                       (const Cx<R>*)x, sx, (Cx<R>*)tbuf, i > 0 ? 1 : 0, plan.tile_a[i],
                       plan.flip_lo[i], plan.flip_hi[i], nblk);
  }
  launch_lo_any<R, SITE>(plan.lo_bits, c, diag, x, sx, out,
                         plan.n_hi_passes > 0 ? tbuf : nullptr, prev, cprev, partial, n, s);
  return hipGetLastError();
}

}  // namespace

TilePlan make_tile_plan(int prec, int n) {
  TilePlan p{};
  p.n = n;
  const int L = prec == kC128 ? Geo<double>::L : Geo<float>::L;
  p.hi_bits = prec == kC128 ? Geo<double>::H : Geo<float>::H;
  p.r_bits = prec == kC128 ? Geo<double>::RL : Geo<float>::RL;
  p.lo_bits = n < L ? n : L;
  p.n_hi_passes = 0;
  const int g = p.hi_bits - p.r_bits;
  for (int f0 = p.lo_bits; f0 < n; f0 += g) {
    const int f1 = f0 + g < n ? f0 + g : n;
    int a = f0;
    if (a + g > n) a = n - g;  // keep the whole tile inside the index; extra bits are not flipped
    p.flip_lo[p.n_hi_passes] = f0;
    p.flip_hi[p.n_hi_passes] = f1;
    p.tile_a[p.n_hi_passes] = a;
    ++p.n_hi_passes;
  }
  return p;
}

int64_t hpsi_num_partials(int prec, int n) {
  if (n < 8) return 1;
  const TilePlan p = make_tile_plan(prec, n);
  return int64_t(1) << (n - p.lo_bits);
}

hipError_t hpsi_apply(int prec, int n, const StepCoef& c, const void* diag, const void* x,
                      double sx, void* out, const void* prev, double cprev, void* tbuf,
                      double* partial, hipStream_t s) {
  if (prec == kC128) {
    return c.site ? apply_t<double, true>(n, c, diag, x, sx, out, prev, cprev, tbuf, partial, s)
                  : apply_t<double, false>(n, c, diag, x, sx, out, prev, cprev, tbuf, partial, s);
  }
  return c.site ? apply_t<float, true>(n, c, diag, x, sx, out, prev, cprev, tbuf, partial, s)
                : apply_t<float, false>(n, c, diag, x, sx, out, prev, cprev, tbuf, partial, s);
}

}  // namespace rsv
