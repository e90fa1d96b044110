// Liouvillian of the Lindblad master equation (Sec. III.A: open-system dynamics by the full
// master equation, evolved with a Krylov method) on the vectorised density matrix.
//
//   d rho / dt = L rho = -i [H_k, rho] + sum_i (L_i rho L_i^+ - 1/2 {L_i^+ L_i, rho})
//
// with H_k the Hamiltonian of eq. (3) for step k and, per atom, relaxation of the Rydberg
// level L_i = sqrt(gamma_r) |0><1|_i and dephasing L_i = sqrt(2 gamma_phi) n_i (coherences of
// one atom decay at gamma_phi).  rho (2^n x 2^n) is stored row-major as a vector of 4^n
// amplitudes, index (r << n) | c, so the row's bits are the high n bits of the index and the
// column's the low n: bit p of r or c is atom n-1-p as in the state vector.  Element (r, c):
//
//   (L rho)_rc = [-i (D_r - D_c) - sum_p (gamma_r (r_p + c_p) / 2 + gamma_phi (r_p xor c_p))] rho_rc
//              + sum_p [ -i h(r_p) rho_{r^p, c}  +  i h(1 - c_p) rho_{r, c^p} ]
//              + gamma_r sum_{p: r_p = c_p = 0} rho_{r|p, c|p}
//
// where D_x = E_x - sum_p delta_p x_p is H's diagonal (E_x the interaction energy of pattern
// x), h(1) = <1|h_p|0> = Omega_p/2 e^{-i phi_p} and h(0) = <0|h_p|1>.  Every element needs
// 3n + 1 inputs; arithmetic is FP64, results are stored in the storage precision, and the
// 4^n vector is at most 4 GiB (n <= 14).  Up to 12 atoms one thread per element gathers its
// inputs through the cache (the whole density matrix fits the 256 MB last-level cache); from
// 13 atoms on, tiles of 4096 elements go through LDS.
#include "device_common.h"
#include "lindblad.h"

namespace rsv {
namespace {

template <class R, int N>
__global__ __launch_bounds__(kBlock) void liouvillian_kernel(const LindbladCoef c,
                                                             const double* __restrict__ e,
                                                             const Cx<R>* __restrict__ x,
                                                             Cx<R>* __restrict__ y) {
  constexpr int n = N;
  const uint64_t count = uint64_t(1) << (2 * n);
  const uint32_t cmask = (1u << n) - 1u;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count; idx += stride) {
    const uint32_t r = (uint32_t)(idx >> n), col = (uint32_t)idx & cmask;
    double dr = e[r], dc = e[col], loss = 0.0;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      const uint32_t rp = (r >> p) & 1u, cp = (col >> p) & 1u;
      dr -= rp ? c.delta[p] : 0.0;
      dc -= cp ? c.delta[p] : 0.0;
      loss += 0.5 * c.gamma_r * (double)(rp + cp) + ((rp ^ cp) ? c.gamma_phi : 0.0);
    }
    const Cx<R> v = x[idx];
    // (-i (dr - dc) - loss) * v
    double are = -loss * (double)v.x + (dr - dc) * (double)v.y;
    double aim = -loss * (double)v.y - (dr - dc) * (double)v.x;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      const uint32_t rp = (r >> p) & 1u, cp = (col >> p) & 1u;
      // row flip: -i h(r_p) rho_{r^p, c}
      const Cx<R> a = x[idx ^ (uint64_t(1) << (n + p))];
      const double hr = rp ? c.up_re[p] : c.dn_re[p], hi = rp ? c.up_im[p] : c.dn_im[p];
      // -i (hr + i hi)(a) = (hi a.x + hr a.y) + i (hi a.y - hr a.x)
      are += hi * (double)a.x + hr * (double)a.y;
      aim += hi * (double)a.y - hr * (double)a.x;
      // column flip: +i h(1 - c_p) rho_{r, c^p}
      const Cx<R> b = x[idx ^ (uint64_t(1) << p)];
      const double gr = cp ? c.dn_re[p] : c.up_re[p], gi = cp ? c.dn_im[p] : c.up_im[p];
      // i (gr + i gi)(b) = (-gi b.x - gr b.y) + i (gr b.x - gi b.y)
      are += -gi * (double)b.x - gr * (double)b.y;
      aim += gr * (double)b.x - gi * (double)b.y;
      // relaxation feeds (0, 0) of atom p from (1, 1)
      if (c.gamma_r != 0.0 && !rp && !cp) {
        const Cx<R> q = x[idx | (uint64_t(1) << (n + p)) | (uint64_t(1) << p)];
        are += c.gamma_r * (double)q.x;
        aim += c.gamma_r * (double)q.y;
      }
    }
    Cx<R> o;
    o.x = (R)are;
    o.y = (R)aim;
    y[idx] = o;
  }
}

// The same operator on tiles of 2^12 consecutive elements (n >= 13), one tile per
// workgroup.  The tile holds whole column ranges: its columns' flips (index bits 0..11) read
// LDS.  Every index bit above the tile (all row bits, and from 13 atoms the top column bits)
// has one value across the tile, so its flip reads the neighbouring tile in one coalesced
// sweep with one coefficient for the workgroup; as in the H|psi> low pass, the loads of one
// neighbour tile are issued together before any is used, and all of them before the
// barrier.  A relaxation source rho_{r|p, c|p} lies in the tile of the flipped row bit, at
// the element with column bit p set; it is read from global memory as well (that tile was
// just swept: mostly cache hits), and only where the tile's row bit p is 0.
constexpr int kTileBits = 12, kTileThreads = 1024, kTilePer = (1 << kTileBits) / kTileThreads;
constexpr int kTileThreadBits = 10;
static_assert((1 << kTileThreadBits) == kTileThreads, "thread bits");
// The tiled form from 13 atoms; below, one thread per element gathers its inputs through
// the cache.  At 12 atoms (a 256 MB density matrix, last-level-cache resident) the gather
// form measured 0.58 ms against 0.61 ms tiled (complex128; complex64 0.45 against 0.44).  At
// 13 atoms this form takes 2.86 ms (complex128) and 1.92 ms (complex64), where a tile kernel
// that read each neighbour where it was used took 2.84 and 2.35 ms: complex128 is bound by
// neighbour tiles that miss the caches (14 index bits lie above the tile).
constexpr int kLiouvillianTileAtoms = 13;

template <class R, int N>
__global__ __launch_bounds__(kTileThreads) void liouvillian_tile_kernel(
    const LindbladCoef c, const double* __restrict__ e, const Cx<R>* __restrict__ x,
    Cx<R>* __restrict__ y) {
  using C = Cx<R>;
  static_assert(N >= kTileBits, "tiles hold whole column ranges (12 atoms and more)");
  constexpr int n = N;
  __shared__ C tile[1 << kTileBits];
  const uint32_t tid = threadIdx.x;
  const uint64_t base = (uint64_t)xcd_remap(blockIdx.x, gridDim.x) << kTileBits;
  double are[kTilePer], aim[kTilePer];
#pragma unroll
  for (int s = 0; s < kTilePer; ++s) {
    tile[tid + kTileThreads * s] = x[base + tid + kTileThreads * s];
    are[s] = 0.0;
    aim[s] = 0.0;
  }
  // flips of the index bits above the tile
#pragma unroll
  for (int q = kTileBits; q < 2 * n; ++q) {
    const bool bit = (base >> q) & 1u;
    const uint64_t nbase = base ^ (uint64_t(1) << q);
    C nb[kTilePer];
#pragma unroll
    for (int s = 0; s < kTilePer; ++s) nb[s] = x[nbase + tid + kTileThreads * s];
    if (q >= n) {
      // row flip of bit p: -i h(r_p) rho_{r^p, c} = (hi a.x + hr a.y) + i (hi a.y - hr a.x)
      const int p = q - n;
      const double hr = bit ? c.up_re[p] : c.dn_re[p], hi = bit ? c.up_im[p] : c.dn_im[p];
#pragma unroll
      for (int s = 0; s < kTilePer; ++s) {
        are[s] += hi * (double)nb[s].x + hr * (double)nb[s].y;
        aim[s] += hi * (double)nb[s].y - hr * (double)nb[s].x;
      }
    } else {
      // column flip of bit q: +i h(1 - c_q) rho_{r, c^q} = (-gi b.x - gr b.y) + i (gr b.x - gi b.y)
      const double gr = bit ? c.dn_re[q] : c.up_re[q], gi = bit ? c.dn_im[q] : c.up_im[q];
#pragma unroll
      for (int s = 0; s < kTilePer; ++s) {
        are[s] += -gi * (double)nb[s].x - gr * (double)nb[s].y;
        aim[s] += gr * (double)nb[s].x - gi * (double)nb[s].y;
      }
    }
  }
  // relaxation feeds (0, 0) of atom p from (1, 1): rho_{r|p, c|p} where r_p = c_p = 0
  if (c.gamma_r != 0.0) {
#pragma unroll
    for (int p = 0; p < n; ++p) {
      if ((base >> (n + p)) & 1u) continue;  // r_p = 1 across the tile
      if (p >= kTileBits && ((base >> p) & 1u)) continue;  // c_p = 1 across the tile
      // element el (with c_p = 0) takes its source at element el | 2^p of the tile with row
      // bit p set (every address formed here lies inside the matrix, also where c_p = 1)
      const uint64_t sbase = (base | (uint64_t(1) << (n + p))) | (p >= kTileBits ? (uint64_t(1) << p) : 0);
      const uint32_t pin = p < kTileBits ? (1u << p) : 0u;
      C src[kTilePer];
#pragma unroll
      for (int s = 0; s < kTilePer; ++s) {
        const uint32_t el = tid + kTileThreads * s;
        const bool on = !(el & pin);
        src[s] = on ? x[sbase + (el | pin)] : C{0, 0};
      }
#pragma unroll
      for (int s = 0; s < kTilePer; ++s) {
        are[s] += c.gamma_r * (double)src[s].x;
        aim[s] += c.gamma_r * (double)src[s].y;
      }
    }
  }
  __syncthreads();

  const uint32_t cmask = (1u << n) - 1u;
  const uint32_t r = (uint32_t)(base >> n);  // one row per tile
  double dr = e[r];
#pragma unroll
  for (int p = 0; p < n; ++p)
    if ((r >> p) & 1u) dr -= c.delta[p];
#pragma unroll
  for (int s = 0; s < kTilePer; ++s) {
    const uint32_t el = tid + kTileThreads * s;
    const uint64_t idx = base + el;
    const uint32_t col = (uint32_t)idx & cmask;
    double dc = e[col], loss = 0.0;
#pragma unroll
    for (int p = 0; p < n; ++p) {
      const uint32_t rp = (r >> p) & 1u, cp = (col >> p) & 1u;
      dc -= cp ? c.delta[p] : 0.0;
      loss += 0.5 * c.gamma_r * (double)(rp + cp) + ((rp ^ cp) ? c.gamma_phi : 0.0);
    }
    const C v = tile[el];
    // (-i (dr - dc) - loss) v
    double ore = -loss * (double)v.x + (dr - dc) * (double)v.y + are[s];
    double oim = -loss * (double)v.y - (dr - dc) * (double)v.x + aim[s];
#pragma unroll
    for (int p = 0; p < kTileBits; ++p) {
      const uint32_t cp = (el >> p) & 1u;
      const C b = tile[el ^ (1u << p)];
      const double gr = cp ? c.dn_re[p] : c.up_re[p], gi = cp ? c.dn_im[p] : c.up_im[p];
      ore += -gi * (double)b.x - gr * (double)b.y;
      oim += gr * (double)b.x - gi * (double)b.y;
    }
    C o;
    o.x = (R)ore;
    o.y = (R)oim;
    y[idx] = o;
  }
}

// Diagonal of rho: out[r] = Re rho_rr (FP64), r < 2^n.
template <class R>
__global__ __launch_bounds__(kBlock) void rho_diag_kernel(const Cx<R>* __restrict__ x, const int n,
                                                         double* __restrict__ out) {
  const uint32_t dim = 1u << n;
  for (uint32_t r = blockIdx.x * blockDim.x + threadIdx.x; r < dim; r += gridDim.x * blockDim.x)
    out[r] = (double)x[((uint64_t)r << n) | r].x;
}

template <class R, int N>
void launch_liouvillian(const LindbladCoef& c, const double* e, const void* x, void* y,
                        hipStream_t s) {
  constexpr uint64_t count = uint64_t(1) << (2 * N);
  if constexpr (N >= kLiouvillianTileAtoms) {
    hipLaunchKernelGGL((liouvillian_tile_kernel<R, N>), dim3((uint32_t)(count >> kTileBits)),
                       dim3(kTileThreads), 0, s, c, e, (const Cx<R>*)x, (Cx<R>*)y);
  } else {
    uint64_t g = (count + kBlock - 1) / kBlock;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL((liouvillian_kernel<R, N>), dim3((uint32_t)g), dim3(kBlock), 0, s, c, e,
                       (const Cx<R>*)x, (Cx<R>*)y);
  }
}

template <class R>
hipError_t liouvillian_r(const LindbladCoef& c, const double* e, const void* x, void* y,
                         hipStream_t s) {
  switch (c.n) {
    case 1: launch_liouvillian<R, 1>(c, e, x, y, s); break;
    case 2: launch_liouvillian<R, 2>(c, e, x, y, s); break;
    case 3: launch_liouvillian<R, 3>(c, e, x, y, s); break;
    case 4: launch_liouvillian<R, 4>(c, e, x, y, s); break;
    case 5: launch_liouvillian<R, 5>(c, e, x, y, s); break;
    case 6: launch_liouvillian<R, 6>(c, e, x, y, s); break;
    case 7: launch_liouvillian<R, 7>(c, e, x, y, s); break;
    case 8: launch_liouvillian<R, 8>(c, e, x, y, s); break;
    case 9: launch_liouvillian<R, 9>(c, e, x, y, s); break;
    case 10: launch_liouvillian<R, 10>(c, e, x, y, s); break;
    case 11: launch_liouvillian<R, 11>(c, e, x, y, s); break;
    case 12: launch_liouvillian<R, 12>(c, e, x, y, s); break;
    case 13: launch_liouvillian<R, 13>(c, e, x, y, s); break;
    case 14: launch_liouvillian<R, 14>(c, e, x, y, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t liouvillian_apply(int prec, const LindbladCoef& c, const double* e, const void* x,
                             void* y, hipStream_t s) {
  static_assert(kMaxLindbladAtoms == 14, "liouvillian_r instantiates 1..14 atoms");
  return prec == kC128 ? liouvillian_r<double>(c, e, x, y, s) : liouvillian_r<float>(c, e, x, y, s);
}

hipError_t rho_diagonal(int prec, int n, const void* x, double* out, hipStream_t s) {
  const uint32_t dim = 1u << n;
  const uint32_t g = (dim + kBlock - 1) / kBlock;
  if (prec == kC128)
    hipLaunchKernelGGL(rho_diag_kernel<double>, dim3(g), dim3(kBlock), 0, s, (const double2*)x, n, out);
  else
    hipLaunchKernelGGL(rho_diag_kernel<float>, dim3(g), dim3(kBlock), 0, s, (const float2*)x, n, out);
  return hipGetLastError();
}

}  // namespace rsv
