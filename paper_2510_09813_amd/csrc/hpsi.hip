// Matrix-free H|psi> for the Rydberg Hamiltonian (eq. 3 with the drive phase), fused with
// the Lanczos recurrence.
//
// Sec. III.A applies H in two steps: the diagonal, then for every atom the amplitudes with
// that atom's level swapped, scaled by the drive.  On gfx950 this is a bandwidth-bound
// stencil on the n-dimensional hypercube, done in passes over LDS tiles:
//
//  * low pass:  a tile of 2^L contiguous amplitudes (L = 12 for complex128, 13 for
//    complex64: 64 KiB of LDS, 512 threads) covers the L least significant bits.  The
//    thread-index bits are flipped through the LDS tile, the remaining bits inside each
//    thread's registers.  This pass applies the diagonal: the interaction energy E_b from
//    two small FP64 tables (a 2^L table of the low-bit pairs, read from L2, and per tile the
//    high-bit pairs and the low-high couplings), so no 2^n diagonal is read from HBM, plus
//    the detuning from the bit pattern; and it adds the high-pass result t.  Where that
//    saves a high pass, it also flips up to 7 of the top bits, reading those neighbours from
//    the other tiles of a group in global memory (mostly cache hits): n = 23..29 complex128
//    and 22..29 complex64 then need one high pass, over the bits between (complex64 on
//    12-bit tiles of 256 threads holding pairs of adjacent amplitudes, up to n = 28).
//  * high passes (n > L): a tile of 2^H amplitudes (H = 13 for complex128, 12 for
//    complex64), 2^r contiguous (r = 3..6: runs of 64 B to 1 KiB) times the combinations of
//    up to H - r high bits, flips those high bits.  The
//    first high pass writes t, later ones accumulate into it.  The passes are as few as the
//    shortest run allows; the tile bits left over lengthen the runs, the forming pass's
//    first.  For vectors of 64 MiB and more the passes request streaming stores.
//
// The first pass of a sweep may *form* its input from up to three stored vectors,
//   u = a0 x0 + (a1 + c * dot[0]) x1 + a2 x2,
// which is the three-term Lanczos recurrence u_{k+1} = H v_k - alpha_k v_k - beta_{k-1}
// v_{k-1} with H v_k, v_k and v_{k-1} stored unnormalised; alpha_k arrives through dot[0]
// (device memory), so no host round trip sits between two sweeps.  That pass stores u and
// the FP64 partial sums of |u|^2; the low pass returns the partial sums of Re<u, H u>.
//
// Coefficient modes (template CM): kCoefUniform (every atom shares Omega, delta, phi),
// kCoefReal (shared and phi = 0: one real coupling, the cheapest form) and kCoefSite.
//
// No MFMA: the operator has no dense contraction.
#include "device_common.h"

namespace rsv {
namespace {

// Tile geometry per storage precision: low-pass tile bits L and threads NL; high-pass tile
// bits H and threads NH, with a contiguous run of RL..RLW bits per pass (longer runs stream
// better; the planner gives each pass the longest run the bit count allows).
template <class R> struct Geo;
template <> struct Geo<double> {
  // 13-bit high tiles (128 KiB of LDS, one workgroup per CU): at 27 atoms the high pass then
  // covers 9 bits with 256-byte runs, so the low pass's extension needs only 6 bits (groups
  // of 4 MB, one XCD's L2) -- measured 7 % less per Lanczos iteration than 12-bit high tiles
  static constexpr int L = 12, NL = 512, H = 13, RL = 3, RLW = 6, NH = 1024;
};
template <> struct Geo<float> {
  static constexpr int L = 13, NL = 512, H = 12, RL = 3, RLW = 6, NH = 1024;
};
// Low-pass threads: NL (8 amplitudes per thread at L bits, room for every operand in
// registers); the extended complex64 pass on 12-bit tiles takes 256 threads of 16
// amplitudes (measured 5 % faster at 27 atoms: 0.93 against 0.98 ms).
template <class R, int CM, int LB, int E>
constexpr int lo_threads() {
  return sizeof(R) == 4 && LB == 12 && E > 0 ? 256 : Geo<R>::NL;
}
static_assert(Geo<double>::RL == 3 && Geo<double>::RLW == 6 && Geo<float>::RL == 3 &&
                  Geo<float>::RLW == 6,
              "launch_hi instantiates run lengths 3..6");

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

// Sum of a double over an NT-thread workgroup (fixed tree; valid in thread 0).
template <int NT>
__device__ __forceinline__ double wg_sum(double v, double* red /* NT / 64 doubles */) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) r += red[w];
  }
  __syncthreads();
  return r;
}

// Device-side arguments of one pass.
template <class R>
struct PassArgs {
  const Cx<R>* x0;
  const Cx<R>* x1;
  const Cx<R>* x2;
  double a0, a1, a2;
  const double* dot;  // optional: a1 += dot_coef * dot[0]
  double dot_coef;
  const double* nrm1;  // optional: coefficients from device norms (see SweepIn)
  const double* nrm2;
  Cx<R>* u_out;       // optional: store the formed input
  double* part_norm;  // optional: per-workgroup |u|^2
  // high pass
  Cx<R>* tb;
  int accumulate, a, f0, f1;
  // low pass: interaction-diagonal tables (elo: 2^L values, etile: L + 1 per tile)
  const double* elo;
  const double* etile;
  Cx<R>* out;
  double* part_dot;  // optional: per-workgroup Re<u, out>
  int ext_bit;       // low pass: tile-index bit of the first extension bit
  uint32_t nblk;
  int streaming;     // vectors larger than the caches hold: stores bypass them
};

// Store of one amplitude; streaming stores skip the caches (nothing written by a pass is
// read again before the whole vector has streamed through).  Where both branches store the
// same value to the same address, the compiler may merge them into one plain store and drop
// the hint: the high pass's partial t keeps it, the low pass's stores do not.
template <class T>
__device__ __forceinline__ void put(T* p, const T& v, int streaming) {
  if (streaming) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}

// Coefficients of the formed input u = a0 x0 + b1 x1 + a2 x2.
struct Coefs {
  double a0, b1, a2;
};

template <class R>
__device__ __forceinline__ Coefs input_coefs(const PassArgs<R>& p) {
  if (p.nrm1) {  // s_{k-1}, s_{k-2} from the norms of the stored vectors
    const double s1 = 1.0 / sqrt(p.nrm1[0]);
    const double s2 = p.nrm2 ? 1.0 / sqrt(p.nrm2[0]) : 0.0;
    return Coefs{s1, -s1 * s1 * s1 * p.dot[0], -s2 / s1};
  }
  return Coefs{p.a0, p.dot ? p.a1 + p.dot_coef * p.dot[0] : p.a1, p.a2};
}

// u = a0 x0[i] + b1 x1[i] + a2 x2[i] in FP64, rounded once to the storage precision.
template <class R>
__device__ __forceinline__ Cx<R> form(const PassArgs<R>& p, const Coefs& co, size_t i) {
  const Cx<R> v0 = p.x0[i];
  if (!p.x1 && !p.x2 && co.a0 == 1.0) return v0;
  double re = co.a0 * (double)v0.x, im = co.a0 * (double)v0.y;
  if (p.x1) {
    const Cx<R> v1 = p.x1[i];
    re += co.b1 * (double)v1.x;
    im += co.b1 * (double)v1.y;
  }
  if (p.x2) {
    const Cx<R> v2 = p.x2[i];
    re += co.a2 * (double)v2.x;
    im += co.a2 * (double)v2.y;
  }
  Cx<R> r;
  r.x = (R)re;
  r.y = (R)im;
  return r;
}

// Detuning lookup: lut[256 q + v] = -sum_j delta[8q + j] over the set bits j of byte v.
template <class R>
__device__ __forceinline__ void build_delta_lut(const StepCoef& c, R* lut) {
  for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
    const int q = i >> 8, v = i & 255;
    double s = 0.0;
    for (int j = 0; j < 8; ++j) {
      const int p = 8 * q + j;
      if (p < c.n && ((v >> j) & 1)) s -= c.delta[p];
    }
    lut[i] = (R)s;
  }
}

template <class R, int CM>
__device__ __forceinline__ R detuning(const StepCoef& c, const R* lut, uint32_t b) {
  if (CM == kCoefSite) {
    return (lut[b & 255u] + lut[256 + ((b >> 8) & 255u)]) +
           (lut[512 + ((b >> 16) & 255u)] + lut[768 + ((b >> 24) & 255u)]);
  } else {
    return (R)(-c.delta[0] * (double)__popc(b));
  }
}

// acc += coef(bit) * v with the coefficients of bit position p.
template <class R>
__device__ __forceinline__ void cmad(Cx<R>& acc, const StepCoef& c, int p, bool bit, Cx<R> v) {
  const R cr = (R)(bit ? c.up_re[p] : c.dn_re[p]);
  const R ci = (R)(bit ? c.up_im[p] : c.dn_im[p]);
  acc.x += cr * v.x - ci * v.y;
  acc.y += cr * v.y + ci * v.x;
}

template <class R>
__device__ __forceinline__ void cadd(Cx<R>& a, Cx<R> v) {
  a.x += v.x;
  a.y += v.y;
}


// Accumulates the drive terms of one output amplitude flip by flip.
template <class R, int CM>
struct DriveSum {
  Cx<R> acc = {0, 0}, all = {0, 0}, one = {0, 0};
  __device__ __forceinline__ void add(const StepCoef& c, int p, bool bit, Cx<R> nb) {
    if (CM == kCoefSite) {
      cmad<R>(acc, c, p, bit, nb);
    } else {
      cadd<R>(all, nb);
      if (CM == kCoefUniform && bit) cadd<R>(one, nb);
    }
  }
  __device__ __forceinline__ void finish(const StepCoef& c, Cx<R>& out) {
    if (CM == kCoefSite) {
      cadd<R>(out, acc);
    } else if (CM == kCoefReal) {
      const R cr = (R)c.up_re[0];
      out.x += cr * all.x;
      out.y += cr * all.y;
    } else {
      const Cx<R> zero = {all.x - one.x, all.y - one.y};
      cmad<R>(out, c, 0, true, one);
      cmad<R>(out, c, 0, false, zero);
    }
  }
};

// ----------------------------------------------------------------------------- low pass
template <class R, int LB, int NT, int CM, int E>
constexpr int lo_min_waves() {
  // two complex128 workgroups per CU (4 waves per SIMD) where the registers allow it without
  // spilling: the extension's loads would otherwise push the global-drive forms past 128
  return sizeof(R) == 8 && LB == 12 && NT == 512 && CM != kCoefSite ? 4 : 1;
}

// Which tile positions a thread holds.  The extended low pass issues about ten vector
// memory instructions per amplitude (its tile, t, the diagonal table, the extension's
// neighbours, the store).  With 8-byte complex64 accesses the vector memory unit's address
// stage was busy 86 % of the pass (TA_BUSY) while the bytes ran below the copy ceiling, so
// there a thread holds pairs of adjacent amplitudes and every access moves 16 bytes per lane:
// the register bits below VB are the lowest tile bits, then come the thread bits, then the
// other register bits.  At 27 atoms this took the complex64 low pass from 0.91 to 0.76 ms.
// (VB = 0 for complex128, whose amplitude is already 16 bytes, and for the unextended
// complex64 tiles, where the pairs would cost registers the wide tiles do not have.)
template <class R, int A, int E>
constexpr int lo_vec_bits() { return sizeof(R) == 4 && A >= 2 && E > 0 ? 1 : 0; }

// Tile position of register slot s of thread tid.
template <int TB, int VB>
__device__ __forceinline__ uint32_t lo_pos(uint32_t tid, int s) {
  // (sums rather than ors: tid < 2^TB, and the compiler then folds the slot part into the
  // immediate offsets of the accesses)
  return (tid << VB) + (uint32_t)(s & ((1 << VB) - 1)) + ((uint32_t)(s >> VB) << (TB + VB));
}

// Tile-position bit of register bit q.
template <int TB, int VB>
constexpr int lo_reg_bit(int q) { return q < VB ? q : q + TB; }

typedef float lo_f4 __attribute__((ext_vector_type(4)));
typedef float lo_f2 __attribute__((ext_vector_type(2)));

// r[0 .. 2^VB) = the 2^VB adjacent amplitudes at p (aligned to 2^VB amplitudes); nt: a
// non-temporal load.
template <class R, int VB>
__device__ __forceinline__ void ld_run(const Cx<R>* p, Cx<R>* r, bool nt = false) {
  if constexpr (VB == 0) {
    if (nt) {
      r[0].x = __builtin_nontemporal_load(&p->x);
      r[0].y = __builtin_nontemporal_load(&p->y);
    } else {
      r[0] = *p;
    }
  } else {
    static_assert(sizeof(R) == 4 && VB == 1, "pairs of complex64 amplitudes only");
    if (nt) {
      // (two 8-byte non-temporal loads, which the compiler joins into one 16-byte access;
      // a non-temporal load of the 16-byte vector type loses the hint)
      const double* q = reinterpret_cast<const double*>(p);
      const lo_f2 a = __builtin_bit_cast(lo_f2, __builtin_nontemporal_load(q));
      const lo_f2 b = __builtin_bit_cast(lo_f2, __builtin_nontemporal_load(q + 1));
      r[0] = Cx<R>{a.x, a.y};
      r[1] = Cx<R>{b.x, b.y};
    } else {
      const lo_f4 w = *reinterpret_cast<const lo_f4*>(p);
      r[0] = Cx<R>{w.x, w.y};
      r[1] = Cx<R>{w.z, w.w};
    }
  }
}

// The 2^VB adjacent amplitudes at p (aligned) = r[0 .. 2^VB).
template <class R, int VB>
__device__ __forceinline__ void st_run(Cx<R>* p, const Cx<R>* r, int streaming) {
  if constexpr (VB == 0) {
    put(p, r[0], streaming);
  } else {
    lo_f4* q = reinterpret_cast<lo_f4*>(p);
    const lo_f4 w = {r[0].x, r[0].y, r[1].x, r[1].y};
    if (streaming) {
      __builtin_nontemporal_store(w, q);
    } else {
      *q = w;
    }
  }
}

// E > 0: the pass also flips the E amplitude bits LB + g0 .. LB + g0 + E - 1 (g0 =
// p.ext_bit; the planner puts them at the top), whose neighbours lie in E other tiles of the
// same group of 2^E tiles (those differing in tile-index bits g0 .. g0 + E - 1).  Those are
// read straight from global memory (the input is then a stored vector): a group's tiles take
// consecutive positions on one XCD, so most of these reads are served by its L2 or the
// last-level cache rather than HBM.
template <class R, int LB, int NT, int CM, int E>
__global__ __launch_bounds__(NT, (lo_min_waves<R, LB, NT, CM, E>())) void hpsi_lo_kernel(const StepCoef c, const PassArgs<R> p) {
  using C = Cx<R>;
  constexpr int TB = ilog2(NT);      // thread-index bits
  static_assert(LB >= TB, "tile smaller than the workgroup");
  constexpr int A = 1 << (LB - TB);  // amplitudes per thread
  constexpr int RB = LB - TB;        // bits held in registers
  constexpr int VB = lo_vec_bits<R, A, E>();
  constexpr int V = 1 << VB;         // adjacent amplitudes per access
  __shared__ __align__(16) C tile[1 << LB];
  __shared__ R lut[CM == kCoefSite ? 1024 : 1];
  __shared__ double red[NT / 64];

  const uint32_t tid = threadIdx.x;
  uint32_t blk = xcd_remap(blockIdx.x, p.nblk);
  if constexpr (E > 0) {
    // position -> tile: the low E bits of the position pick the tile within its group
    const uint32_t g0 = p.ext_bit, h = blk & ((1u << E) - 1u), rest = blk >> E;
    blk = (rest & ((1u << g0) - 1u)) | (h << g0) | ((rest >> g0) << (g0 + E));
  }
  const uint32_t base = blk << LB;
  if (CM == kCoefSite) build_delta_lut<R>(c, lut);

  const Coefs co = input_coefs(p);
  C v[A], tv[A];
  R dg[A];
  double nrm = 0.0;
  // every operand is requested before the barrier, so the loads of the high-pass partial
  // and the diagonal table overlap those of the state
  const double* et = p.etile + (size_t)blk * (LB + 1);
  double eth = et[0];  // the tile's high-bit pairs plus the couplings of the thread bits
#pragma unroll
  for (int q = 0; q < TB; ++q)
    if ((tid >> q) & 1u) eth += et[1 + VB + q];
  // (the input test sits outside the loops, so that the loads of a stored input are issued
  // back to back rather than one branch at a time)
  if (!p.x1 && !p.x2 && co.a0 == 1.0) {
#pragma unroll
    for (int s = 0; s < A; s += V) ld_run<R, VB>(&p.x0[base + lo_pos<TB, VB>(tid, s)], &v[s]);
  } else {
#pragma unroll
    for (int s = 0; s < A; ++s) v[s] = form<R>(p, co, base + lo_pos<TB, VB>(tid, s));
  }
  if (p.tb) {
    // the high-pass partial is read once: a non-temporal load keeps it from displacing the
    // state tiles that neighbouring workgroups read through the cache
#pragma unroll
    for (int s = 0; s < A; s += V) ld_run<R, VB>(&p.tb[base + lo_pos<TB, VB>(tid, s)], &tv[s], true);
  } else {
#pragma unroll
    for (int s = 0; s < A; ++s) tv[s] = C{0, 0};
  }
#pragma unroll
  for (int s = 0; s < A; ++s) {
    double es = eth;
#pragma unroll
    for (int q = 0; q < RB; ++q)
      if ((s >> q) & 1) es += et[1 + lo_reg_bit<TB, VB>(q)];
    dg[s] = (R)(p.elo[lo_pos<TB, VB>(tid, s)] + es);
  }
#pragma unroll
  for (int s = 0; s < A; ++s) tile[lo_pos<TB, VB>(tid, s)] = v[s];
  if (p.u_out) {
#pragma unroll
    for (int s = 0; s < A; s += V) st_run<R, VB>(&p.u_out[base + lo_pos<TB, VB>(tid, s)], &v[s], p.streaming);
#pragma unroll
    for (int s = 0; s < A; ++s) nrm = norm_add(nrm, (double)v[s].x, (double)v[s].y);
  }
  // flips of the bits above the tile: bit LB + tb of every amplitude here is bit tb of the
  // tile index, so its coefficient is the same for the whole workgroup; the terms join the
  // high-pass partial (requested before the barrier, like the tile).  The loads of one bit
  // are issued together into their own registers before any is used: written as one
  // load-and-add per amplitude, the compiler issues them one at a time at this register
  // budget, which made the pass about 30 % slower.
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int tb = p.ext_bit + j;  // tile-index bit
    const bool bit = (blk >> tb) & 1u;
    const int q = CM == kCoefSite ? LB + tb : 0;
    const R cr = (R)(bit ? c.up_re[q] : c.dn_re[q]);
    const R ci = (R)(bit ? c.up_im[q] : c.dn_im[q]);
    const uint32_t nbase = (blk ^ (1u << tb)) << LB;
    C nb[A];
#pragma unroll
    for (int s = 0; s < A; s += V) ld_run<R, VB>(&p.x0[nbase + lo_pos<TB, VB>(tid, s)], &nb[s]);
#pragma unroll
    for (int s = 0; s < A; ++s) {
      tv[s].x += cr * nb[s].x - ci * nb[s].y;
      tv[s].y += cr * nb[s].y + ci * nb[s].x;
    }
  }
  __syncthreads();
  if constexpr (E > 0) {
    // the thread's own amplitudes come back from the tile: not holding them in registers
    // across the barrier leaves room for the neighbour loads to be in flight together
#pragma unroll
    for (int s = 0; s < A; ++s) v[s] = tile[lo_pos<TB, VB>(tid, s)];
  }

  double dot = 0.0;
  if constexpr (CM == kCoefSite) {
    // per-site couplings: a thread-index bit has the same level in all of this thread's
    // amplitudes, so its coefficient is chosen once and applied to all of them
    C acc[A];
#pragma unroll
    for (int s = 0; s < A; ++s) {
      const R d = dg[s] + detuning<R, CM>(c, lut, base + lo_pos<TB, VB>(tid, s));
      acc[s] = C{d * v[s].x, d * v[s].y};
    }
#pragma unroll
    for (int q = 0; q < TB; ++q) {
      const bool bit = (tid >> q) & 1u;
      const R cr = (R)(bit ? c.up_re[VB + q] : c.dn_re[VB + q]);
      const R ci = (R)(bit ? c.up_im[VB + q] : c.dn_im[VB + q]);
#pragma unroll
      for (int s = 0; s < A; ++s) {
        const C nb = tile[lo_pos<TB, VB>(tid, s) ^ (1u << (VB + q))];
        acc[s].x += cr * nb.x - ci * nb.y;
        acc[s].y += cr * nb.y + ci * nb.x;
      }
    }
#pragma unroll
    for (int s = 0; s < A; ++s) {
#pragma unroll
      for (int q = 0; q < RB; ++q)
        cmad<R>(acc[s], c, lo_reg_bit<TB, VB>(q), (s >> q) & 1, v[s ^ (1 << q)]);
      if (E > 0 || p.tb) cadd<R>(acc[s], tv[s]);
      dot += (double)v[s].x * (double)acc[s].x + (double)v[s].y * (double)acc[s].y;
    }
#pragma unroll
    for (int s = 0; s < A; s += V) st_run<R, VB>(&p.out[base + lo_pos<TB, VB>(tid, s)], &acc[s], p.streaming);
  } else {
#pragma unroll
    for (int s0 = 0; s0 < A; s0 += V) {
      C acc[V];
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int s = s0 + k;
        const uint32_t e = lo_pos<TB, VB>(tid, s);
        const R d = dg[s] + detuning<R, CM>(c, lut, base + e);
        acc[k] = C{d * v[s].x, d * v[s].y};
        DriveSum<R, CM> ds;
#pragma unroll
        for (int q = 0; q < TB; ++q) ds.add(c, VB + q, (tid >> q) & 1, tile[e ^ (1u << (VB + q))]);
#pragma unroll
        for (int q = 0; q < RB; ++q) ds.add(c, lo_reg_bit<TB, VB>(q), (s >> q) & 1, v[s ^ (1 << q)]);
        ds.finish(c, acc[k]);
        if (E > 0 || p.tb) cadd<R>(acc[k], tv[s]);
        if constexpr (V == 1) put(&p.out[base + e], acc[0], p.streaming);
        dot += (double)v[s].x * (double)acc[k].x + (double)v[s].y * (double)acc[k].y;
      }
      if constexpr (V > 1) st_run<R, VB>(&p.out[base + lo_pos<TB, VB>(tid, s0)], acc, p.streaming);
    }
  }
  if (p.part_norm) {
    const double t = wg_sum<NT>(nrm, red);
    if (tid == 0) p.part_norm[blockIdx.x] = t;
  }
  if (p.part_dot) {
    const double t = wg_sum<NT>(dot, red);
    if (tid == 0) p.part_dot[blockIdx.x] = t;
  }
}

// ----------------------------------------------------------------------------- small n
// n < 8: one workgroup, one amplitude per thread, every flip through LDS.
template <class R, int CM>
__global__ __launch_bounds__(kBlock) void hpsi_small_kernel(const StepCoef c, const PassArgs<R> p) {
  using C = Cx<R>;
  __shared__ C tile[128];
  __shared__ R lut[CM == kCoefSite ? 1024 : 1];
  __shared__ double red[4];
  const uint32_t tid = threadIdx.x;
  const uint32_t dim = 1u << c.n;
  if (CM == kCoefSite) build_delta_lut<R>(c, lut);
  C v = {0, 0};
  double nrm = 0.0, dot = 0.0;
  if (tid < dim) {
    v = form<R>(p, input_coefs(p), tid);
    tile[tid] = v;
    if (p.u_out) {
      p.u_out[tid] = v;
      nrm = norm_add(0.0, (double)v.x, (double)v.y);
    }
  }
  __syncthreads();
  if (tid < dim) {
    const R d = (R)(p.elo[tid] + p.etile[0]) + detuning<R, CM>(c, lut, tid);
    C acc = {d * v.x, d * v.y};
    DriveSum<R, CM> ds;
    for (int q = 0; q < c.n; ++q) ds.add(c, q, (tid >> q) & 1, tile[tid ^ (1u << q)]);
    ds.finish(c, acc);
    p.out[tid] = acc;
    dot = (double)v.x * (double)acc.x + (double)v.y * (double)acc.y;
  }
  if (p.part_norm) {
    const double t = block_sum_256(nrm, red);
    if (tid == 0) p.part_norm[0] = t;
  }
  if (p.part_dot) {
    const double t = block_sum_256(dot, red);
    if (tid == 0) p.part_dot[0] = t;
  }
}

// ----------------------------------------------------------------------------- high pass
// Tile: bits [0, RL) and [a, a + HB - RL) of the index; flips bits in [f0, f1) only.
template <class R, int HB, int RL, int NT, int CM>
__global__ __launch_bounds__(NT) void hpsi_hi_kernel(const StepCoef c, const PassArgs<R> p) {
  using C = Cx<R>;
  constexpr int G = HB - RL;
  constexpr int TB = ilog2(NT);
  static_assert(HB >= TB && TB > RL, "tile shape");
  constexpr int A = 1 << (HB - TB);
  __shared__ C tile[1 << HB];
  __shared__ double red[NT / 64];

  const uint32_t tid = threadIdx.x;
  const uint32_t blk = xcd_remap(blockIdx.x, p.nblk);
  const int gap = p.a - RL;  // outside bits between the contiguous run and the tile's high bits
  const uint32_t obase = ((blk & ((1u << gap) - 1u)) << RL) | ((blk >> gap) << (p.a + G));

  const Coefs co = input_coefs(p);
  C v[A], tv[A];
  uint32_t gi[A];
  double nrm = 0.0;
  // the partial being accumulated is requested with the state, before the barrier
  // (one amplitude's vectors after another: issuing each vector's loads for the whole tile
  // first measured slower here, 16 % for complex64 on the top bits)
#pragma unroll
  for (int s = 0; s < A; ++s) {
    const uint32_t e = tid + NT * s;
    gi[s] = obase | (e & ((1u << RL) - 1u)) | ((e >> RL) << p.a);
    v[s] = form<R>(p, co, gi[s]);
    tv[s] = p.accumulate ? p.tb[gi[s]] : C{0, 0};
  }
#pragma unroll
  for (int s = 0; s < A; ++s) tile[tid + NT * s] = v[s];
  if (p.u_out) {
#pragma unroll
    for (int s = 0; s < A; ++s) {
      put(&p.u_out[gi[s]], v[s], p.streaming);
      nrm = norm_add(nrm, (double)v[s].x, (double)v[s].y);
    }
  }
  __syncthreads();

#pragma unroll
  for (int s = 0; s < A; ++s) {
    const uint32_t e = tid + NT * s;
    C acc = {0, 0};
    DriveSum<R, CM> ds;
#pragma unroll
    for (int eb = RL; eb < HB; ++eb) {
      const int q = p.a + eb - RL;
      if (q < p.f0 || q >= p.f1) continue;
      const C nb = eb < TB ? tile[e ^ (1u << eb)] : v[s ^ (1 << (eb - TB))];
      ds.add(c, q, (e >> eb) & 1u, nb);
    }
    ds.finish(c, acc);
    if (p.accumulate) cadd<R>(acc, tv[s]);
    put(&p.tb[gi[s]], acc, p.streaming);
  }
  if (p.part_norm) {
    const double t = wg_sum<NT>(nrm, red);
    if (tid == 0) p.part_norm[blockIdx.x] = t;
  }
}

template <class R, int LB, int CM, int E = 0>
void launch_lo(const StepCoef& c, PassArgs<R> p, int n, hipStream_t s) {
  constexpr int NT = lo_threads<R, CM, LB, E>() < (1 << LB) ? lo_threads<R, CM, LB, E>() : (1 << LB);
  p.nblk = 1u << (n - LB);
  hipLaunchKernelGGL((hpsi_lo_kernel<R, LB, NT, CM, E>), dim3(p.nblk), dim3(NT), 0, s, c, p);
}

template <class R, int CM, int LB>
void launch_lo_ext(int ext, const StepCoef& c, const PassArgs<R>& p, int n, hipStream_t s) {
  static_assert(kMaxLoExt == 7, "launch_lo_ext instantiates extensions 1..7");
  switch (ext) {
    case 1: launch_lo<R, LB, CM, 1>(c, p, n, s); break;
    case 2: launch_lo<R, LB, CM, 2>(c, p, n, s); break;
    case 3: launch_lo<R, LB, CM, 3>(c, p, n, s); break;
    case 4: launch_lo<R, LB, CM, 4>(c, p, n, s); break;
    case 5: launch_lo<R, LB, CM, 5>(c, p, n, s); break;
    case 6: launch_lo<R, LB, CM, 6>(c, p, n, s); break;
    default: launch_lo<R, LB, CM, 7>(c, p, n, s); break;
  }
}

template <class R, int CM>
void launch_lo_any(int lb, int ext, const StepCoef& c, const PassArgs<R>& p, int n, hipStream_t s) {
  if (ext > 0) {  // extensions are planned on 12-bit tiles, and complex64's 13-bit ones
    if constexpr (Geo<R>::L >= 13) {
      if (lb == 13) return launch_lo_ext<R, CM, 13>(ext, c, p, n, s);
    }
    return launch_lo_ext<R, CM, 12>(ext, c, p, n, s);
  }
  switch (lb) {
    case 8: launch_lo<R, 8, CM>(c, p, n, s); break;
    case 9: launch_lo<R, 9, CM>(c, p, n, s); break;
    case 10: launch_lo<R, 10, CM>(c, p, n, s); break;
    case 11: launch_lo<R, 11, CM>(c, p, n, s); break;
    case 12: launch_lo<R, 12, CM>(c, p, n, s); break;
    default:
      if constexpr (Geo<R>::L >= 13) launch_lo<R, 13, CM>(c, p, n, s);
      break;
  }
}

template <class R, int CM>
void launch_hi(int rl, const StepCoef& c, const PassArgs<R>& p, hipStream_t s) {
  constexpr int HB = Geo<R>::H, NT = Geo<R>::NH;
  switch (rl) {
    case 3: hipLaunchKernelGGL((hpsi_hi_kernel<R, HB, 3, NT, CM>), dim3(p.nblk), dim3(NT), 0, s, c, p); break;
    case 4: hipLaunchKernelGGL((hpsi_hi_kernel<R, HB, 4, NT, CM>), dim3(p.nblk), dim3(NT), 0, s, c, p); break;
    case 5: hipLaunchKernelGGL((hpsi_hi_kernel<R, HB, 5, NT, CM>), dim3(p.nblk), dim3(NT), 0, s, c, p); break;
    default: hipLaunchKernelGGL((hpsi_hi_kernel<R, HB, 6, NT, CM>), dim3(p.nblk), dim3(NT), 0, s, c, p); break;
  }
}

template <class R, int CM>
hipError_t sweep_t(int n, const StepCoef& c, const double* dtab, const SweepIn& in, void* out,
                   void* tbuf, const SweepOut& so, int part, hipStream_t s) {
  PassArgs<R> base{};
  base.x0 = (const Cx<R>*)in.x0;
  base.x1 = (const Cx<R>*)in.x1;
  base.x2 = (const Cx<R>*)in.x2;
  base.a0 = in.a0;
  base.a1 = in.a1;
  base.a2 = in.a2;
  base.dot = in.dot;
  base.dot_coef = in.dot_coef;
  base.nrm1 = in.nrm1;
  base.nrm2 = in.nrm2;
  const int lbits = make_tile_plan(sizeof(R) == 8 ? kC128 : kC64, n).lo_bits;
  base.elo = dtab;
  base.etile = dtab + (size_t(1) << lbits);
  base.out = (Cx<R>*)out;
  // vectors of 64 MiB and more stream past the caches: a Lanczos iteration touches five of
  // them, more than the 256 MB last-level cache holds (from 64 MiB rather than 256 MiB the
  // step measured 1.5-2.5 % faster at 22-24 atoms)
  base.streaming = (size_t(1) << n) * sizeof(Cx<R>) >= (size_t(64) << 20);

  const bool first = part != kLaterPasses, later = part != kFirstPass;
  if (n < 8) {
    if (!first) return hipSuccess;
    PassArgs<R> p = base;
    p.u_out = (Cx<R>*)so.u_out;
    p.part_norm = so.part_norm;
    p.part_dot = so.part_dot;
    hipLaunchKernelGGL((hpsi_small_kernel<R, CM>), dim3(1), dim3(kBlock), 0, s, c, p);
    return hipGetLastError();
  }
  const TilePlan plan = make_tile_plan(sizeof(R) == 8 ? kC128 : kC64, n);
  // the formed input, once stored, is the plain input of every later pass
  const bool forming = in.x1 || in.x2 || in.a0 != 1.0 || in.dot || in.nrm1;
  if (forming && plan.n_hi_passes > 0 && !so.u_out) return hipErrorInvalidValue;
  const Cx<R>* stored = so.u_out ? (const Cx<R>*)so.u_out : (const Cx<R>*)in.x0;
  for (int i = 0; i < plan.n_hi_passes; ++i) {
    if ((i == 0 && !first) || (i > 0 && !later)) continue;
    PassArgs<R> p = base;
    if (i > 0) {
      p.x0 = stored;
      p.x1 = p.x2 = nullptr;
      p.a0 = 1.0;
      p.dot = nullptr;
      p.nrm1 = p.nrm2 = nullptr;
    } else {
      p.u_out = (Cx<R>*)so.u_out;
      p.part_norm = so.part_norm;
    }
    p.tb = (Cx<R>*)tbuf;
    p.accumulate = i > 0 ? 1 : 0;
    p.a = plan.tile_a[i];
    p.f0 = plan.flip_lo[i];
    p.f1 = plan.flip_hi[i];
    p.nblk = 1u << (n - plan.hi_bits);
    launch_hi<R, CM>(plan.run_bits[i], c, p, s);
  }
  if ((plan.n_hi_passes > 0 && !later) || (plan.n_hi_passes == 0 && !first)) return hipGetLastError();
  PassArgs<R> p = base;
  if (plan.n_hi_passes > 0) {
    p.x0 = stored;
    p.x1 = p.x2 = nullptr;
    p.a0 = 1.0;
    p.dot = nullptr;
    p.nrm1 = p.nrm2 = nullptr;
    p.tb = (Cx<R>*)tbuf;
  } else {
    p.u_out = (Cx<R>*)so.u_out;
    p.part_norm = so.part_norm;
  }
  p.part_dot = so.part_dot;
  // an extended low pass reads the neighbouring tiles of a stored input
  if (plan.lo_ext > 0 && ((plan.lo_bits != 12 && plan.lo_bits != Geo<R>::L) ||
                          plan.n_hi_passes == 0 || p.x1 || p.x2 || p.a0 != 1.0 || p.dot || p.nrm1))
    return hipErrorInvalidValue;
  p.ext_bit = plan.lo_ext_bit - plan.lo_bits;
  launch_lo_any<R, CM>(plan.lo_bits, plan.lo_ext, c, p, n, s);
  return hipGetLastError();
}

template <class R>
hipError_t sweep_r(int n, const StepCoef& c, const double* dtab, const SweepIn& in, void* out,
                   void* tbuf, const SweepOut& so, int part, hipStream_t s) {
  switch (c.mode) {
    case kCoefReal: return sweep_t<R, kCoefReal>(n, c, dtab, in, out, tbuf, so, part, s);
    case kCoefSite: return sweep_t<R, kCoefSite>(n, c, dtab, in, out, tbuf, so, part, s);
    default: return sweep_t<R, kCoefUniform>(n, c, dtab, in, out, tbuf, so, part, s);
  }
}

}  // namespace

TilePlan make_tile_plan(int prec, int n) {
  TilePlan p{};
  p.n = n;
  const int L = prec == kC128 ? Geo<double>::L : Geo<float>::L;
  const int rl = prec == kC128 ? Geo<double>::RL : Geo<float>::RL;
  const int rlw = prec == kC128 ? Geo<double>::RLW : Geo<float>::RLW;
  p.hi_bits = prec == kC128 ? Geo<double>::H : Geo<float>::H;
  p.lo_bits = n < L ? n : L;
  // complex64 takes 12-bit low tiles where the extension then leaves a single high pass (22..28
  // atoms): its 13-bit tiles hold 16 amplitudes per thread, whose registers allow one
  // workgroup per CU, and the extended pass measured about 12 % faster on the smaller tile
  if (prec != kC128 && n - 12 > p.hi_bits - rl && n - 12 <= p.hi_bits - rl + kMaxLoExt)
    p.lo_bits = 12;
  p.n_hi_passes = 0;
  p.lo_ext = 0;
  p.lo_ext_bit = p.lo_bits;
  const int rest = n - p.lo_bits;  // bits above the low-pass tile
  if (rest <= 0) return p;
  // fewest passes at the shortest run
  const int per = p.hi_bits - rl;
  int passes = (rest + per - 1) / per;
  // the low pass can flip up to kMaxLoExt more bits from the neighbouring tiles; where that
  // saves a high pass it takes the fewest bits that do, plus one (a longer run for the
  // high pass costs less than the one more neighbour tile)
  if (passes >= 2) {
    const int fewer = (rest - kMaxLoExt + per - 1) / per;
    if (fewer < passes) {
      const int emin = rest - fewer * per;
      p.lo_ext = emin < kMaxLoExt ? emin + 1 : emin;
      passes = fewer;
    }
  }
  // the extension takes the top bits and the high passes the bits between: the forming pass
  // over bits 12..19 measured 5 % faster than over the top bits (its tile then spans 16 MB
  // rather than the whole vector), and the low pass's groups keep their size either way
  const int top = n - p.lo_ext;
  if (p.lo_ext > 0) p.lo_ext_bit = top;
  // then the spare tile bits lengthen the runs (the first, forming pass first: it moves the
  // most bytes), up to rlw each
  int spare = passes * per - (rest - p.lo_ext);
  int f0 = p.lo_bits;
  for (int i = 0; i < passes; ++i) {
    const int more = (spare + (passes - i) - 1) / (passes - i);  // spread, rounding up first
    const int r = rl + more < rlw ? rl + more : rlw;
    spare -= r - rl;
    const int gw = p.hi_bits - r;
    const int f1 = f0 + gw < top ? f0 + gw : top;
    int a = f0;
    if (a + gw > n) a = n - gw;  // keep the whole tile inside the index; extra bits are not flipped
    p.flip_lo[i] = f0;
    p.flip_hi[i] = f1;
    p.tile_a[i] = a;
    p.run_bits[i] = r;
    ++p.n_hi_passes;
    f0 = f1;
  }
  return p;
}

int64_t sweep_num_partials(int prec, int n) {
  if (n < 8) return 1;
  const TilePlan p = make_tile_plan(prec, n);
  const int64_t lo = int64_t(1) << (n - p.lo_bits);
  const int64_t hi = p.n_hi_passes ? int64_t(1) << (n - p.hi_bits) : 0;
  return lo > hi ? lo : hi;
}

int64_t sweep_norm_partials(int prec, int n) {
  if (n < 8) return 1;
  const TilePlan p = make_tile_plan(prec, n);
  return p.n_hi_passes ? int64_t(1) << (n - p.hi_bits) : int64_t(1) << (n - p.lo_bits);
}

int64_t sweep_dot_partials(int prec, int n) {
  if (n < 8) return 1;
  const TilePlan p = make_tile_plan(prec, n);
  return int64_t(1) << (n - p.lo_bits);
}

int sweep_passes(int prec, int n) {
  if (n < 8) return 1;
  return 1 + make_tile_plan(prec, n).n_hi_passes;
}

hipError_t hpsi_sweep(int prec, int n, const StepCoef& c, const double* dtab, const SweepIn& in,
                      void* out, void* tbuf, const SweepOut& so, int part, hipStream_t s) {
  if (prec == kC128) return sweep_r<double>(n, c, dtab, in, out, tbuf, so, part, s);
  return sweep_r<float>(n, c, dtab, in, out, tbuf, so, part, s);
}

}  // namespace rsv
