// Packed small-job evolution: one workgroup per job runs the whole time evolution of a
// small register (2^n amplitudes held by the workgroup) without host round trips.
//
// Each step is the same method as the host-driven path (Sec. III and III.A): midpoint
// parameters of step k, Lanczos recurrence with FP64 reductions, the a-posteriori estimate
// beta_{m-1} |[exp(-i dt T_m) e_1]_{m-1}| |psi| <= tol, sub-steps on non-convergence, and
// psi <- |psi| sum_l y_l v_l.  Only the small exponential differs: instead of the host
// eigendecomposition, y = exp(-i tau T) e_1 is evaluated on the device by the Chebyshev
// expansion
//   exp(-i a x) = J_0(a) + 2 sum_{k>=1} (-i)^k J_k(a) T_k(x),   x in [-1, 1],
// applied to X = (T - c)/r with c, r from Gershgorin bounds and a = tau r (Bessel
// coefficients by Miller's backward recurrence normalised with J_0 + 2 sum J_2k = 1).  One
// wave evaluates it, lane i holding row i of T (m <= 64).  The series is capped at
// kMaxBessel terms; a step whose tau r exceeds what that resolves is shortened (halved
// until it fits) before the estimate is tested, which only adds sub-steps.
//
// Krylov vectors of a job live in global memory (L2-resident at these sizes); the newest
// one is kept in the LDS tile, where the level swaps read it, and H u in registers.
#include "device_common.h"
#include "packed.h"

namespace rsv {
namespace {

constexpr int kThreadBits = 9;
constexpr int kThreads = 1 << kThreadBits;
constexpr int kWaves = kThreads / 64;
constexpr int kMaxBessel = 512;

template <class R> struct PackGeo;
template <> struct PackGeo<double> { static constexpr int A = 8; };   // n <= 12
template <> struct PackGeo<float> { static constexpr int A = 16; };   // n <= 13

__device__ __forceinline__ double wg_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double r = 0.0;
#pragma unroll
  for (int w = 0; w < kWaves; ++w) r += red[w];
  __syncthreads();
  return r;
}

struct Shared {
  double alpha[kMaxKrylov + 1], beta[kMaxKrylov + 1], scale[kMaxKrylov + 1];
  double yre[kMaxKrylov], yim[kMaxKrylov];
  double bessel[kMaxBessel + 1];
  double dl[kMaxAtoms];  // detuning of bit p at the current step
  double red[kWaves];
  double est, cheb_c, cheb_r;
  int cheb_k;
};

// Midpoint value of step k (Sec. III): mean of the samples at floor(m) and ceil(m),
// m = (k + 1/2) dt in ns.
__device__ __forceinline__ double midpoint(const double* x, long k, int dt_ns) {
  const long twice = (2 * k + 1) * (long)dt_ns;
  return 0.5 * (x[twice / 2] + x[(twice + 1) / 2]);
}

// y = exp(-i tau T_m) e_1 (all m rows into sh.yre / sh.yim when full, else |y_{m-1}| into
// sh.est).  Called by every thread of the workgroup; thread 0 computes the Bessel
// coefficients, wave 0 runs the Chebyshev recurrence with lane i holding row i.  Returns
// false (and est = inf) when tau times the spectral half-width of T_m needs more than
// kMaxBessel terms: the caller shortens tau.
__device__ bool cheb_expm(Shared& sh, int m, double tau, bool full) {
  const int tid = threadIdx.x, lane = tid & 63;
  if (tid == 0) {
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < m; ++i) {
      const double bl = i > 0 ? fabs(sh.beta[i - 1]) : 0.0;
      const double br = i + 1 < m ? fabs(sh.beta[i]) : 0.0;
      lo = fmin(lo, sh.alpha[i] - bl - br);
      hi = fmax(hi, sh.alpha[i] + bl + br);
    }
    const double c = 0.5 * (hi + lo), r = 0.5 * (hi - lo);
    sh.cheb_c = c;
    sh.cheb_r = r;
    int K = -1;  // -1: T is numerically a multiple of the identity; -2: series too long
    if (r > 1e-300 && tau * r > 1e-30) {
      const double a = tau * r;
      // terms: J_k(a) <= (a/2)^k / k! bounds the tail for small a; a + 8 a^(1/3) + 20 for
      // large a (both leave a tail below 1e-15)
      K = (int)(a + 8.0 * cbrt(a) + 20.0);
      double bound = 1.0;
      for (int k = 1; k < K; ++k) {
        bound *= 0.5 * a / k;
        if (k > 0.5 * a + 1.0 && bound < 1e-17) {
          K = k;
          break;
        }
      }
      if (K > kMaxBessel - 1) {
        sh.cheb_k = -2;
        K = -3;
      }
    }
    if (K >= 0) {
      const double a = tau * r;
      // Miller's backward recurrence for J_0..J_K(a), normalised by J_0 + 2 sum J_2k = 1
      const int M = K + 24 + (int)sqrt(40.0 * (K + 1));
      const double two_over_a = 2.0 / a;
      double jp = 0.0, j = 1e-280, norm = 0.0;
      for (int k = 0; k <= K; ++k) sh.bessel[k] = 0.0;
      for (int k = M; k >= 1; --k) {
        if (k <= K) sh.bessel[k] = j;
        if (!(k & 1)) norm += 2.0 * j;
        const double jm = (k * two_over_a) * j - jp;
        jp = j;
        j = jm;
        if (fabs(j) > 1e200) {  // rescale everything recurred so far
          j *= 1e-200;
          jp *= 1e-200;
          norm *= 1e-200;
          for (int q = k; q <= K; ++q) sh.bessel[q] *= 1e-200;
        }
      }
      norm += j;
      sh.bessel[0] = j;
      const double inv = 1.0 / norm;
      for (int k = 0; k <= K; ++k) sh.bessel[k] *= inv;
    }
    if (K != -3) sh.cheb_k = K;
  }
  __syncthreads();
  const int K = sh.cheb_k;  // every thread reads it before the closing barrier
  if (tid < 64) {
    const bool live = lane < m;
    const double c = sh.cheb_c, r = sh.cheb_r;
    const double a_i = live ? sh.alpha[lane] : 0.0;
    const double bl = (live && lane > 0) ? sh.beta[lane - 1] : 0.0;
    const double br = (live && lane + 1 < m) ? sh.beta[lane] : 0.0;
    double yr = 0.0, yi = 0.0;
    if (K == -2) {  // not resolvable with kMaxBessel terms: report "not converged"
      yr = __builtin_inf();
    } else if (K < 0) {
      yr = lane == 0 ? 1.0 : 0.0;
    } else {
      // t_0 = e_1, t_1 = X e_1, t_{k+1} = 2 X t_k - t_{k-1};  X = (T - c) / r
      auto apply_x = [&](double t) {
        const double tm = __shfl_up(t, 1, 64);
        const double tp = __shfl_down(t, 1, 64);
        double v = (a_i - c) * t;
        if (lane > 0) v += bl * tm;
        if (lane < 63) v += br * tp;
        return live ? v / r : 0.0;
      };
      double t0 = lane == 0 ? 1.0 : 0.0;
      double t1 = apply_x(t0);
      yr = sh.bessel[0] * t0;
      for (int k = 1; k <= K; ++k) {
        const double w = 2.0 * sh.bessel[k] * t1;
        switch (k & 3) {  // (-i)^k
          case 0: yr += w; break;
          case 1: yi -= w; break;
          case 2: yr -= w; break;
          default: yi += w; break;
        }
        const double t2 = 2.0 * apply_x(t1) - t0;
        t0 = t1;
        t1 = t2;
      }
    }
    const double ph = -tau * c;
    const double er = cos(ph), ei = sin(ph);
    const double zr = er * yr - ei * yi, zi = er * yi + ei * yr;
    if (full) {
      if (live) {
        sh.yre[lane] = zr;
        sh.yim[lane] = zi;
      }
    } else if (lane == m - 1) {
      sh.est = hypot(zr, zi);
    }
  }
  __syncthreads();
  return K != -2;
}

template <class R>
__global__ __launch_bounds__(kThreads) void packed_evolve_kernel(const PackedJob* __restrict__ jobs) {
  using C = Cx<R>;
  constexpr int AMAX = PackGeo<R>::A;
  __shared__ C tile[kThreads * AMAX];  // the current Krylov vector u (each thread owns tile[e])
  __shared__ Shared sh;
  __shared__ R cf[4 * kMaxPackBits];   // couplings of bit p: <1|h|0> re, im, <0|h|1> re, im
  __shared__ R dg[kThreads * AMAX];    // diagonal of H_k
  const PackedJob& jb = jobs[blockIdx.x];
  const int n = jb.n;
  const uint32_t dim = 1u << n;
  const uint32_t tid = threadIdx.x;
  const int A = dim >= (uint32_t)kThreads ? (int)(dim / kThreads) : 1;
  C* psi = (C*)jb.psi;
  C* basis = (C*)jb.basis;
  const R* diag = (const R*)jb.diag;
  auto mine = [&](int s) { return s < A && tid + kThreads * s < dim; };

  C z[AMAX];  // H u of the newest Krylov vector
  // the diagonal of H_k lives in LDS (dg[e], written and read by the thread that owns e)
#pragma unroll
  for (int s = 0; s < AMAX; ++s) {
    z[s] = C{0, 0};
    const uint32_t e = tid + kThreads * s;
    if (mine(s)) tile[e] = jb.init_zero ? C{(R)(e == 0 ? 1 : 0), 0} : psi[e];
  }
  int64_t iters = 0, kmax_used = 0, substeps = 0;
  int m_prev = 0;  // Krylov dimension of the previous Lanczos run of this job
  int status = RSV_OK;
  const double tau = jb.dt_ns * 1e-3;

  // z = H u with u in the tile; returns Re<u, z>
  // element s of this thread is e = tid | s << 9: bits below 9 are the thread's, the others
  // are known at compile time in the unrolled loops
  auto apply_h = [&]() -> double {
    __syncthreads();
    double dot = 0.0;
    if (!jb.per_site) {
      // one coupling for every atom: sum the neighbours with the bit set and all of them,
      // then apply <1|h|0> and <0|h|1> once
      const R ur = cf[0], ui = cf[1], dr = cf[2], di = cf[3];
#pragma unroll
      for (int s = 0; s < AMAX; ++s) {
        const uint32_t e = tid | ((uint32_t)s << kThreadBits);
        if (mine(s)) {
          const C us = tile[e];
          C all = {0, 0}, one = {0, 0};
          for (int p = 0; p < n; ++p) {
            const C nb = tile[e ^ (1u << p)];
            all.x += nb.x;
            all.y += nb.y;
            if ((e >> p) & 1u) {
              one.x += nb.x;
              one.y += nb.y;
            }
          }
          const C zr = {all.x - one.x, all.y - one.y};
          C acc;
          const R de = dg[e];
          acc.x = de * us.x + (ur * one.x - ui * one.y) + (dr * zr.x - di * zr.y);
          acc.y = de * us.y + (ur * one.y + ui * one.x) + (dr * zr.y + di * zr.x);
          z[s] = acc;
          dot += (double)us.x * (double)acc.x + (double)us.y * (double)acc.y;
        }
      }
    } else {
#pragma unroll
      for (int s = 0; s < AMAX; ++s) {
        const uint32_t e = tid | ((uint32_t)s << kThreadBits);
        if (mine(s)) {
          const C us = tile[e];
          const R de = dg[e];
          C acc = {de * us.x, de * us.y};
          for (int p = 0; p < n; ++p) {
            const C nb = tile[e ^ (1u << p)];
            const int o = 4 * p + (((e >> p) & 1u) ? 0 : 2);
            const R cr = cf[o], ci = cf[o + 1];
            acc.x += cr * nb.x - ci * nb.y;
            acc.y += cr * nb.y + ci * nb.x;
          }
          z[s] = acc;
          dot += (double)us.x * (double)acc.x + (double)us.y * (double)acc.y;
        }
      }
    }
    return wg_sum(dot, sh.red);  // its barriers end every read of the tile
  };
  auto norm2 = [&]() -> double {
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < AMAX; ++s) {
      const uint32_t e = tid + kThreads * s;
      if (mine(s)) acc = norm_add(acc, (double)tile[e].x, (double)tile[e].y);
    }
    return wg_sum(acc, sh.red);
  };

  for (int64_t step = jb.first_step; step < jb.first_step + jb.n_steps && status == RSV_OK; ++step) {
    // coefficients of H_k by bit position p (atom n-1-p)
    if (tid < (uint32_t)n) {
      const int i = n - 1 - tid;
      const size_t off = jb.per_site ? (size_t)i * jb.n_samples : 0;
      const double om = midpoint(jb.omega + off, step, jb.dt_ns);
      const double de = midpoint(jb.delta + off, step, jb.dt_ns);
      const double ph = jb.phi ? midpoint(jb.phi + off, step, jb.dt_ns) : 0.0;
      cf[4 * tid] = (R)(0.5 * om * cos(ph));
      cf[4 * tid + 1] = (R)(-0.5 * om * sin(ph));
      cf[4 * tid + 2] = (R)(0.5 * om * cos(ph));
      cf[4 * tid + 3] = (R)(0.5 * om * sin(ph));
      sh.dl[tid] = de;
    }
    __syncthreads();
#pragma unroll
    for (int s = 0; s < AMAX; ++s) {
      const uint32_t e = tid + kThreads * s;
      double v = 0.0;
      if (mine(s)) {
        v = (double)diag[e];
        for (int p = 0; p < n; ++p)
          if ((e >> p) & 1u) v -= sh.dl[p];
      }
      dg[e] = (R)v;
    }

    double remaining = tau;
    while (remaining > 0.0 && status == RSV_OK) {
      const double nrm = sqrt(norm2());
      if (!(nrm > 0.0) || !isfinite(nrm)) {
        status = RSV_ENUMERIC;
        break;
      }
      if (tid == 0) sh.scale[0] = 1.0 / nrm;
#pragma unroll
      for (int s = 0; s < AMAX; ++s) {
        const uint32_t e = tid + kThreads * s;
        if (mine(s)) basis[e] = tile[e];
      }
      double dot = apply_h();  // z_0 = H u_0
      ++iters;
      int m = 0;
      // target: the part of the step this basis must resolve; shortened while the
      // exponential of the growing T_m is too wide for one Chebyshev series
      double target = remaining, sub = remaining;
      // the estimate is first tested two dimensions below the previous run's (every
      // dimension on the first run): a larger m than the smallest converged one is as exact
      const int k_test = m_prev > 3 ? m_prev - 2 : 1;
      for (int k = 1; k <= jb.kmax; ++k) {
        const double sk1 = sh.scale[k - 1];
        const double alpha = sk1 * sk1 * dot;
        const double c2 = k >= 2 ? -sh.scale[k - 2] / sk1 : 0.0;
        // u_k = s z - alpha s u_{k-1} - (s_{k-2}/s_{k-1}) u_{k-2}, rounded once, in place
#pragma unroll
        for (int s = 0; s < AMAX; ++s) {
          const uint32_t e = tid + kThreads * s;
          if (mine(s)) {
            const C u1 = tile[e];
            const C u2 = k >= 2 ? basis[(size_t)(k - 2) * dim + e] : C{0, 0};
            const double re = sk1 * (double)z[s].x - alpha * sk1 * (double)u1.x + c2 * (double)u2.x;
            const double im = sk1 * (double)z[s].y - alpha * sk1 * (double)u1.y + c2 * (double)u2.y;
            tile[e] = C{(R)re, (R)im};
          }
        }
        const double b2 = norm2();
        if (tid == 0) sh.alpha[k - 1] = alpha;
        __syncthreads();
        if (!isfinite(b2) || !isfinite(alpha)) {
          status = RSV_ENUMERIC;
          break;
        }
        const double bk = sqrt(b2);
        m = k;
        // the estimate meets the tolerance (always so at beta = 0, an invariant subspace)
        auto resolved = [&]() { return bk * sh.est * nrm <= jb.tol; };
        if (k >= k_test || k == jb.kmax || bk == 0.0) {
          bool fits = cheb_expm(sh, m, target, false);
          for (int h = 0; h < 64 && !fits; ++h) fits = cheb_expm(sh, m, target *= 0.5, false);
          if (!fits) {
            status = RSV_ENOTCONV;
            break;
          }
          if (resolved()) {
            sub = target;
            break;
          }
          if (k == jb.kmax || bk == 0.0) {
            // the longest part of the target this basis resolves: dyadic bracket, bisection
            bool ok = false;
            double bad = target;
            for (int dd = 1; dd <= jb.max_depth && !ok; ++dd) {
              sub = ldexp(target, -dd);
              cheb_expm(sh, m, sub, false);
              ok = resolved();
              __syncthreads();
              if (!ok) bad = sub;
            }
            if (!ok) {
              status = RSV_ENOTCONV;
              break;
            }
            for (int it = 0; it < 10; ++it) {
              const double mid = 0.5 * (sub + bad);
              cheb_expm(sh, m, mid, false);
              if (resolved()) sub = mid;
              else bad = mid;
              __syncthreads();
            }
            break;
          }
        }
        if (tid == 0) {
          sh.beta[k - 1] = bk;
          sh.scale[k] = 1.0 / bk;
        }
#pragma unroll
        for (int s = 0; s < AMAX; ++s) {
          const uint32_t e = tid + kThreads * s;
          if (mine(s)) basis[(size_t)k * dim + e] = tile[e];
        }
        __syncthreads();
        dot = apply_h();  // z_k = H u_k
        ++iters;
      }
      if (status != RSV_OK) break;
      kmax_used = max(kmax_used, (int64_t)m);
      m_prev = m;
      cheb_expm(sh, m, sub, true);
      // psi <- |psi| sum_l y_l s_l u_l over this thread's own amplitudes
#pragma unroll
      for (int s = 0; s < AMAX; ++s) {
        const uint32_t e = tid + kThreads * s;
        if (mine(s)) {
          double re = 0.0, im = 0.0;
          for (int l = 0; l < m; ++l) {
            const C x = basis[(size_t)l * dim + e];
            const double cr = nrm * sh.yre[l] * sh.scale[l], ci = nrm * sh.yim[l] * sh.scale[l];
            re += cr * (double)x.x - ci * (double)x.y;
            im += cr * (double)x.y + ci * (double)x.x;
          }
          tile[e] = C{(R)re, (R)im};
        }
      }
      __syncthreads();
      if (sub == remaining) {
        remaining = 0.0;
      } else {
        remaining -= sub;
        ++substeps;
      }
    }
  }
  // final state, occupations (FP64), bookkeeping
  double tot = 0.0, occ[kMaxPackBits];
#pragma unroll
  for (int p = 0; p < kMaxPackBits; ++p) occ[p] = 0.0;
#pragma unroll
  for (int s = 0; s < AMAX; ++s) {
    const uint32_t e = tid + kThreads * s;
    if (mine(s)) {
      const C v = tile[e];
      psi[e] = v;
      const double pr = norm_add(0.0, (double)v.x, (double)v.y);
      tot += pr;
#pragma unroll
      for (int p = 0; p < kMaxPackBits; ++p)
        if ((e >> p) & 1u) occ[p] += pr;
    }
  }
  const double total = wg_sum(tot, sh.red);
  for (int p = 0; p < n; ++p) {
    const double t = wg_sum(occ[p], sh.red);
    if (tid == 0) jb.out[kPackOccOffset + p] = t;
  }
  if (tid == 0) {
    jb.out[0] = status;
    jb.out[1] = (double)iters;
    jb.out[2] = (double)kmax_used;
    jb.out[3] = (double)substeps;
    jb.out[4] = total;
  }
}

}  // namespace

int packed_max_atoms(int prec) { return prec == kC128 ? 12 : 13; }

hipError_t packed_evolve(int prec, const PackedJob* d_jobs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (prec == kC128)
    hipLaunchKernelGGL(packed_evolve_kernel<double>, dim3(count), dim3(kThreads), 0, s, d_jobs);
  else
    hipLaunchKernelGGL(packed_evolve_kernel<float>, dim3(count), dim3(kThreads), 0, s, d_jobs);
  return hipGetLastError();
}

}  // namespace rsv
