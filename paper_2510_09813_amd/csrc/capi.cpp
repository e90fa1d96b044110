// C ABI of librsv: handles, validation, the time stepper and the Lanczos driver.
//
// Stepper (Sec. III): step k holds the pulse at its midpoint sample value and advances
// psi by exp(-i H_k dt) (eq. 6).  Lanczos driver (Sec. III.A), per iteration j:
//   w    = H v_j - beta_{j-1} v_{j-1}          (H psi passes, fused recurrence term)
//   alpha_j = Re<v_j, w>                        (FP64 partials, device-side finalise)
//   u    = w - alpha_j v_j,  beta_j = |u|       (one sweep; u stored unnormalised as the
//                                                next basis vector, v_{j+1} = u / beta_j is
//                                                applied as a scale on every later read)
//   host: eigendecomposition of T_{j+1}, y = exp(-i dt T_{j+1}) e_1 and the estimate
//         beta_j |y_j| |psi|; stop when it is at most tol.
// One device-to-host copy of (alpha_j, beta_j^2) per iteration.  After convergence,
// psi_{k+1} = |psi_k| sum_l y_l v_l (one combine sweep, which also returns |psi_{k+1}|^2).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdarg>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rsv.h"
#include "rsv_internal.h"

using namespace rsv;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (expr);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(RSV_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                  __FILE__, __LINE__);                                                   \
  } while (0)

#define RSV_TRY(expr)            \
  do {                           \
    int r_ = (expr);             \
    if (r_ != RSV_OK) return r_; \
  } while (0)

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// ------------------------------------------------------------------------------ handles
struct rsv_ctx {
  int device = 0;
  size_t budget = 0;
  size_t in_use = 0;
  double* h_pinned = nullptr;  // host-visible scalars of the per-iteration exchange
};

struct Workspace {
  int kmax = 0;
  void* block = nullptr;  // (kmax + 3) vectors
  std::vector<void*> basis;
  void* w = nullptr;
  void* t = nullptr;
  double* partial = nullptr;
  double* dscal = nullptr;  // [0] alpha, [1] beta^2, [2] |psi|^2
  size_t bytes = 0;
};

struct rsv_register {
  rsv_ctx* ctx = nullptr;
  int n = 0;
  int prec = 0;
  double c6 = 0;
  double* d_ub = nullptr;
  void* d_diag = nullptr;
  void* d_hbuf = nullptr;  // high-bit partial of rsv_apply_hamiltonian
  size_t bytes = 0;
  Workspace ws;
};

struct rsv_result {
  rsv_ctx* ctx = nullptr;
  int n = 0;
  int prec = 0;
  void* d_psi = nullptr;
  size_t bytes = 0;
  rsv_stats stats{};
};

namespace {

int dev_alloc(rsv_ctx* ctx, size_t bytes, void** p) {
  *p = nullptr;
  if (ctx->budget && ctx->in_use + bytes > ctx->budget)
    return fail(RSV_ENOMEM, "HBM budget exceeded: %zu in use + %zu requested > %zu budget",
                ctx->in_use, bytes, ctx->budget);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(RSV_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  ctx->in_use += bytes;
  return RSV_OK;
}

void dev_free(rsv_ctx* ctx, void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  ctx->in_use -= bytes;
}

size_t vec_bytes(int n, int prec) { return (size_t(1) << n) * amp_bytes(prec); }

size_t partial_doubles(int n, int prec) {
  int64_t a = hpsi_num_partials(prec, n), b = vec_num_partials(prec, n);
  int64_t c = occ_num_partials(n), d = sample_scratch_doubles(n);
  return (size_t)std::max(std::max(a, b), std::max(c, d));
}

size_t workspace_bytes(int n, int kmax, int prec) {
  return (size_t)(kmax + 3) * vec_bytes(n, prec) + partial_doubles(n, prec) * 8 + 256;
}

void ws_release(rsv_register* reg) {
  Workspace& ws = reg->ws;
  dev_free(reg->ctx, ws.block, ws.bytes);
  ws = Workspace{};
}

int ws_acquire(rsv_register* reg, int kmax) {
  Workspace& ws = reg->ws;
  if (ws.block && ws.kmax == kmax) return RSV_OK;
  ws_release(reg);
  const size_t vb = vec_bytes(reg->n, reg->prec);
  const size_t pb = partial_doubles(reg->n, reg->prec) * 8;
  const size_t bytes = (size_t)(kmax + 3) * vb + pb + 256;
  void* block = nullptr;
  RSV_TRY(dev_alloc(reg->ctx, bytes, &block));
  ws.block = block;
  ws.bytes = bytes;
  ws.kmax = kmax;
  char* p = (char*)block;
  ws.basis.resize(kmax + 1);
  for (int i = 0; i <= kmax; ++i) ws.basis[i] = p + (size_t)i * vb;
  ws.w = p + (size_t)(kmax + 1) * vb;
  ws.t = p + (size_t)(kmax + 2) * vb;
  ws.partial = (double*)(p + (size_t)(kmax + 3) * vb);
  ws.dscal = (double*)(p + (size_t)(kmax + 3) * vb + pb);
  return RSV_OK;
}

// ------------------------------------------------------------------------------ pulses
int check_pulses(const rsv_pulses* pl, int n) {
  if (!pl || !pl->omega || !pl->delta) return fail(RSV_EINVAL, "pulses: omega and delta required");
  if (pl->n_samples < 1) return fail(RSV_EINVAL, "pulses: n_samples must be >= 1");
  if (pl->per_site != 0 && pl->per_site != 1) return fail(RSV_EINVAL, "pulses: per_site is 0 or 1");
  const size_t cnt = (size_t)pl->n_samples * (pl->per_site ? (size_t)n : 1);
  if (!finite_all(pl->omega, cnt) || !finite_all(pl->delta, cnt) ||
      (pl->phi && !finite_all(pl->phi, cnt)))
    return fail(RSV_EINVAL, "pulses: non-finite sample");
  return RSV_OK;
}

// Midpoint value of step k (Sec. III): mean of the samples at floor(m) and ceil(m),
// m = (k + 1/2) dt in ns.
double midpoint(const double* x, int64_t k, int dt_ns) {
  const int64_t twice = (2 * k + 1) * (int64_t)dt_ns;  // 2m, an integer
  const int64_t lo = twice / 2, hi = (twice + 1) / 2;
  return 0.5 * (x[lo] + x[hi]);
}

StepCoef step_coef(const rsv_pulses* pl, int n, int64_t k, int dt_ns) {
  StepCoef c;
  std::memset(&c, 0, sizeof c);
  c.n = n;
  std::vector<double> om(n), de(n), ph(n);
  for (int i = 0; i < n; ++i) {
    const size_t off = pl->per_site ? (size_t)i * pl->n_samples : 0;
    om[i] = midpoint(pl->omega + off, k, dt_ns);
    de[i] = midpoint(pl->delta + off, k, dt_ns);
    ph[i] = pl->phi ? midpoint(pl->phi + off, k, dt_ns) : 0.0;
  }
  bool uniform = true;
  for (int i = 1; i < n; ++i)
    uniform = uniform && om[i] == om[0] && de[i] == de[0] && ph[i] == ph[0];
  c.site = uniform ? 0 : 1;
  for (int i = 0; i < n; ++i) {
    const int p = n - 1 - i;  // atom i is bit n-1-i
    const double h = 0.5 * om[i];
    c.up_re[p] = h * std::cos(ph[i]);
    c.up_im[p] = -h * std::sin(ph[i]);
    c.dn_re[p] = h * std::cos(ph[i]);
    c.dn_im[p] = h * std::sin(ph[i]);
    c.delta[p] = de[i];
  }
  return c;
}

int check_opts(const rsv_evolve_opts* o, const rsv_pulses* pl, int64_t* first, int64_t* count) {
  if (!o) return fail(RSV_EINVAL, "opts is NULL");
  if (o->dt_ns < 1) return fail(RSV_EINVAL, "dt_ns must be >= 1");
  if ((pl->n_samples - 1) % o->dt_ns != 0)
    return fail(RSV_EINVAL, "pulse duration %lld ns is not a multiple of dt = %d ns",
                (long long)(pl->n_samples - 1), o->dt_ns);
  if (!(o->tol > 0.0) || !std::isfinite(o->tol)) return fail(RSV_EINVAL, "tol must be > 0");
  if (o->kmax < 2 || o->kmax > kMaxKrylov) return fail(RSV_EINVAL, "kmax must be in 2..64");
  if (o->max_substep_depth < 0 || o->max_substep_depth > 40)
    return fail(RSV_EINVAL, "max_substep_depth must be in 0..40");
  const int64_t K = (pl->n_samples - 1) / o->dt_ns;
  if (o->first_step < 0 || o->first_step > K) return fail(RSV_EINVAL, "first_step out of range");
  const int64_t cnt = o->n_steps < 0 ? K - o->first_step : o->n_steps;
  if (o->first_step + cnt > K) return fail(RSV_EINVAL, "steps beyond the end of the pulse");
  *first = o->first_step;
  *count = cnt;
  return RSV_OK;
}

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

// ------------------------------------------------------------------------------ Lanczos
struct Lanczos {
  rsv_register* reg;
  hipStream_t s;
  rsv_stats* st;
  double norm2;  // |psi|^2 of the state in basis[0]
  std::vector<double> alpha, beta, scale, yre, yim, work;
};

int exchange(Lanczos& L, int nvals, double* out) {
  rsv_ctx* ctx = L.reg->ctx;
  HIP_TRY(hipMemcpyAsync(ctx->h_pinned, L.reg->ws.dscal, nvals * sizeof(double),
                         hipMemcpyDeviceToHost, L.s));
  HIP_TRY(hipStreamSynchronize(L.s));
  for (int i = 0; i < nvals; ++i) out[i] = ctx->h_pinned[i];
  return RSV_OK;
}

// psi <- exp(-i tau H) psi with psi in basis[0] (|psi|^2 = L.norm2).
int propagate(Lanczos& L, const StepCoef& c, double tau, double tol, int kmax, int max_depth) {
  rsv_register* reg = L.reg;
  Workspace& ws = reg->ws;
  const int n = reg->n, prec = reg->prec;
  const int64_t np_h = hpsi_num_partials(prec, n), np_v = vec_num_partials(prec, n);
  const double hbytes = (double)(size_t(1) << n) * (prec == kC128 ? 40.0 : 20.0);
  double remaining = tau;
  while (remaining > 0.0) {
    const double nrm = std::sqrt(L.norm2);
    if (!(nrm > 0.0) || !std::isfinite(nrm))
      return fail(RSV_ENUMERIC, "state norm is %g", nrm);
    L.scale[0] = 1.0 / nrm;
    int m = 0;
    double sub = remaining;
    for (int j = 0; j < kmax; ++j) {
      const void* prev = j > 0 ? ws.basis[j - 1] : nullptr;
      const double cprev = j > 0 ? L.beta[j - 1] * L.scale[j - 1] : 0.0;
      HIP_TRY(hpsi_apply(prec, n, c, reg->d_diag, ws.basis[j], L.scale[j], ws.w, prev, cprev,
                         ws.t, ws.partial, L.s));
      HIP_TRY(finalize_sum(ws.partial, np_h, ws.dscal + 0, L.s));
      HIP_TRY(lanczos_update(prec, n, ws.w, ws.basis[j], L.scale[j], ws.dscal + 0,
                             ws.basis[j + 1], ws.partial, L.s));
      HIP_TRY(finalize_sum(ws.partial, np_v, ws.dscal + 1, L.s));
      double ab[2];
      RSV_TRY(exchange(L, 2, ab));
      L.st->krylov_iters += 1;
      L.st->bytes_hpsi += hbytes;
      if (!std::isfinite(ab[0]) || !std::isfinite(ab[1]))
        return fail(RSV_ENUMERIC, "Lanczos coefficient not finite at iteration %d", j);
      L.alpha[j] = ab[0];
      const double bj = std::sqrt(std::max(ab[1], 0.0));
      m = j + 1;
      if (tridiag_expm(m, L.alpha.data(), L.beta.data(), remaining, L.yre.data(), L.yim.data(),
                       L.work.data()) != 0)
        return fail(RSV_ENUMERIC, "tridiagonal eigensolver failed (m = %d)", m);
      const double est = bj * std::hypot(L.yre[m - 1], L.yim[m - 1]) * nrm;
      if (est <= tol || bj == 0.0) break;
      if (j == kmax - 1) {
        // not converged: the largest dyadic sub-step the basis already resolves
        bool ok = false;
        for (int d = 1; d <= max_depth && !ok; ++d) {
          sub = std::ldexp(remaining, -d);
          if (tridiag_expm(m, L.alpha.data(), L.beta.data(), sub, L.yre.data(), L.yim.data(),
                           L.work.data()) != 0)
            return fail(RSV_ENUMERIC, "tridiagonal eigensolver failed (m = %d)", m);
          ok = bj * std::hypot(L.yre[m - 1], L.yim[m - 1]) * nrm <= tol;
        }
        if (!ok)
          return fail(RSV_ENOTCONV, "Krylov exponential not converged with kmax = %d", kmax);
        L.st->substeps += 1;
        break;
      }
      L.beta[j] = bj;
      L.scale[j + 1] = 1.0 / bj;
    }
    L.st->krylov_max = std::max<int64_t>(L.st->krylov_max, m);
    CombineCoef cc;
    std::memset(&cc, 0, sizeof cc);
    cc.m = m;
    for (int l = 0; l < m; ++l) {
      cc.re[l] = nrm * L.yre[l] * L.scale[l];
      cc.im[l] = nrm * L.yim[l] * L.scale[l];
      cc.x[l] = ws.basis[l];
    }
    HIP_TRY(krylov_combine(prec, n, cc, ws.w, ws.partial, L.s));
    HIP_TRY(finalize_sum(ws.partial, np_v, ws.dscal + 2, L.s));
    std::swap(ws.basis[0], ws.w);
    double nn[3];
    RSV_TRY(exchange(L, 3, nn));
    L.norm2 = nn[2];
    remaining = (sub == remaining) ? 0.0 : remaining - sub;
  }
  return RSV_OK;
}

int evolve_impl(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o, void* d_psi,
                hipStream_t s, rsv_stats* st) {
  if (!reg) return fail(RSV_EINVAL, "register is NULL");
  if (!d_psi) return fail(RSV_EINVAL, "state pointer is NULL");
  RSV_TRY(check_pulses(pl, reg->n));
  int64_t first = 0, count = 0;
  RSV_TRY(check_opts(o, pl, &first, &count));
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipSetDevice(reg->ctx->device));
  RSV_TRY(ws_acquire(reg, o->kmax));
  Workspace& ws = reg->ws;
  const int n = reg->n, prec = reg->prec;
  const size_t vb = vec_bytes(n, prec);
  HIP_TRY(hipMemcpyAsync(ws.basis[0], d_psi, vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(norm2_partial(prec, n, ws.basis[0], ws.partial, s));
  HIP_TRY(finalize_sum(ws.partial, vec_num_partials(prec, n), ws.dscal + 2, s));
  Lanczos L{reg, s, st, 0.0, {}, {}, {}, {}, {}, {}};
  L.alpha.assign(kMaxKrylov + 1, 0.0);
  L.beta.assign(kMaxKrylov + 1, 0.0);
  L.scale.assign(kMaxKrylov + 1, 0.0);
  L.yre.assign(kMaxKrylov, 0.0);
  L.yim.assign(kMaxKrylov, 0.0);
  L.work.assign(tridiag_work_doubles(kMaxKrylov), 0.0);
  double nn[3];
  RSV_TRY(exchange(L, 3, nn));
  L.norm2 = nn[2];
  const double tau = o->dt_ns * 1e-3;  // us
  for (int64_t k = first; k < first + count; ++k) {
    const StepCoef c = step_coef(pl, n, k, o->dt_ns);
    RSV_TRY(propagate(L, c, tau, o->tol, o->kmax, o->max_substep_depth));
    st->steps += 1;
  }
  HIP_TRY(hipMemcpyAsync(d_psi, ws.basis[0], vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  st->norm_final = std::sqrt(L.norm2);
  st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return RSV_OK;
}

int check_state_args(int n, int prec) {
  if (n < 1 || n > kMaxAtoms) return fail(RSV_EINVAL, "n_atoms must be in 1..%d", kMaxAtoms);
  if (prec != kC128 && prec != kC64) return fail(RSV_EINVAL, "unknown precision %d", prec);
  return RSV_OK;
}

int occupations_impl(rsv_ctx* ctx, int n, int prec, const void* d_psi, double* out,
                     hipStream_t s) {
  RSV_TRY(check_state_args(n, prec));
  if (!ctx || !d_psi || !out) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t np = (size_t)occ_num_partials(n) + 64;
  void* buf = nullptr;
  RSV_TRY(dev_alloc(ctx, np * 8, &buf));
  double* part = (double*)buf;
  double* res = part + occ_num_partials(n);
  hipError_t e = occupations(prec, n, d_psi, part, res, s);
  double h[kMaxAtoms + 1];
  if (e == hipSuccess) e = hipMemcpyAsync(h, res, (n + 1) * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(ctx, buf, np * 8);
  if (e != hipSuccess) return fail(RSV_EDEVICE, "occupations: %s", hipGetErrorString(e));
  if (!(h[0] > 0.0)) return fail(RSV_ENUMERIC, "state has zero norm");
  for (int i = 0; i < n; ++i) out[i] = h[1 + (n - 1 - i)] / h[0];
  return RSV_OK;
}

int sample_impl(rsv_ctx* ctx, int n, int prec, const void* d_psi, uint64_t seed, int shots,
                uint64_t* out, hipStream_t s) {
  RSV_TRY(check_state_args(n, prec));
  if (!ctx || !d_psi || (shots > 0 && !out)) return fail(RSV_EINVAL, "NULL argument");
  if (shots < 0) return fail(RSV_EINVAL, "n_shots must be >= 0");
  if (shots == 0) return RSV_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  const size_t nd = (size_t)sample_scratch_doubles(n);
  const size_t bytes = nd * 8 + (size_t)shots * 8;
  void* buf = nullptr;
  RSV_TRY(dev_alloc(ctx, bytes, &buf));
  double* scratch = (double*)buf;
  uint64_t* d_idx = (uint64_t*)(scratch + nd);
  hipError_t e = sample(prec, n, d_psi, seed, shots, scratch, d_idx, s);
  if (e == hipSuccess) e = hipMemcpyAsync(out, d_idx, (size_t)shots * 8, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dev_free(ctx, buf, bytes);
  if (e != hipSuccess) return fail(RSV_EDEVICE, "sample: %s", hipGetErrorString(e));
  return RSV_OK;
}

}  // namespace

// ============================================================================== C ABI
extern "C" {

const char* rsv_version(void) { return "librsv 0.1 (gfx950)"; }

const char* rsv_last_error(void) { return g_err.c_str(); }

int rsv_ctx_create(int hip_device, size_t budget, rsv_ctx** out) {
  if (!out) return fail(RSV_EINVAL, "out is NULL");
  *out = nullptr;
  int count = 0;
  HIP_TRY(hipGetDeviceCount(&count));
  if (hip_device < 0 || hip_device >= count)
    return fail(RSV_EINVAL, "device %d not present (%d devices)", hip_device, count);
  HIP_TRY(hipSetDevice(hip_device));
  rsv_ctx* c = new (std::nothrow) rsv_ctx();
  if (!c) return fail(RSV_ENOMEM, "host allocation failed");
  c->device = hip_device;
  c->budget = budget;
  hipError_t e = hipHostMalloc((void**)&c->h_pinned, 64 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return fail(RSV_EDEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
  }
  *out = c;
  return RSV_OK;
}

void rsv_ctx_destroy(rsv_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  delete ctx;
}

size_t rsv_ctx_bytes_in_use(const rsv_ctx* ctx) { return ctx ? ctx->in_use : 0; }

size_t rsv_workspace_bytes(int n, int kmax, rsv_precision prec) {
  if (n < 1 || n > kMaxAtoms || kmax < 2 || kmax > kMaxKrylov) return 0;
  const size_t diag = (size_t(1) << n) * real_bytes(prec);
  return workspace_bytes(n, kmax, prec) + diag + vec_bytes(n, prec) + 32 * 32 * 8;
}

int rsv_register_create(rsv_ctx* ctx, int n, const double* xyz, double c6, rsv_precision prec,
                        rsv_register** out) {
  if (!out) return fail(RSV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx || !xyz) return fail(RSV_EINVAL, "NULL argument");
  RSV_TRY(check_state_args(n, prec));
  if (!std::isfinite(c6)) return fail(RSV_EINVAL, "C6 not finite");
  if (!finite_all(xyz, (size_t)3 * n)) return fail(RSV_EINVAL, "positions not finite");
  // U_ij = C / |r_i - r_j|^6 (eq. 3), stored by bit position p = n-1-i
  std::vector<double> ub(32 * 32, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < i; ++j) {
      const double dx = xyz[3 * i] - xyz[3 * j], dy = xyz[3 * i + 1] - xyz[3 * j + 1],
                   dz = xyz[3 * i + 2] - xyz[3 * j + 2];
      const double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 == 0.0) return fail(RSV_EINVAL, "atoms %d and %d coincide", j, i);
      const double u = c6 / (r2 * r2 * r2);
      const int p = n - 1 - i, q = n - 1 - j;
      ub[p * 32 + q] = ub[q * 32 + p] = u;
    }
  }
  HIP_TRY(hipSetDevice(ctx->device));
  rsv_register* r = new (std::nothrow) rsv_register();
  if (!r) return fail(RSV_ENOMEM, "host allocation failed");
  r->ctx = ctx;
  r->n = n;
  r->prec = prec;
  r->c6 = c6;
  const size_t dbytes = (size_t(1) << n) * real_bytes(prec);
  void* p = nullptr;
  int rc = dev_alloc(ctx, 32 * 32 * 8 + dbytes, &p);
  if (rc != RSV_OK) {
    delete r;
    return rc;
  }
  r->bytes = 32 * 32 * 8 + dbytes;
  r->d_ub = (double*)p;
  r->d_diag = (char*)p + 32 * 32 * 8;
  hipError_t e = hipMemcpy(r->d_ub, ub.data(), 32 * 32 * 8, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = diag_build(prec, n, r->d_ub, r->d_diag, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    rsv_register_destroy(r);
    return fail(RSV_EDEVICE, "interaction diagonal: %s", hipGetErrorString(e));
  }
  *out = r;
  return RSV_OK;
}

void rsv_register_destroy(rsv_register* reg) {
  if (!reg) return;
  (void)hipSetDevice(reg->ctx->device);
  (void)hipDeviceSynchronize();
  ws_release(reg);
  dev_free(reg->ctx, reg->d_hbuf, reg->d_hbuf ? vec_bytes(reg->n, reg->prec) : 0);
  dev_free(reg->ctx, reg->d_ub, reg->bytes);
  delete reg;
}

int rsv_register_diagonal(rsv_register* reg, void* d_out, void* stream) {
  if (!reg || !d_out) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(reg->ctx->device));
  hipStream_t s = as_stream(stream);
  HIP_TRY(hipMemcpyAsync(d_out, reg->d_diag, (size_t(1) << reg->n) * real_bytes(reg->prec),
                         hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RSV_OK;
}

int rsv_apply_hamiltonian(rsv_register* reg, const rsv_pulses* pl, int64_t step, int dt_ns,
                          const void* d_in, void* d_out, void* stream) {
  if (!reg || !d_in || !d_out) return fail(RSV_EINVAL, "NULL argument");
  if (d_in == d_out) return fail(RSV_EINVAL, "input and output must differ");
  RSV_TRY(check_pulses(pl, reg->n));
  if (dt_ns < 1) return fail(RSV_EINVAL, "dt_ns must be >= 1");
  const int64_t K = (pl->n_samples - 1) / dt_ns;
  if (step < 0 || step >= K || (2 * step + 1) * (int64_t)dt_ns > 2 * (pl->n_samples - 1))
    return fail(RSV_EINVAL, "step %lld outside the pulse (%lld steps)", (long long)step,
                (long long)K);
  HIP_TRY(hipSetDevice(reg->ctx->device));
  const TilePlan plan = make_tile_plan(reg->prec, reg->n);
  if (plan.n_hi_passes > 0 && !reg->d_hbuf)
    RSV_TRY(dev_alloc(reg->ctx, vec_bytes(reg->n, reg->prec), &reg->d_hbuf));
  const StepCoef c = step_coef(pl, reg->n, step, dt_ns);
  hipStream_t s = as_stream(stream);
  HIP_TRY(hpsi_apply(reg->prec, reg->n, c, reg->d_diag, d_in, 1.0, d_out, nullptr, 0.0,
                     reg->d_hbuf, nullptr, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RSV_OK;
}

int rsv_evolve_device(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o,
                      void* d_psi, void* stream, rsv_stats* stats_out) {
  rsv_stats st{};
  const int rc = evolve_impl(reg, pl, o, d_psi, as_stream(stream), &st);
  if (stats_out) *stats_out = st;
  return rc;
}

int rsv_evolve(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o,
               const void* psi0_host, rsv_result** out) {
  if (!out) return fail(RSV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!reg) return fail(RSV_EINVAL, "register is NULL");
  HIP_TRY(hipSetDevice(reg->ctx->device));
  const int n = reg->n, prec = reg->prec;
  rsv_result* r = new (std::nothrow) rsv_result();
  if (!r) return fail(RSV_ENOMEM, "host allocation failed");
  r->ctx = reg->ctx;
  r->n = n;
  r->prec = prec;
  r->bytes = vec_bytes(n, prec);
  int rc = dev_alloc(reg->ctx, r->bytes, &r->d_psi);
  if (rc != RSV_OK) {
    delete r;
    return rc;
  }
  hipError_t e = hipSuccess;
  if (psi0_host) {
    void* tmp = nullptr;
    const size_t b128 = (size_t(1) << n) * 16;
    if (prec == kC128) {
      e = hipMemcpy(r->d_psi, psi0_host, b128, hipMemcpyHostToDevice);
    } else {
      rc = dev_alloc(reg->ctx, b128, &tmp);
      if (rc == RSV_OK) {
        e = hipMemcpy(tmp, psi0_host, b128, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = convert_from_c128(prec, n, tmp, r->d_psi, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        dev_free(reg->ctx, tmp, b128);
      }
    }
  } else {
    e = hipMemset(r->d_psi, 0, r->bytes);
    if (e == hipSuccess) {
      if (prec == kC128) {
        const double one[2] = {1.0, 0.0};
        e = hipMemcpy(r->d_psi, one, sizeof one, hipMemcpyHostToDevice);
      } else {
        const float one[2] = {1.0f, 0.0f};
        e = hipMemcpy(r->d_psi, one, sizeof one, hipMemcpyHostToDevice);
      }
    }
  }
  if (rc == RSV_OK && e != hipSuccess) rc = fail(RSV_EDEVICE, "state upload: %s", hipGetErrorString(e));
  if (rc == RSV_OK) rc = evolve_impl(reg, pl, o, r->d_psi, nullptr, &r->stats);
  if (rc != RSV_OK) {
    rsv_result_destroy(r);
    return rc;
  }
  *out = r;
  return RSV_OK;
}

int rsv_result_state(const rsv_result* r, void* host) {
  if (!r || !host) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(r->ctx->device));
  const size_t b128 = (size_t(1) << r->n) * 16;
  if (r->prec == kC128) {
    HIP_TRY(hipMemcpy(host, r->d_psi, b128, hipMemcpyDeviceToHost));
    return RSV_OK;
  }
  void* tmp = nullptr;
  RSV_TRY(dev_alloc(r->ctx, b128, &tmp));
  hipError_t e = convert_to_c128(r->prec, r->n, r->d_psi, tmp, nullptr);
  if (e == hipSuccess) e = hipMemcpy(host, tmp, b128, hipMemcpyDeviceToHost);
  dev_free(r->ctx, tmp, b128);
  if (e != hipSuccess) return fail(RSV_EDEVICE, "state download: %s", hipGetErrorString(e));
  return RSV_OK;
}

int rsv_result_occupations(const rsv_result* r, double* out) {
  if (!r) return fail(RSV_EINVAL, "result is NULL");
  return occupations_impl(r->ctx, r->n, r->prec, r->d_psi, out, nullptr);
}

int rsv_result_sample(const rsv_result* r, uint64_t seed, int shots, uint64_t* out) {
  if (!r) return fail(RSV_EINVAL, "result is NULL");
  return sample_impl(r->ctx, r->n, r->prec, r->d_psi, seed, shots, out, nullptr);
}

int rsv_result_stats(const rsv_result* r, rsv_stats* out) {
  if (!r || !out) return fail(RSV_EINVAL, "NULL argument");
  *out = r->stats;
  return RSV_OK;
}

void rsv_result_destroy(rsv_result* r) {
  if (!r) return;
  (void)hipSetDevice(r->ctx->device);
  dev_free(r->ctx, r->d_psi, r->bytes);
  delete r;
}

int rsv_occupations_device(rsv_ctx* ctx, int n, rsv_precision prec, const void* d_psi,
                           double* out, void* stream) {
  return occupations_impl(ctx, n, prec, d_psi, out, as_stream(stream));
}

int rsv_sample_device(rsv_ctx* ctx, int n, rsv_precision prec, const void* d_psi, uint64_t seed,
                      int shots, uint64_t* out, void* stream) {
  return sample_impl(ctx, n, prec, d_psi, seed, shots, out, as_stream(stream));
}

int rsv_tridiag_expm(int m, const double* alpha, const double* beta, double tau, double* y_re,
                     double* y_im) {
  if (m < 1 || m > kMaxKrylov) return fail(RSV_EINVAL, "m must be in 1..%d", kMaxKrylov);
  if (!alpha || !y_re || !y_im || (m > 1 && !beta)) return fail(RSV_EINVAL, "NULL argument");
  if (!finite_all(alpha, m) || (m > 1 && !finite_all(beta, m - 1)) || !std::isfinite(tau))
    return fail(RSV_EINVAL, "non-finite input");
  std::vector<double> work(tridiag_work_doubles(m));
  if (tridiag_expm(m, alpha, beta, tau, y_re, y_im, work.data()) != 0)
    return fail(RSV_ENUMERIC, "tridiagonal eigensolver did not converge");
  return RSV_OK;
}

}  // extern "C"
