// Host engine of librsv: memory, registers, the time stepper and the Lanczos driver.
//
// Stepper (Sec. III): step k holds the pulse at its midpoint sample value and advances psi
// by exp(-i H_k dt) (eq. 6).  Lanczos driver (Sec. III.A): each iteration is one H sweep
// whose first pass also forms the next Krylov vector from the three-term recurrence (alpha
// read from device memory) and whose last pass returns <u, H u>.  After the forming pass
// one device-to-host copy brings (alpha_{k-1}, beta_{k-1}^2) to the host, which
// diagonalises the tridiagonal T_k in FP64 and stops when the a-posteriori estimate
// beta_{k-1} |[exp(-i dt T_k) e_1]_k| |psi| is at most tol.  Then
// psi_{k+1} = |psi_k| sum_l y_l v_l (one combine sweep, which also returns |psi_{k+1}|^2).
#include "engine.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

namespace rsv {

namespace {
thread_local std::string g_err;

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

constexpr size_t kScalarBytes = 4096;
constexpr size_t kGranule = 256;
inline size_t round_up(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }
}  // namespace

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

const char* last_error() { return g_err.c_str(); }

// ------------------------------------------------------------------------------ memory
int DeviceAllocator::alloc(size_t bytes, void** p) {
  *p = nullptr;
  {
    std::lock_guard<std::mutex> lk(mu_);
    if (budget_ && in_use_ + bytes > budget_)
      return fail(RSV_ENOMEM, "HBM budget exceeded: %zu in use + %zu requested > %zu budget",
                  in_use_, bytes, budget_);
    in_use_ += bytes;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    std::lock_guard<std::mutex> lk(mu_);
    in_use_ -= bytes;
    return fail(RSV_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  return RSV_OK;
}

void DeviceAllocator::release(void* p, size_t bytes) {
  if (!p) return;
  (void)hipFree(p);
  std::lock_guard<std::mutex> lk(mu_);
  in_use_ -= bytes;
}

size_t DeviceAllocator::in_use() const {
  std::lock_guard<std::mutex> lk(mu_);
  return in_use_;
}

ArenaAllocator::~ArenaAllocator() {
  if (base_) (void)hipFree(base_);
}

int ArenaAllocator::init(size_t bytes) {
  bytes = round_up(bytes);
  hipError_t e = hipMalloc((void**)&base_, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    base_ = nullptr;
    return fail(RSV_ENOMEM, "arena hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  std::lock_guard<std::mutex> lk(mu_);
  ff_.reset(bytes);
  return RSV_OK;
}

int ArenaAllocator::alloc(size_t bytes, void** p) {
  *p = nullptr;
  bytes = round_up(bytes ? bytes : 1);
  std::lock_guard<std::mutex> lk(mu_);
  size_t off = 0;
  if (!ff_.take(bytes, &off))
    return fail(RSV_ENOMEM, "arena has no free block of %zu bytes (%zu of %zu in use)", bytes,
                ff_.used(), ff_.size());
  *p = base_ + off;
  return RSV_OK;
}

void ArenaAllocator::release(void* p, size_t bytes) {
  if (!p) return;
  bytes = round_up(bytes ? bytes : 1);
  std::lock_guard<std::mutex> lk(mu_);
  ff_.give((size_t)((char*)p - base_), bytes);
}

size_t ArenaAllocator::in_use() const {
  std::lock_guard<std::mutex> lk(mu_);
  return ff_.used();
}

size_t vec_bytes(int n, int prec) { return (size_t(1) << n) * amp_bytes(prec); }

size_t partial_doubles(int n, int prec) {
  int64_t a = sweep_num_partials(prec, n), b = vec_num_partials(prec, n);
  int64_t c = occ_num_partials(n), d = sample_scratch_doubles(n);
  // the two partial arrays are adjacent: together they hold a group of re-orthogonalisation
  // inner products (2 kDotGroup rows of vec_num_partials)
  const int64_t e = (int64_t)kDotGroup * b;
  return (size_t)std::max(std::max(std::max(a, b), std::max(c, d)), e);
}

size_t workspace_bytes(int n, int kmax, int prec) {
  return (size_t)(kmax + 3) * vec_bytes(n, prec) + 2 * round_up(partial_doubles(n, prec) * 8) +
         kScalarBytes;
}

size_t register_bytes(int n, int prec) {
  return 32 * 32 * 8 + round_up(diag_table_doubles(prec, n) * 8);
}

int check_state_args(int n, int prec) {
  if (n < 1 || n > kMaxAtoms) return fail(RSV_EINVAL, "n_atoms must be in 1..%d", kMaxAtoms);
  if (prec != kC128 && prec != kC64) return fail(RSV_EINVAL, "unknown precision %d", prec);
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
static double midpoint(const double* x, int64_t k, int dt_ns) {
  const int64_t twice = (2 * k + 1) * (int64_t)dt_ns;  // 2m, an integer
  const int64_t lo = twice / 2, hi = (twice + 1) / 2;
  return 0.5 * (x[lo] + x[hi]);
}

StepCoef step_coef(const rsv_pulses* pl, int n, int64_t k, int dt_ns) {
  StepCoef c;
  std::memset(&c, 0, sizeof c);
  c.n = n;
  double om[kMaxAtoms], de[kMaxAtoms], ph[kMaxAtoms];
  for (int i = 0; i < n; ++i) {
    const size_t off = pl->per_site ? (size_t)i * pl->n_samples : 0;
    om[i] = midpoint(pl->omega + off, k, dt_ns);
    de[i] = midpoint(pl->delta + off, k, dt_ns);
    ph[i] = pl->phi ? midpoint(pl->phi + off, k, dt_ns) : 0.0;
  }
  bool uniform = true;
  for (int i = 1; i < n; ++i)
    uniform = uniform && om[i] == om[0] && de[i] == de[0] && ph[i] == ph[0];
  c.mode = !uniform ? kCoefSite : (ph[0] == 0.0 ? kCoefReal : kCoefUniform);
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
  if (o->reorth != 0 && o->reorth != 1) return fail(RSV_EINVAL, "reorth must be 0 or 1");
  const int64_t K = (pl->n_samples - 1) / o->dt_ns;
  if (o->first_step < 0 || o->first_step > K) return fail(RSV_EINVAL, "first_step out of range");
  const int64_t cnt = o->n_steps < 0 ? K - o->first_step : o->n_steps;
  if (o->first_step + cnt > K) return fail(RSV_EINVAL, "steps beyond the end of the pulse");
  *first = o->first_step;
  *count = cnt;
  return RSV_OK;
}

// ------------------------------------------------------------------------------ register
int build_interactions(int n, const double* xyz, double c6, double* ub) {
  if (!std::isfinite(c6)) return fail(RSV_EINVAL, "C6 not finite");
  if (!finite_all(xyz, (size_t)3 * n)) return fail(RSV_EINVAL, "positions not finite");
  std::memset(ub, 0, 32 * 32 * sizeof(double));
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
  return RSV_OK;
}

int register_create(rsv_ctx* ctx, Allocator* alloc, int n, const double* xyz, double c6,
                    int prec, hipStream_t stream, double* h_scal, rsv_register** out) {
  *out = nullptr;
  if (!ctx || !xyz) return fail(RSV_EINVAL, "NULL argument");
  RSV_TRY(check_state_args(n, prec));
  double ub[32 * 32];
  RSV_TRY(build_interactions(n, xyz, c6, ub));
  HIP_TRY(hipSetDevice(ctx->device));
  rsv_register* r = new (std::nothrow) rsv_register();
  if (!r) return fail(RSV_ENOMEM, "host allocation failed");
  r->ctx = ctx;
  r->alloc = alloc;
  r->n = n;
  r->prec = prec;
  r->c6 = c6;
  if (h_scal) {
    r->h_scal = h_scal;
  } else {
    hipError_t e = hipHostMalloc((void**)&r->h_scal, 512 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
      delete r;
      return fail(RSV_EDEVICE, "hipHostMalloc failed: %s", hipGetErrorString(e));
    }
    r->own_h_scal = true;
  }
  void* p = nullptr;
  const int rc = alloc->alloc(register_bytes(n, prec), &p);
  if (rc != RSV_OK) {
    register_destroy(r, stream);
    return rc;
  }
  r->bytes = register_bytes(n, prec);
  r->d_ub = (double*)p;
  r->d_dtab = (double*)((char*)p + 32 * 32 * 8);
  // the host array must outlive the asynchronous copy: synchronise before returning
  hipError_t e = hipMemcpyAsync(r->d_ub, ub, sizeof ub, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = diag_tables_build(prec, n, r->d_ub, r->d_dtab, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    register_destroy(r, stream);
    return fail(RSV_EDEVICE, "interaction diagonal: %s", hipGetErrorString(e));
  }
  *out = r;
  return RSV_OK;
}

static void workspace_release(rsv_register* reg) {
  Workspace& ws = reg->ws;
  if (ws.block) reg->alloc->release(ws.block, ws.bytes);
  ws = Workspace{};
}

void register_destroy(rsv_register* reg, hipStream_t stream) {
  if (!reg) return;
  (void)hipSetDevice(reg->ctx->device);
  (void)hipStreamSynchronize(stream);
  workspace_release(reg);
  if (reg->d_hbuf) reg->alloc->release(reg->d_hbuf, vec_bytes(reg->n, reg->prec));
  if (reg->d_efull) reg->alloc->release(reg->d_efull, (size_t(1) << reg->n) * sizeof(double));
  if (reg->d_ub) reg->alloc->release(reg->d_ub, reg->bytes);
  if (reg->own_h_scal && reg->h_scal) (void)hipHostFree(reg->h_scal);
  if (reg->have_ev)
    for (hipEvent_t e : reg->ev) (void)hipEventDestroy(e);
  delete reg;
}

int workspace_acquire(rsv_register* reg, int kmax) {
  Workspace& ws = reg->ws;
  if (ws.block && ws.kmax == kmax) return RSV_OK;
  workspace_release(reg);
  const size_t vb = vec_bytes(reg->n, reg->prec);
  const size_t pb = round_up(partial_doubles(reg->n, reg->prec) * 8);
  const size_t bytes = workspace_bytes(reg->n, kmax, reg->prec);
  void* block = nullptr;
  RSV_TRY(reg->alloc->alloc(bytes, &block));
  ws.block = block;
  ws.bytes = bytes;
  ws.kmax = kmax;
  char* p = (char*)block;
  ws.basis.resize(kmax + 1);
  for (int i = 0; i <= kmax; ++i) ws.basis[i] = p + (size_t)i * vb;
  ws.z = p + (size_t)(kmax + 1) * vb;
  ws.t = p + (size_t)(kmax + 2) * vb;
  ws.pnorm = (double*)(p + (size_t)(kmax + 3) * vb);
  ws.pdot = (double*)(p + (size_t)(kmax + 3) * vb + pb);
  ws.dscal = (double*)(p + (size_t)(kmax + 3) * vb + 2 * pb);
  return RSV_OK;
}

// ------------------------------------------------------------------------------ Lanczos
namespace {

// Device scalars: slot 2k holds |u_k|^2, slot 2k+1 holds Re<u_k, H u_k>; kNormSlot |psi|^2;
// from kDotSlot, Re and Im <u_l, u_k> of the re-orthogonalisation (2 kMaxKrylov values).
constexpr int kNormSlot = 2 * kMaxKrylov + 4;
constexpr int kDotSlot = 256;
static_assert(kDotSlot + 2 * kMaxKrylov <= (int)(kScalarBytes / 8), "device scalar block");

struct Lanczos {
  rsv_register* reg;
  hipStream_t s;
  rsv_stats* st;
  double norm2;  // |psi|^2 of the state in basis[0]
  double alpha[kMaxKrylov + 1], beta[kMaxKrylov + 1], scale[kMaxKrylov + 1];
  double yre[kMaxKrylov], yim[kMaxKrylov];
  std::vector<double> work;
  double* occ_partial = nullptr;  // fused occupation sums of an observed step's combination
  double dir = 1.0;               // -1: exp(+i tau H), the step backwards in time
};

// Device scalar slots [first_slot, first_slot + count) through the same slots of h_scal.
int fetch_scalars(Lanczos& L, int first_slot, int count, double* out) {
  double* h = L.reg->h_scal + first_slot;
  HIP_TRY(hipMemcpyAsync(h, L.reg->ws.dscal + first_slot, count * sizeof(double),
                         hipMemcpyDeviceToHost, L.s));
  HIP_TRY(hipStreamSynchronize(L.s));
  for (int i = 0; i < count; ++i) out[i] = h[i];
  return RSV_OK;
}

// Events marking the per-iteration scalar copies, created once per register.
int ensure_events(rsv_register* reg) {
  if (reg->have_ev) return RSV_OK;
  for (int k = 0; k <= kMaxKrylov; ++k)
    HIP_TRY(hipEventCreateWithFlags(&reg->ev[k], hipEventDisableTiming));
  reg->have_ev = true;
  return RSV_OK;
}

// Full re-orthogonalisation of the new vector u_k (classical Gram-Schmidt with FP64 inner
// products): u_k <- u_k - sum_{l<k} v_l <v_l, u_k>, v_l = s_l u_l.  The result goes to a
// fresh buffer that becomes basis[k] (the old one becomes the high-pass partial t, which
// the caller recomputes).  b2 is |u_k|^2 before on entry and after on return.
int reorthogonalise(Lanczos& L, int k, double* b2) {
  rsv_register* reg = L.reg;
  Workspace& ws = reg->ws;
  const int n = reg->n, prec = reg->prec;
  const int64_t nw = vec_num_partials(prec, n);
  for (int l0 = 0; l0 < k; l0 += kDotGroup) {
    DotGroup d{};
    d.g = std::min(kDotGroup, k - l0);
    for (int g = 0; g < d.g; ++g) d.x[g] = ws.basis[l0 + g];
    HIP_TRY(multi_dot(prec, n, d, ws.basis[k], ws.pnorm, L.s));
    HIP_TRY(finalize_rows(ws.pnorm, nw, 2 * d.g, ws.dscal + kDotSlot + 2 * l0, L.s));
  }
  double dots[2 * kMaxKrylov];
  RSV_TRY(fetch_scalars(L, kDotSlot, 2 * k, dots));
  CombineCoef cc;
  std::memset(&cc, 0, sizeof cc);
  cc.m = k + 1;
  cc.re[0] = 1.0;
  cc.x[0] = ws.basis[k];
  double loss = 0.0;
  for (int l = 0; l < k; ++l) {
    const double sl = L.scale[l];
    if (!std::isfinite(dots[2 * l]) || !std::isfinite(dots[2 * l + 1]))
      return fail(RSV_ENUMERIC, "re-orthogonalisation inner product not finite");
    cc.re[l + 1] = -sl * sl * dots[2 * l];
    cc.im[l + 1] = -sl * sl * dots[2 * l + 1];
    cc.x[l + 1] = ws.basis[l];
    loss = std::max(loss, sl * std::hypot(dots[2 * l], dots[2 * l + 1]));
  }
  if (*b2 > 0.0) L.st->ortho_loss = std::max(L.st->ortho_loss, loss / std::sqrt(*b2));
  HIP_TRY(krylov_combine(prec, n, cc, ws.t, ws.pnorm, L.s));
  HIP_TRY(finalize_sum(ws.pnorm, nw, ws.dscal + 2 * k, L.s));
  std::swap(ws.basis[k], ws.t);
  RSV_TRY(fetch_scalars(L, 2 * k, 1, b2));
  return RSV_OK;
}

// |[exp(-i h T_m) e_1]_{m-1}| for the current T_m.
int last_component(Lanczos& L, int m, double h, double* out) {
  if (tridiag_expm_last(m, L.alpha, L.beta, h, out, L.work.data()) != 0)
    return fail(RSV_ENUMERIC, "tridiagonal eigensolver failed (m = %d)", m);
  return RSV_OK;
}

// psi <- exp(-i tau H) psi with psi in basis[0] (|psi|^2 = L.norm2).
//
// Krylov vectors are kept unnormalised: v_k = s_k u_k with s_0 = 1/|psi| and
// s_k = 1/beta_{k-1}.  Sweep k >= 1 forms
//   u_k = s_{k-1} z_{k-1} - s_{k-1}^3 <u_{k-1}, z_{k-1}> u_{k-1} - (s_{k-2}/s_{k-1}) u_{k-2}
// (= H v_{k-1} - alpha_{k-1} v_{k-1} - beta_{k-2} v_{k-2}) in its first pass, stores it,
// and returns |u_k|^2 = beta_{k-1}^2; the host then tests convergence of the m = k
// dimensional Krylov approximation before the later passes compute z_k = H u_k.
// With obs set, the combination that completes the step also writes the occupation sums of
// the new state to obs (device, n + 1 doubles).
int propagate(Lanczos& L, const StepCoef& c, double tau, double tol, int kmax, int max_depth,
              bool reorth, double* obs = nullptr) {
  rsv_register* reg = L.reg;
  Workspace& ws = reg->ws;
  const int n = reg->n, prec = reg->prec;
  const int64_t np_norm = sweep_norm_partials(prec, n), np_dot = sweep_dot_partials(prec, n);
  const bool single = sweep_passes(prec, n) == 1;
  const double hbytes = (double)(size_t(1) << n) * (prec == kC128 ? 40.0 : 20.0);
  // below 256 MiB per vector an iteration's kernels are short and the host round trip would
  // leave the device idle: queue one iteration ahead (re-orthogonalisation needs the host)
  const bool ahead = !reorth && vec_bytes(n, prec) < (size_t(256) << 20);
  RSV_TRY(ensure_events(reg));
  double remaining = tau;
  while (remaining > 0.0) {
    const double nrm = std::sqrt(L.norm2);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) return fail(RSV_ENUMERIC, "state norm is %g", nrm);
    L.scale[0] = 1.0 / nrm;
    // sweep 0: z_0 = H u_0 and <u_0, z_0>
    {
      const SweepIn in{ws.basis[0], nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
      const SweepOut so{nullptr, nullptr, ws.pdot};
      HIP_TRY(hpsi_sweep(prec, n, c, reg->d_dtab, in, ws.z, ws.t, so, kAllPasses, L.s));
      HIP_TRY(finalize_sum(ws.pdot, np_dot, ws.dscal + 1, L.s));
      L.st->krylov_iters += 1;
      L.st->bytes_hpsi += hbytes;
    }
    int m = 0;
    double sub = remaining;
    // device address of |u_k|^2 (|psi|^2 for k = 0): the forming pass takes s_k from it
    auto dev_norm = [&](int k) { return ws.dscal + (k == 0 ? kNormSlot : 2 * k); };
    // u_k from z_{k-1}, u_{k-1}, u_{k-2} with device-side coefficients, |u_k|^2, and the
    // copy of (<u_{k-1}, z_{k-1}>, |u_k|^2) to the pinned host scalars, marked by ev[k]
    auto form = [&](int k) -> int {
      SweepIn in{ws.z, ws.basis[k - 1], k >= 2 ? ws.basis[k - 2] : nullptr, 0.0, 0.0, 0.0,
                 ws.dscal + (2 * (k - 1) + 1), 0.0};
      in.nrm1 = dev_norm(k - 1);
      in.nrm2 = k >= 2 ? dev_norm(k - 2) : nullptr;
      const SweepOut so{ws.basis[k], ws.pnorm, ws.pdot};
      // single-pass sizes compute z_k in the same pass; otherwise only the forming pass
      HIP_TRY(hpsi_sweep(prec, n, c, reg->d_dtab, in, ws.z, ws.t, so, kFirstPass, L.s));
      HIP_TRY(finalize_sum(ws.pnorm, np_norm, ws.dscal + 2 * k, L.s));
      if (single) HIP_TRY(finalize_sum(ws.pdot, np_dot, ws.dscal + 2 * k + 1, L.s));
      HIP_TRY(hipMemcpyAsync(reg->h_scal + 2 * k - 1, ws.dscal + 2 * k - 1, 2 * sizeof(double),
                             hipMemcpyDeviceToHost, L.s));
      HIP_TRY(hipEventRecord(reg->ev[k], L.s));
      return RSV_OK;
    };
    // z_k = H u_k: the remaining passes, or all of them when u_k was re-orthogonalised
    // after the forming pass
    auto later = [&](int k) -> int {
      if (single && !reorth) return RSV_OK;
      const SweepIn in2{ws.basis[k], nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
      const SweepOut so2{nullptr, nullptr, ws.pdot};
      HIP_TRY(hpsi_sweep(prec, n, c, reg->d_dtab, in2, ws.z, ws.t, so2,
                         reorth ? kAllPasses : kLaterPasses, L.s));
      HIP_TRY(finalize_sum(ws.pdot, np_dot, ws.dscal + 2 * k + 1, L.s));
      return RSV_OK;
    };
    RSV_TRY(form(1));
    for (int k = 1; k <= kmax; ++k) {
      // run ahead: queue iteration k+1 before reading iteration k's scalars, so the device
      // never waits for the host (one iteration is wasted when k converges)
      const bool speculate = ahead && k < kmax;
      if (speculate) {
        RSV_TRY(later(k));
        RSV_TRY(form(k + 1));
        L.st->krylov_iters += 1;
        L.st->bytes_hpsi += hbytes;
      }
      HIP_TRY(hipEventSynchronize(reg->ev[k]));
      double ab[2] = {reg->h_scal[2 * k - 1], reg->h_scal[2 * k]};  // <u_{k-1}, z_{k-1}>, |u_k|^2
      if (!std::isfinite(ab[0]) || !std::isfinite(ab[1]))
        return fail(RSV_ENUMERIC, "Lanczos coefficient not finite at iteration %d", k);
      const double sk1 = L.scale[k - 1];
      L.alpha[k - 1] = sk1 * sk1 * ab[0];
      if (reorth) {
        RSV_TRY(reorthogonalise(L, k, &ab[1]));
        if (!std::isfinite(ab[1]))
          return fail(RSV_ENUMERIC, "Lanczos coefficient not finite at iteration %d", k);
      }
      const double bk = std::sqrt(std::max(ab[1], 0.0));  // beta_{k-1}
      m = k;
      double ylast = 0.0;
      RSV_TRY(last_component(L, m, remaining, &ylast));
      if (bk * ylast * nrm <= tol || bk == 0.0) break;
      if (k == kmax) {
        // Not converged: advance by the longest part of the step that this basis already
        // resolves (same H_k, so the split is exact), then restart from the new state.
        // The first dyadic fraction that converges brackets it; bisection refines it.
        bool ok = false;
        double bad = remaining;
        for (int d = 1; d <= max_depth && !ok; ++d) {
          sub = std::ldexp(remaining, -d);
          RSV_TRY(last_component(L, m, sub, &ylast));
          ok = bk * ylast * nrm <= tol;
          if (!ok) bad = sub;
        }
        if (!ok) return fail(RSV_ENOTCONV, "Krylov exponential not converged with kmax = %d", kmax);
        for (int it = 0; it < 10; ++it) {
          const double mid = 0.5 * (sub + bad);
          RSV_TRY(last_component(L, m, mid, &ylast));
          if (bk * ylast * nrm <= tol) sub = mid;
          else bad = mid;
        }
        L.st->substeps += 1;
        break;
      }
      L.beta[k - 1] = bk;
      L.scale[k] = 1.0 / bk;
      if (!speculate) {
        RSV_TRY(later(k));
        RSV_TRY(form(k + 1));
        L.st->krylov_iters += 1;
        L.st->bytes_hpsi += hbytes;
      }
    }
    L.st->krylov_max = std::max<int64_t>(L.st->krylov_max, m);
    if (tridiag_expm(m, L.alpha, L.beta, L.dir * sub, L.yre, L.yim, L.work.data()) != 0)
      return fail(RSV_ENUMERIC, "tridiagonal eigensolver failed (m = %d)", m);
    CombineCoef cc;
    std::memset(&cc, 0, sizeof cc);
    cc.m = m;
    for (int l = 0; l < m; ++l) {
      cc.re[l] = nrm * L.yre[l] * L.scale[l];
      cc.im[l] = nrm * L.yim[l] * L.scale[l];
      cc.x[l] = ws.basis[l];
    }
    if (obs && sub == remaining)
      HIP_TRY(krylov_combine_occ(prec, n, cc, ws.z, ws.pnorm, L.occ_partial, obs, L.s));
    else
      HIP_TRY(krylov_combine(prec, n, cc, ws.z, ws.pnorm, L.s));
    HIP_TRY(finalize_sum(ws.pnorm, vec_num_partials(prec, n), ws.dscal + kNormSlot, L.s));
    std::swap(ws.basis[0], ws.z);
    RSV_TRY(fetch_scalars(L, kNormSlot, 1, &L.norm2));
    remaining = (sub == remaining) ? 0.0 : remaining - sub;
  }
  return RSV_OK;
}

}  // namespace

namespace {

// Device memory borrowed from an allocator for the duration of one call.
struct Borrowed {
  Allocator* a = nullptr;
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s = nullptr;
  ~Borrowed() {
    if (p) {
      (void)hipStreamSynchronize(s);
      a->release(p, bytes);
    }
  }
};

}  // namespace

int evolve(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o, void* d_psi,
           hipStream_t s, rsv_stats* st, int obs_every, double* obs_out) {
  if (!reg) return fail(RSV_EINVAL, "register is NULL");
  if (!d_psi) return fail(RSV_EINVAL, "state pointer is NULL");
  RSV_TRY(check_pulses(pl, reg->n));
  int64_t first = 0, count = 0;
  RSV_TRY(check_opts(o, pl, &first, &count));
  if (obs_out && obs_every < 1) return fail(RSV_EINVAL, "observation interval must be >= 1");
  const int64_t n_obs = obs_out ? count / obs_every : 0;
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipSetDevice(reg->ctx->device));
  RSV_TRY(workspace_acquire(reg, o->kmax));
  Workspace& ws = reg->ws;
  const int n = reg->n, prec = reg->prec;
  const size_t vb = vec_bytes(n, prec);
  HIP_TRY(hipMemcpyAsync(ws.basis[0], d_psi, vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(norm2_partial(prec, n, ws.basis[0], ws.pnorm, s));
  HIP_TRY(finalize_sum(ws.pnorm, vec_num_partials(prec, n), ws.dscal + kNormSlot, s));
  Lanczos L;
  L.reg = reg;
  L.s = s;
  L.st = st;
  std::memset(L.alpha, 0, sizeof L.alpha);
  std::memset(L.beta, 0, sizeof L.beta);
  std::memset(L.scale, 0, sizeof L.scale);
  L.work.assign(tridiag_work_doubles(kMaxKrylov), 0.0);
  RSV_TRY(fetch_scalars(L, kNormSlot, 1, &L.norm2));
  // observed steps: fused occupation partials, then n + 1 sums per observation
  Borrowed ob;
  double* obs_dev = nullptr;
  if (n_obs > 0) {
    const size_t part = (size_t)combine_occ_partial_doubles(n);
    ob.a = reg->alloc;
    ob.s = s;
    ob.bytes = (part + (size_t)n_obs * (n + 1)) * sizeof(double);
    RSV_TRY(reg->alloc->alloc(ob.bytes, &ob.p));
    L.occ_partial = (double*)ob.p;
    obs_dev = L.occ_partial + part;
  }
  const double tau = o->dt_ns * 1e-3;  // us
  for (int64_t k = first; k < first + count; ++k) {
    const StepCoef c = step_coef(pl, n, k, o->dt_ns);
    const int64_t j = k - first + 1;  // steps done after this one
    double* slot = (n_obs > 0 && j % obs_every == 0) ? obs_dev + (j / obs_every - 1) * (n + 1)
                                                      : nullptr;
    RSV_TRY(propagate(L, c, tau, o->tol, o->kmax, o->max_substep_depth, o->reorth != 0, slot));
    st->steps += 1;
  }
  HIP_TRY(hipMemcpyAsync(d_psi, ws.basis[0], vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (n_obs > 0) {
    std::vector<double> h((size_t)n_obs * (n + 1));
    HIP_TRY(hipMemcpy(h.data(), obs_dev, h.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < n_obs; ++r) {
      const double* v = h.data() + r * (n + 1);
      if (!(v[0] > 0.0)) return fail(RSV_ENUMERIC, "observed state has zero norm");
      for (int i = 0; i < n; ++i) obs_out[r * n + i] = v[1 + (n - 1 - i)] / v[0];
    }
  }
  st->norm_final = std::sqrt(L.norm2);
  st->seconds += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return RSV_OK;
}

int krylov_exp(rsv_register* reg, const StepCoef& c, double tau, double dir, double tol,
               int kmax, int max_depth, void* d_psi, hipStream_t s, rsv_stats* st) {
  if (!reg || !d_psi) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(reg->ctx->device));
  RSV_TRY(workspace_acquire(reg, kmax));
  Workspace& ws = reg->ws;
  const int n = reg->n, prec = reg->prec;
  const size_t vb = vec_bytes(n, prec);
  HIP_TRY(hipMemcpyAsync(ws.basis[0], d_psi, vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(norm2_partial(prec, n, ws.basis[0], ws.pnorm, s));
  HIP_TRY(finalize_sum(ws.pnorm, vec_num_partials(prec, n), ws.dscal + kNormSlot, s));
  Lanczos L;
  L.reg = reg;
  L.s = s;
  L.st = st;
  L.dir = dir < 0 ? -1.0 : 1.0;
  std::memset(L.alpha, 0, sizeof L.alpha);
  std::memset(L.beta, 0, sizeof L.beta);
  std::memset(L.scale, 0, sizeof L.scale);
  L.work.assign(tridiag_work_doubles(kMaxKrylov), 0.0);
  RSV_TRY(fetch_scalars(L, kNormSlot, 1, &L.norm2));
  if (L.norm2 == 0.0) return RSV_OK;  // exp(...) 0 = 0
  RSV_TRY(propagate(L, c, tau, tol, kmax, max_depth, false));
  HIP_TRY(hipMemcpyAsync(d_psi, ws.basis[0], vb, hipMemcpyDeviceToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RSV_OK;
}

// ------------------------------------------------------------------------------ outputs
size_t occupation_scratch_bytes(int n) { return round_up((size_t)(occ_num_partials(n) + 64) * 8); }

size_t sample_scratch_bytes(int n, int shots) {
  return round_up((size_t)sample_scratch_doubles(n) * 8) + round_up((size_t)shots * 8);
}

int occupations_with(int n, int prec, const void* d_psi, void* d_scratch, double* h_tmp,
                     double* out, hipStream_t s) {
  double* part = (double*)d_scratch;
  double* res = part + occ_num_partials(n);
  HIP_TRY(occupations(prec, n, d_psi, part, res, s));
  HIP_TRY(hipMemcpyAsync(h_tmp, res, (n + 1) * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!(h_tmp[0] > 0.0)) return fail(RSV_ENUMERIC, "state has zero norm");
  for (int i = 0; i < n; ++i) out[i] = h_tmp[1 + (n - 1 - i)] / h_tmp[0];
  return RSV_OK;
}

int sample_with(int n, int prec, const void* d_psi, uint64_t seed, int shots, void* d_scratch,
                uint64_t* out, hipStream_t s) {
  if (shots <= 0) return RSV_OK;
  double* scratch = (double*)d_scratch;
  uint64_t* d_idx = (uint64_t*)((char*)d_scratch + round_up((size_t)sample_scratch_doubles(n) * 8));
  HIP_TRY(sample(prec, n, d_psi, seed, shots, scratch, d_idx, s));
  HIP_TRY(hipMemcpyAsync(out, d_idx, (size_t)shots * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RSV_OK;
}

}  // namespace rsv
