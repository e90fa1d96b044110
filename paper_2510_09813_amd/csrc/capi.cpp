// C ABI of librsv (include/rsv.h): argument checks and handle management around the engine.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

using namespace rsv;

namespace {

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// Temporary device scratch from the context for one output call.
struct Scratch {
  rsv_ctx* ctx;
  void* p = nullptr;
  size_t bytes = 0;
  double* h = nullptr;
  explicit Scratch(rsv_ctx* c) : ctx(c) {}
  int get(size_t b) {
    bytes = b;
    RSV_TRY(ctx->dev->alloc(b, &p));
    if (hipHostMalloc((void**)&h, 64 * sizeof(double), hipHostMallocDefault) != hipSuccess) {
      h = nullptr;
      return fail(RSV_EDEVICE, "hipHostMalloc failed");
    }
    return RSV_OK;
  }
  ~Scratch() {
    if (p) {
      (void)hipDeviceSynchronize();
      ctx->dev->release(p, bytes);
    }
    if (h) (void)hipHostFree(h);
  }
};

int occupations_impl(rsv_ctx* ctx, int n, int prec, const void* d_psi, double* out,
                     hipStream_t s) {
  RSV_TRY(check_state_args(n, prec));
  if (!ctx || !d_psi || !out) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  Scratch sc(ctx);
  RSV_TRY(sc.get(occupation_scratch_bytes(n)));
  return occupations_with(n, prec, d_psi, sc.p, sc.h, out, s);
}

int sample_impl(rsv_ctx* ctx, int n, int prec, const void* d_psi, uint64_t seed, int shots,
                uint64_t* out, hipStream_t s) {
  RSV_TRY(check_state_args(n, prec));
  if (!ctx || !d_psi || (shots > 0 && !out)) return fail(RSV_EINVAL, "NULL argument");
  if (shots < 0) return fail(RSV_EINVAL, "n_shots must be >= 0");
  if (shots == 0) return RSV_OK;
  HIP_TRY(hipSetDevice(ctx->device));
  Scratch sc(ctx);
  RSV_TRY(sc.get(sample_scratch_bytes(n, shots)));
  return sample_with(n, prec, d_psi, seed, shots, sc.p, out, s);
}

}  // namespace

extern "C" {

const char* rsv_version(void) { return "librsv 0.2 (gfx950)"; }

const char* rsv_last_error(void) { return last_error(); }

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
  c->dev = new (std::nothrow) DeviceAllocator(budget);
  if (!c->dev) {
    delete c;
    return fail(RSV_ENOMEM, "host allocation failed");
  }
  if (static_sample_scratch(hip_device, &c->static_scratch) != 0) {
    delete c->dev;
    delete c;
    return fail(RSV_EDEVICE, "device address of the static sampling scratch not available");
  }
  *out = c;
  return RSV_OK;
}

void rsv_ctx_destroy(rsv_ctx* ctx) {
  if (!ctx) return;
  delete ctx->dev;
  delete ctx;
}

size_t rsv_ctx_bytes_in_use(const rsv_ctx* ctx) { return ctx ? ctx->dev->in_use() : 0; }

size_t rsv_workspace_bytes(int n, int kmax, rsv_precision prec) {
  if (n < 1 || n > kMaxAtoms || kmax < 2 || kmax > kMaxKrylov) return 0;
  return workspace_bytes(n, kmax, prec) + register_bytes(n, prec) + vec_bytes(n, prec);
}

int rsv_register_create(rsv_ctx* ctx, int n, const double* xyz, double c6, rsv_precision prec,
                        rsv_register** out) {
  if (!out) return fail(RSV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx) return fail(RSV_EINVAL, "context is NULL");
  return register_create(ctx, ctx->dev, n, xyz, c6, prec, nullptr, nullptr, out);
}

void rsv_register_destroy(rsv_register* reg) { register_destroy(reg, nullptr); }

int rsv_register_diagonal(rsv_register* reg, void* d_out, void* stream) {
  if (!reg || !d_out) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(reg->ctx->device));
  hipStream_t s = as_stream(stream);
  HIP_TRY(diag_build(reg->prec, reg->n, reg->d_ub, d_out, s));
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
  if (step < 0 || step >= K)
    return fail(RSV_EINVAL, "step %lld outside the pulse (%lld steps)", (long long)step,
                (long long)K);
  HIP_TRY(hipSetDevice(reg->ctx->device));
  const TilePlan plan = make_tile_plan(reg->prec, reg->n);
  if (plan.n_hi_passes > 0 && !reg->d_hbuf)
    RSV_TRY(reg->alloc->alloc(vec_bytes(reg->n, reg->prec), &reg->d_hbuf));
  const StepCoef c = step_coef(pl, reg->n, step, dt_ns);
  hipStream_t s = as_stream(stream);
  const SweepIn in{d_in, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
  const SweepOut so{nullptr, nullptr, nullptr};
  HIP_TRY(hpsi_sweep(reg->prec, reg->n, c, reg->d_dtab, in, d_out, reg->d_hbuf, so, kAllPasses, s));
  return RSV_OK;
}

int rsv_evolve_device(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o,
                      void* d_psi, void* stream, rsv_stats* stats_out) {
  rsv_stats st{};
  const int rc = evolve(reg, pl, o, d_psi, as_stream(stream), &st);
  if (stats_out) *stats_out = st;
  return rc;
}

int rsv_evolve_device_observed(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o,
                               void* d_psi, void* stream, int every, double* occ_out,
                               rsv_stats* stats_out) {
  if (!occ_out) return fail(RSV_EINVAL, "occ_out is NULL");
  if (every < 1) return fail(RSV_EINVAL, "every must be >= 1");
  rsv_stats st{};
  const int rc = evolve(reg, pl, o, d_psi, as_stream(stream), &st, every, occ_out);
  if (stats_out) *stats_out = st;
  return rc;
}

int rsv_energy_device(rsv_register* reg, const rsv_pulses* pl, int64_t step, int dt_ns,
                      const void* d_psi, double* energy, void* stream) {
  if (!reg || !d_psi || !energy) return fail(RSV_EINVAL, "NULL argument");
  RSV_TRY(check_pulses(pl, reg->n));
  if (dt_ns < 1) return fail(RSV_EINVAL, "dt_ns must be >= 1");
  const int64_t K = (pl->n_samples - 1) / dt_ns;
  if (step < 0 || step >= K)
    return fail(RSV_EINVAL, "step %lld outside the pulse (%lld steps)", (long long)step,
                (long long)K);
  HIP_TRY(hipSetDevice(reg->ctx->device));
  const int n = reg->n, prec = reg->prec;
  const TilePlan plan = make_tile_plan(prec, n);
  if (plan.n_hi_passes > 0 && !reg->d_hbuf)
    RSV_TRY(reg->alloc->alloc(vec_bytes(n, prec), &reg->d_hbuf));
  // H psi, the partial sums of Re<psi, H psi> and of |psi|^2, their two sums
  const size_t vb = (vec_bytes(n, prec) + 255) / 256 * 256;
  const int64_t np_dot = sweep_dot_partials(prec, n), np_norm = vec_num_partials(prec, n);
  const size_t bytes = vb + (size_t)(np_dot + np_norm + 2) * sizeof(double);
  void* blk = nullptr;
  RSV_TRY(reg->alloc->alloc(bytes, &blk));
  hipStream_t s = as_stream(stream);
  double* pdot = (double*)((char*)blk + vb);
  double* pnorm = pdot + np_dot;
  double* res = pnorm + np_norm;
  const StepCoef c = step_coef(pl, n, step, dt_ns);
  const SweepIn in{d_psi, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
  const SweepOut so{nullptr, nullptr, pdot};
  hipError_t e = hpsi_sweep(prec, n, c, reg->d_dtab, in, blk, reg->d_hbuf, so, kAllPasses, s);
  if (e == hipSuccess) e = finalize_sum(pdot, np_dot, res, s);
  if (e == hipSuccess) e = norm2_partial(prec, n, d_psi, pnorm, s);
  if (e == hipSuccess) e = finalize_sum(pnorm, np_norm, res + 1, s);
  double h[2] = {0.0, 0.0};
  if (e == hipSuccess) e = hipMemcpyAsync(h, res, sizeof h, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipStreamSynchronize(s);
  reg->alloc->release(blk, bytes);
  if (e != hipSuccess) return fail(RSV_EDEVICE, "energy: %s", hipGetErrorString(e));
  if (!(h[1] > 0.0)) return fail(RSV_ENUMERIC, "state has zero norm");
  *energy = h[0] / h[1];
  return RSV_OK;
}

int rsv_correlations_device(rsv_ctx* ctx, int n, rsv_precision prec, const void* d_psi,
                            double* out, void* stream) {
  RSV_TRY(check_state_args(n, prec));
  if (!ctx || !d_psi || !out) return fail(RSV_EINVAL, "NULL argument");
  HIP_TRY(hipSetDevice(ctx->device));
  Scratch sc(ctx);
  RSV_TRY(sc.get((size_t)corr_scratch_doubles(n) * sizeof(double)));
  hipStream_t s = as_stream(stream);
  double* dev = nullptr;
  HIP_TRY(correlations(prec, n, d_psi, (double*)sc.p, &dev, s));
  std::vector<double> h(1 + (size_t)n * n);
  HIP_TRY(hipMemcpyAsync(h.data(), dev, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (!(h[0] > 0.0)) return fail(RSV_ENUMERIC, "state has zero norm");
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const int p = std::min(n - 1 - i, n - 1 - j), q = std::max(n - 1 - i, n - 1 - j);
      out[i * n + j] = h[1 + p * n + q] / h[0];
    }
  return RSV_OK;
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
  int rc = reg->ctx->dev->alloc(r->bytes, &r->d_psi);
  if (rc != RSV_OK) {
    delete r;
    return rc;
  }
  hipError_t e = hipSuccess;
  if (psi0_host) {
    const size_t b128 = (size_t(1) << n) * 16;
    if (prec == kC128) {
      e = hipMemcpy(r->d_psi, psi0_host, b128, hipMemcpyHostToDevice);
    } else {
      void* tmp = nullptr;
      rc = reg->ctx->dev->alloc(b128, &tmp);
      if (rc == RSV_OK) {
        e = hipMemcpy(tmp, psi0_host, b128, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = convert_from_c128(prec, n, tmp, r->d_psi, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        reg->ctx->dev->release(tmp, b128);
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
  if (rc == RSV_OK && e != hipSuccess)
    rc = fail(RSV_EDEVICE, "state upload: %s", hipGetErrorString(e));
  if (rc == RSV_OK) rc = evolve(reg, pl, o, r->d_psi, nullptr, &r->stats);
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
  RSV_TRY(r->ctx->dev->alloc(b128, &tmp));
  hipError_t e = convert_to_c128(r->prec, r->n, r->d_psi, tmp, nullptr);
  if (e == hipSuccess) e = hipMemcpy(host, tmp, b128, hipMemcpyDeviceToHost);
  r->ctx->dev->release(tmp, b128);
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
  r->ctx->dev->release(r->d_psi, r->bytes);
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

int rsv_sample_device_static(rsv_ctx* ctx, int n, rsv_precision prec, const void* d_psi,
                             uint64_t seed, int shots, uint64_t* out, void* stream) {
  RSV_TRY(check_state_args(n, prec));
  if (!ctx || !d_psi || (shots > 0 && !out)) return fail(RSV_EINVAL, "NULL argument");
  if (shots < 0 || shots > kStaticMaxShots)
    return fail(RSV_EINVAL, "n_shots must be in 0..%d for the allocation-free sampler",
                kStaticMaxShots);
  if (shots == 0) return RSV_OK;
  if (!ctx->static_scratch) return fail(RSV_EDEVICE, "static scratch not resolved");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  // every scratch word is written before it is read (block sums, their scan, the indices)
  double* scan = (double*)ctx->static_scratch;
  uint64_t* d_idx = (uint64_t*)((char*)ctx->static_scratch + static_sample_idx_offset_bytes());
  HIP_TRY(sample(prec, n, d_psi, seed, shots, scan, d_idx, s));
  HIP_TRY(hipMemcpyAsync(out, d_idx, (size_t)shots * sizeof(uint64_t), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  return RSV_OK;
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
