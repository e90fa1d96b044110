// Open-system evolution by the Lindblad master equation (Sec. III.A), on the vectorised
// density matrix: rho_{k+1} = exp(dt L_k) rho_k with L_k the Liouvillian of step k (the same
// midpoint parameters as the closed system, Sec. III), exp(dt L_k) rho by the Arnoldi Krylov
// exponential (L is not Hermitian, so Lanczos does not apply).
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <vector>

#include "arnoldi.h"
#include "engine.h"
#include "lindblad.h"

using namespace rsv;

namespace {

hipStream_t as_stream(void* s) { return (hipStream_t)s; }

int check_rates(const rsv_lindblad* r) {
  if (!r) return fail(RSV_EINVAL, "rates are NULL");
  if (!(std::isfinite(r->relax_rate) && r->relax_rate >= 0.0 && std::isfinite(r->dephasing_rate) &&
        r->dephasing_rate >= 0.0))
    return fail(RSV_EINVAL, "rates must be finite and >= 0");
  return RSV_OK;
}

int check_register(const rsv_register* reg) {
  if (!reg) return fail(RSV_EINVAL, "register is NULL");
  if (reg->n > kMaxLindbladAtoms)
    return fail(RSV_EINVAL, "the density matrix of %d atoms exceeds the %d-atom limit", reg->n,
                kMaxLindbladAtoms);
  return RSV_OK;
}

LindbladCoef lindblad_coef(const StepCoef& c, const rsv_lindblad* r) {
  LindbladCoef l{};
  l.n = c.n;
  for (int p = 0; p < c.n; ++p) {
    l.up_re[p] = c.up_re[p];
    l.up_im[p] = c.up_im[p];
    l.dn_re[p] = c.dn_re[p];
    l.dn_im[p] = c.dn_im[p];
    l.delta[p] = c.delta[p];
  }
  l.gamma_r = r->relax_rate;
  l.gamma_phi = r->dephasing_rate;
  return l;
}

// Device memory from the register's allocator for one call.
struct Block {
  Allocator* a;
  void* p = nullptr;
  size_t bytes = 0;
  hipStream_t s;
  Block(Allocator* al, hipStream_t st) : a(al), s(st) {}
  int get(size_t b) {
    bytes = b;
    return a->alloc(b, &p);
  }
  ~Block() {
    if (p) {
      (void)hipStreamSynchronize(s);
      a->release(p, bytes);
    }
  }
};

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

// The register's 2^N interaction energies in FP64, built on first use and kept.
int energies(rsv_register* reg, hipStream_t s, const double** out) {
  if (!reg->d_efull) {
    void* p = nullptr;
    RSV_TRY(reg->alloc->alloc((size_t(1) << reg->n) * sizeof(double), &p));
    const hipError_t e = diag_build(kC128, reg->n, reg->d_ub, p, s);
    if (e != hipSuccess) {
      reg->alloc->release(p, (size_t(1) << reg->n) * sizeof(double));
      return fail(RSV_EDEVICE, "interaction energies: %s", hipGetErrorString(e));
    }
    reg->d_efull = (double*)p;
  }
  *out = reg->d_efull;
  return RSV_OK;
}

}  // namespace

extern "C" {

int rsv_lindblad_apply(rsv_register* reg, const rsv_pulses* pl, int64_t step, int dt_ns,
                       const rsv_lindblad* rates, const void* d_in, void* d_out, void* stream) {
  RSV_TRY(check_register(reg));
  RSV_TRY(check_rates(rates));
  if (!d_in || !d_out || d_in == d_out) return fail(RSV_EINVAL, "input and output must be distinct");
  RSV_TRY(check_pulses(pl, reg->n));
  if (dt_ns < 1) return fail(RSV_EINVAL, "dt_ns must be >= 1");
  const int64_t K = (pl->n_samples - 1) / dt_ns;
  if (step < 0 || step >= K) return fail(RSV_EINVAL, "step outside the pulse");
  HIP_TRY(hipSetDevice(reg->ctx->device));
  hipStream_t s = as_stream(stream);
  const double* e = nullptr;
  RSV_TRY(energies(reg, s, &e));
  const LindbladCoef lc = lindblad_coef(step_coef(pl, reg->n, step, dt_ns), rates);
  HIP_TRY(liouvillian_apply(reg->prec, lc, e, d_in, d_out, s));
  return RSV_OK;
}

int rsv_lindblad_evolve_device(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o,
                               const rsv_lindblad* rates, void* d_rho, void* stream,
                               rsv_stats* stats_out) {
  RSV_TRY(check_register(reg));
  RSV_TRY(check_rates(rates));
  if (!d_rho) return fail(RSV_EINVAL, "density matrix is NULL");
  RSV_TRY(check_pulses(pl, reg->n));
  int64_t first = 0, count = 0;
  RSV_TRY(check_opts(o, pl, &first, &count));
  if (o->kmax > kMaxKrylov - 1) return fail(RSV_EINVAL, "kmax must be <= %d here", kMaxKrylov - 1);
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipSetDevice(reg->ctx->device));
  hipStream_t s = as_stream(stream);
  const int n = reg->n, prec = reg->prec;
  const double* e = nullptr;
  RSV_TRY(energies(reg, s, &e));
  Block blk(reg->alloc, s);
  RSV_TRY(blk.get(arnoldi_device_bytes(prec, 2 * n, o->kmax)));
  ArnoldiSpace sp;
  arnoldi_carve(blk.p, reg->h_scal, prec, 2 * n, o->kmax, &sp);
  rsv_stats st{};
  const double tau = o->dt_ns * 1e-3;
  for (int64_t k = first; k < first + count; ++k) {
    const LindbladCoef lc = lindblad_coef(step_coef(pl, n, k, o->dt_ns), rates);
    const OpFn op = [&](const void* in, void* out, hipStream_t st_) -> int {
      HIP_TRY(liouvillian_apply(prec, lc, e, in, out, st_));
      return RSV_OK;
    };
    const int rc = arnoldi_expm(op, sp, d_rho, tau, o->tol, o->max_substep_depth, s, &st);
    if (rc != RSV_OK) {
      if (stats_out) *stats_out = st;
      return rc;
    }
    st.steps += 1;
  }
  HIP_TRY(norm2_partial(prec, 2 * n, d_rho, sp.partial, s));
  HIP_TRY(finalize_sum(sp.partial, vec_num_partials(prec, 2 * n), sp.dscal, s));
  double nrm2 = 0.0;
  HIP_TRY(hipMemcpyAsync(sp.h_scal, sp.dscal, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  nrm2 = sp.h_scal[0];
  st.norm_final = std::sqrt(nrm2);
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats_out) *stats_out = st;
  return RSV_OK;
}

int rsv_lindblad_occupations(rsv_ctx* ctx, int n, rsv_precision prec, const void* d_rho,
                             double* occ_out, double* trace_out, void* stream) {
  if (!ctx || !d_rho || !occ_out) return fail(RSV_EINVAL, "NULL argument");
  if (n < 1 || n > kMaxLindbladAtoms) return fail(RSV_EINVAL, "n_atoms must be in 1..%d", kMaxLindbladAtoms);
  if (prec != RSV_C128 && prec != RSV_C64) return fail(RSV_EINVAL, "unknown precision");
  HIP_TRY(hipSetDevice(ctx->device));
  hipStream_t s = as_stream(stream);
  const size_t dim = size_t(1) << n;
  Block d(ctx->dev, s);
  RSV_TRY(d.get(up256(dim * sizeof(double))));
  HIP_TRY(rho_diagonal(prec, n, d_rho, (double*)d.p, s));
  std::vector<double> h(dim);
  HIP_TRY(hipMemcpyAsync(h.data(), d.p, dim * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  double tr = 0.0;
  std::vector<double> acc(n, 0.0);
  for (size_t r = 0; r < dim; ++r) {
    tr += h[r];
    for (int p = 0; p < n; ++p)
      if ((r >> p) & 1) acc[p] += h[r];
  }
  if (!(tr > 0.0)) return fail(RSV_ENUMERIC, "density matrix has trace %g", tr);
  for (int i = 0; i < n; ++i) occ_out[i] = acc[n - 1 - i] / tr;
  if (trace_out) *trace_out = tr;
  return RSV_OK;
}

}  // extern "C"
