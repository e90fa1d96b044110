// Gradients of emulator outputs with respect to the pulse samples (Sec. IV: the emulator is
// differentiable, so derivatives of expectation values with respect to the pulse can drive
// optimisation), by the adjoint method on the piecewise-constant propagator of eq. (6).
//
// C = <psi_K| O |psi_K> with O = sum_i w_i n_i and psi_K = U_{K-1} ... U_0 psi_0,
// U_k = exp(-i H_k dt).  For a parameter theta of step k,
//   dC/dtheta = 2 Re <lambda_{k+1}| dU_k/dtheta |psi_k>,  lambda_{k+1} = U_{k+1}^+ ... U_{K-1}^+ O psi_K.
// dU_k/dtheta psi_k is the Frechet derivative of the exponential at -i H_k dt in the
// direction -i V dt (V = dH/dtheta), read from the exponential of the block operator
//   exp(dt A) (0, psi_k) = (dU_k/dtheta psi_k, U_k psi_k),  A = -i [[H_k, V], [0, H_k]]
// (Higham, "Functions of Matrices", the block-triangular form of the Frechet derivative),
// which is evaluated on the device by the Arnoldi exponential (A is not Hermitian).  The
// backward sweep recovers psi_k = U_k^+ psi_{k+1} and lambda_k = U_k^+ lambda_{k+1} with the
// Lanczos exponential run backwards in time (unitary, so no states are stored).  With the
// global drive, theta is the step's Omega (V = sum_i (e^{-i phi}|1><0|_i + e^{i phi}|0><1|_i)/2)
// and its delta (V = -sum_i n_i); a sample x_j enters steps through the midpoint rule of
// Sec. III, theta_k = (x_floor(m) + x_ceil(m)) / 2, so dC/dx_j sums half of each such step's
// derivative.  Every operator here is H psi of the library's kernels: V and O are H psi with
// zero interaction tables and chosen drive and detuning.
#include <hip/hip_runtime.h>

#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "arnoldi.h"
#include "engine.h"

using namespace rsv;

namespace {

size_t up256(size_t b) { return (b + 255) / 256 * 256; }

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

// out = sum_l coef_l x_l for up to two vectors (in place allowed: element-wise).
int combine2(int prec, int n, void* out, const void* x0, double r0, double i0, const void* x1,
             double r1, double i1, double* partial, hipStream_t s) {
  CombineCoef cc;
  std::memset(&cc, 0, sizeof cc);
  cc.m = x1 ? 2 : 1;
  cc.x[0] = x0;
  cc.re[0] = r0;
  cc.im[0] = i0;
  if (x1) {
    cc.x[1] = x1;
    cc.re[1] = r1;
    cc.im[1] = i1;
  }
  HIP_TRY(krylov_combine(prec, n, cc, out, partial, s));
  return RSV_OK;
}

}  // namespace

extern "C" {

int rsv_gradient_occupations(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o,
                             const double* weights, const void* psi0_host, double* value,
                             double* grad_omega, double* grad_delta, rsv_stats* stats_out) {
  if (!reg || !pl || !weights || !value || !grad_omega || !grad_delta)
    return fail(RSV_EINVAL, "NULL argument");
  RSV_TRY(check_pulses(pl, reg->n));
  if (pl->per_site) return fail(RSV_EINVAL, "gradients are taken for global pulses");
  int64_t first = 0, count = 0;
  RSV_TRY(check_opts(o, pl, &first, &count));
  if (o->kmax > kMaxKrylov - 1) return fail(RSV_EINVAL, "kmax must be <= %d here", kMaxKrylov - 1);
  const int n = reg->n, prec = reg->prec;
  if (n + 1 > kMaxAtoms) return fail(RSV_EINVAL, "at most %d atoms", kMaxAtoms - 1);
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(weights[i])) return fail(RSV_EINVAL, "weights must be finite");
  const auto t0 = std::chrono::steady_clock::now();
  HIP_TRY(hipSetDevice(reg->ctx->device));
  hipStream_t s = nullptr;
  const size_t vraw = vec_bytes(n, prec), vb = up256(vraw);
  const size_t tabs = up256(diag_table_doubles(prec, n) * sizeof(double));
  const int64_t npd = sweep_dot_partials(prec, n);
  const int64_t npv = vec_num_partials(prec, n + 1);
  const size_t parts = up256((size_t)(npd + 2 * kDotGroup * npv + 8) * sizeof(double));
  // device: psi, lambda, V-product scratch, high-pass partial, zero tables, partial sums, the
  // augmented vector (two halves back to back), the Arnoldi space of the augmented operator
  const size_t fixed = 4 * vb + tabs + parts + up256(2 * vraw);
  Block blk(reg->alloc, s);
  RSV_TRY(blk.get(fixed + arnoldi_device_bytes(prec, n + 1, o->kmax)));
  char* p = (char*)blk.p;
  void* psi = p;
  void* lam = p + vb;
  void* tmp = p + 2 * vb;
  void* hb = p + 3 * vb;
  double* zt = (double*)(p + 4 * vb);
  double* part = (double*)(p + 4 * vb + tabs);
  double* res = part + npd + 2 * kDotGroup * npv;
  char* aug = p + 4 * vb + tabs + parts;  // [a | b], each 2^n amplitudes
  ArnoldiSpace sp;
  arnoldi_carve(p + fixed, reg->h_scal, prec, n + 1, o->kmax, &sp);
  HIP_TRY(hipMemsetAsync(zt, 0, tabs, s));
  if (psi0_host) {
    if (prec == kC128) {
      HIP_TRY(hipMemcpy(psi, psi0_host, vraw, hipMemcpyHostToDevice));
    } else {  // stage the complex128 input in the augmented vector (2 x 2^n complex64)
      HIP_TRY(hipMemcpy(aug, psi0_host, (size_t(1) << n) * 16, hipMemcpyHostToDevice));
      HIP_TRY(convert_from_c128(prec, n, aug, psi, s));
    }
  } else {
    HIP_TRY(hipMemsetAsync(psi, 0, vb, s));
    const double one128[2] = {1.0, 0.0};
    const float one64[2] = {1.0f, 0.0f};
    HIP_TRY(hipMemcpyAsync(psi, prec == kC128 ? (const void*)one128 : (const void*)one64,
                           amp_bytes(prec), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  rsv_stats st{};
  const double tau = o->dt_ns * 1e-3;
  for (int64_t k = first; k < first + count; ++k)  // forward sweep to psi_K
    RSV_TRY(krylov_exp(reg, step_coef(pl, n, k, o->dt_ns), tau, 1.0, o->tol, o->kmax,
                       o->max_substep_depth, psi, s, &st));
  // lambda_K = O psi_K (H psi with zero tables, no drive, delta_p = -w_p) and C = <psi_K, O psi_K>
  StepCoef oc;
  std::memset(&oc, 0, sizeof oc);
  oc.n = n;
  oc.mode = kCoefSite;
  for (int i = 0; i < n; ++i) oc.delta[n - 1 - i] = -weights[i];
  {
    const SweepIn in{psi, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
    const SweepOut so{nullptr, nullptr, part};
    HIP_TRY(hpsi_sweep(prec, n, oc, zt, in, lam, hb, so, kAllPasses, s));
    HIP_TRY(finalize_sum(part, npd, res, s));
    HIP_TRY(hipMemcpyAsync(reg->h_scal, res, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *value = reg->h_scal[0];
  }
  const int64_t ns = pl->n_samples;
  for (int64_t j = 0; j < ns; ++j) grad_omega[j] = grad_delta[j] = 0.0;
  // unit-Omega drive coefficients with the pulse's phase, step by step
  std::vector<double> ones(ns, 1.0), zeros(ns, 0.0);
  rsv_pulses unit = *pl;
  unit.omega = ones.data();
  unit.delta = zeros.data();
  for (int64_t k = first + count - 1; k >= first; --k) {
    const StepCoef c = step_coef(pl, n, k, o->dt_ns);
    RSV_TRY(krylov_exp(reg, c, tau, -1.0, o->tol, o->kmax, o->max_substep_depth, psi, s, &st));
    for (int which = 0; which < 2; ++which) {
      StepCoef v;
      if (which == 0) {  // dH/dOmega: the drive at unit Omega with the step's phase
        v = step_coef(&unit, n, k, o->dt_ns);
      } else {           // dH/ddelta = -sum n
        std::memset(&v, 0, sizeof v);
        v.n = n;
        for (int q = 0; q < n; ++q) v.delta[q] = 1.0;
      }
      v.mode = kCoefSite;
      // (a, b) -> -i (H a + V b, H b) on the augmented vector
      const OpFn op = [&](const void* in, void* out, hipStream_t st_) -> int {
        const char* ia = (const char*)in;
        const char* ib = ia + vraw;
        char* oa = (char*)out;
        char* ob = oa + vraw;
        const SweepOut none{nullptr, nullptr, nullptr};
        const SweepIn sa{ia, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
        const SweepIn sb{ib, nullptr, nullptr, 1.0, 0.0, 0.0, nullptr, 0.0};
        HIP_TRY(hpsi_sweep(prec, n, c, reg->d_dtab, sa, oa, hb, none, kAllPasses, st_));
        HIP_TRY(hpsi_sweep(prec, n, v, zt, sb, tmp, hb, none, kAllPasses, st_));
        RSV_TRY(combine2(prec, n, oa, oa, 0.0, -1.0, tmp, 0.0, -1.0, part, st_));
        HIP_TRY(hpsi_sweep(prec, n, c, reg->d_dtab, sb, ob, hb, none, kAllPasses, st_));
        RSV_TRY(combine2(prec, n, ob, ob, 0.0, -1.0, nullptr, 0.0, 0.0, part, st_));
        return RSV_OK;
      };
      HIP_TRY(hipMemsetAsync(aug, 0, vraw, s));
      HIP_TRY(hipMemcpyAsync(aug + vraw, psi, vraw, hipMemcpyDeviceToDevice, s));
      RSV_TRY(arnoldi_expm(op, sp, aug, tau, o->tol, o->max_substep_depth, s, &st));
      // g = 2 Re <lambda_{k+1}, dU_k/dtheta psi_k>
      DotGroup d{};
      d.g = 1;
      d.x[0] = lam;
      HIP_TRY(multi_dot(prec, n, d, aug, part, s));
      HIP_TRY(finalize_rows(part, vec_num_partials(prec, n), 1, res, s));
      HIP_TRY(hipMemcpyAsync(reg->h_scal, res, sizeof(double), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      const double g = 2.0 * reg->h_scal[0];
      if (!std::isfinite(g)) return fail(RSV_ENUMERIC, "gradient not finite at step %lld", (long long)k);
      double* grad = which == 0 ? grad_omega : grad_delta;
      const double m = (k + 0.5) * o->dt_ns;
      grad[(int64_t)std::floor(m)] += 0.5 * g;
      grad[(int64_t)std::ceil(m)] += 0.5 * g;
    }
    RSV_TRY(krylov_exp(reg, c, tau, -1.0, o->tol, o->kmax, o->max_substep_depth, lam, s, &st));
  }
  st.steps = count;
  st.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats_out) *stats_out = st;
  return RSV_OK;
}

}  // extern "C"
