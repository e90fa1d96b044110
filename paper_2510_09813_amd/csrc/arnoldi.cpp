// Arnoldi Krylov exponential on device vectors, driven from the host (see arnoldi.h).
#include "arnoldi.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace rsv {

namespace {

using cd = std::complex<double>;
size_t up256(size_t b) { return (b + 255) / 256 * 256; }
constexpr int kScal = 2 * kMaxKrylov + 8;

int fetch(ArnoldiSpace& sp, int count, hipStream_t s, double* out) {
  HIP_TRY(hipMemcpyAsync(sp.h_scal, sp.dscal, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(out, sp.h_scal, count * sizeof(double));
  return RSV_OK;
}

// |x|^2 of a vector of the space.
int norm2(ArnoldiSpace& sp, const void* x, hipStream_t s, double* out) {
  HIP_TRY(norm2_partial(sp.prec, sp.nb, x, sp.partial, s));
  HIP_TRY(finalize_sum(sp.partial, vec_num_partials(sp.prec, sp.nb), sp.dscal, s));
  return fetch(sp, 1, s, out);
}

// <u_i, y> for i < k (Re, Im interleaved into dots[2 i], dots[2 i + 1]).
// <u_i, y> for i < k, and <y, y> after them when self_dot (in the same sweeps over y).
int dots_against(ArnoldiSpace& sp, int k, const void* y, hipStream_t s, double* dots,
                 bool self_dot = false) {
  const int64_t nw = vec_num_partials(sp.prec, sp.nb);
  const int total = k + (self_dot ? 1 : 0);
  for (int i0 = 0; i0 < total; i0 += kDotGroup) {
    DotGroup d{};
    d.g = std::min(kDotGroup, total - i0);
    for (int g = 0; g < d.g; ++g) d.x[g] = i0 + g < k ? sp.vec[i0 + g] : y;
    HIP_TRY(multi_dot(sp.prec, sp.nb, d, y, sp.partial, s));
    HIP_TRY(finalize_rows(sp.partial, nw, 2 * d.g, sp.dscal + 2 * i0, s));
  }
  return fetch(sp, 2 * total, s, dots);
}

int expm_once(const OpFn& op, ArnoldiSpace& sp, void* d_x, double tau, double tol, hipStream_t s,
              rsv_stats* st, bool* converged) {
  const int kmax = sp.kmax;
  std::vector<void*>& v = sp.vec;
  void* w = v[kmax + 1];
  void* t = v[kmax + 2];
  const size_t vb = (size_t(1) << sp.nb) * amp_bytes(sp.prec);
  double nx2 = 0.0;
  RSV_TRY(norm2(sp, d_x, s, &nx2));
  const double nx = std::sqrt(nx2);
  *converged = true;
  if (!std::isfinite(nx)) return fail(RSV_ENUMERIC, "state norm is not finite");
  if (nx == 0.0) return RSV_OK;
  HIP_TRY(hipMemcpyAsync(v[0], d_x, vb, hipMemcpyDeviceToDevice, s));
  std::vector<double> scale(kmax + 2, 0.0);
  scale[0] = 1.0 / nx;
  std::vector<cd> h((size_t)(kmax + 1) * kmax, 0.0);  // h[i * kmax + j], i <= j + 1
  auto H = [&](int i, int j) -> cd& { return h[(size_t)i * kmax + j]; };
  std::vector<cd> hm, e;
  std::vector<double> dots(2 * kMaxKrylov + 2);
  int m = 0;
  for (int j = 0; j < kmax; ++j) {
    RSV_TRY(op(v[j], w, s));  // w = Op u_j, v_j = s_j u_j
    st->krylov_iters += 1;
    // y = Op v_j = s_j w, orthogonalised against v_0..v_j by classical Gram-Schmidt; the first
    // pass applies s_j, so every stored vector has the size of a Hessenberg entry (no growth
    // by |Op|^j, which would overflow complex64 storage).  A second pass runs only when the
    // first removed most of y: |y'| < |y| / sqrt(2) (the criterion of Daniel, Gragg, Kaufman
    // and Stewart, 1976), the case where rounding in y' is no longer small against y'.
    double y2 = 0.0, beta2 = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
      const double f = pass == 0 ? scale[j] : 1.0;
      RSV_TRY(dots_against(sp, j + 1, w, s, dots.data(), pass == 0));
      if (pass == 0) y2 = f * f * dots[2 * (j + 1)];
      CombineCoef cc;
      std::memset(&cc, 0, sizeof cc);
      cc.m = j + 2;
      cc.re[0] = f;
      cc.x[0] = w;
      for (int i = 0; i <= j; ++i) {
        const cd d(dots[2 * i], dots[2 * i + 1]);
        if (!std::isfinite(d.real()) || !std::isfinite(d.imag()))
          return fail(RSV_ENUMERIC, "Arnoldi inner product not finite");
        H(i, j) += f * scale[i] * d;           // <v_i, y>
        const cd c = -f * scale[i] * scale[i] * d;  // y - v_i <v_i, y>
        cc.re[i + 1] = c.real();
        cc.im[i + 1] = c.imag();
        cc.x[i + 1] = v[i];
      }
      HIP_TRY(krylov_combine(sp.prec, sp.nb, cc, t, sp.partial, s));
      std::swap(w, t);
      HIP_TRY(finalize_sum(sp.partial, vec_num_partials(sp.prec, sp.nb), sp.dscal, s));
      RSV_TRY(fetch(sp, 1, s, &beta2));
      if (!std::isfinite(beta2)) return fail(RSV_ENUMERIC, "Arnoldi residual not finite");
      if (pass == 0 && beta2 >= 0.5 * y2) break;
    }
    // the scratch slots keep naming the two buffers that are not basis vectors, whichever
    // way the passes swapped them (the next call takes its scratch from these slots)
    v[kmax + 1] = w;
    v[kmax + 2] = t;
    const double beta = std::sqrt(std::max(beta2, 0.0));
    H(j + 1, j) = beta;  // h_{j+1,j} = |y - sum_i v_i <v_i, y>|
    m = j + 1;
    hm.assign((size_t)m * m, 0.0);
    for (int r = 0; r < m; ++r)
      for (int c = 0; c < m; ++c) hm[(size_t)r * m + c] = tau * H(r, c);
    e.assign((size_t)m * m, 0.0);
    if (dense_expm(m, hm.data(), e.data()) != 0)
      return fail(RSV_ENUMERIC, "Hessenberg exponential failed (m = %d)", m);
    const double est = nx * std::abs(H(j + 1, j)) * std::abs(e[(size_t)(m - 1) * m]);
    const bool done = !(est > tol) || beta == 0.0;
    if (done || j + 1 == kmax) {
      if (!done) {
        *converged = false;
        return RSV_OK;
      }
      st->krylov_max = std::max<int64_t>(st->krylov_max, m);
      CombineCoef cc;
      std::memset(&cc, 0, sizeof cc);
      cc.m = m;
      for (int l = 0; l < m; ++l) {
        const cd y = nx * scale[l] * e[(size_t)l * m];
        cc.re[l] = y.real();
        cc.im[l] = y.imag();
        cc.x[l] = v[l];
      }
      HIP_TRY(krylov_combine(sp.prec, sp.nb, cc, d_x, sp.partial, s));
      return RSV_OK;
    }
    scale[j + 1] = 1.0 / beta;
    std::swap(v[j + 1], v[kmax + 1]);  // the orthogonalised residual becomes u_{j+1}
    w = v[kmax + 1];
  }
  *converged = false;
  return RSV_OK;
}

int expm_depth(const OpFn& op, ArnoldiSpace& sp, void* d_x, double tau, double tol, int depth,
               int max_depth, hipStream_t s, rsv_stats* st) {
  bool ok = false;
  RSV_TRY(expm_once(op, sp, d_x, tau, tol, s, st, &ok));
  if (ok) return RSV_OK;
  if (depth >= max_depth)
    return fail(RSV_ENOTCONV, "Arnoldi exponential not converged with kmax = %d", sp.kmax);
  st->substeps += 1;
  RSV_TRY(expm_depth(op, sp, d_x, 0.5 * tau, tol, depth + 1, max_depth, s, st));
  return expm_depth(op, sp, d_x, 0.5 * tau, tol, depth + 1, max_depth, s, st);
}

}  // namespace

size_t arnoldi_device_bytes(int prec, int nb, int kmax) {
  const size_t vb = up256((size_t(1) << nb) * amp_bytes(prec));
  const size_t part = up256((size_t)2 * kDotGroup * vec_num_partials(prec, nb) * sizeof(double));
  return (size_t)(kmax + 3) * vb + part + up256(kScal * sizeof(double));
}

void arnoldi_carve(void* block, double* h_scal, int prec, int nb, int kmax, ArnoldiSpace* sp) {
  const size_t vb = up256((size_t(1) << nb) * amp_bytes(prec));
  char* p = (char*)block;
  sp->prec = prec;
  sp->nb = nb;
  sp->kmax = kmax;
  sp->vec.assign(kmax + 3, nullptr);
  for (int i = 0; i < kmax + 3; ++i, p += vb) sp->vec[i] = p;
  sp->partial = (double*)p;
  p += up256((size_t)2 * kDotGroup * vec_num_partials(prec, nb) * sizeof(double));
  sp->dscal = (double*)p;
  sp->h_scal = h_scal;
}

int arnoldi_expm(const OpFn& op, ArnoldiSpace& sp, void* d_x, double tau, double tol,
                 int max_depth, hipStream_t s, rsv_stats* st) {
  if (sp.kmax < 2 || sp.kmax > kMaxKrylov - 1) return fail(RSV_EINVAL, "kmax must be in 2..%d", kMaxKrylov - 1);
  return expm_depth(op, sp, d_x, tau, tol, 0, max_depth, s, st);
}

}  // namespace rsv
