// Host FP64 exponentials of the library (csrc/tridiag.cpp, csrc/dense_expm.cpp) against each
// other, built with the sanitizers: exp(-i tau T) e_1 of random symmetric tridiagonal T by
// the implicit QR eigendecomposition, by the Pade scaling-and-squaring exponential of the
// same T as a dense matrix, and the convergence test's |y_{m-1}|; plus unit norm and the
// 1 x 1 closed form.  Prints "host_expm ok" when every check holds.
#include <cmath>
#include <complex>
#include <cstdio>
#include <random>
#include <vector>

namespace rsv {
int tridiag_expm(int m, const double* alpha, const double* beta, double tau, double* y_re,
                 double* y_im, double* work);
size_t tridiag_work_doubles(int m);
int tridiag_expm_last(int m, const double* alpha, const double* beta, double tau,
                      double* last_abs, double* work);
int dense_expm(int m, const std::complex<double>* a, std::complex<double>* out);
}  // namespace rsv

int main() {
  using cd = std::complex<double>;
  std::mt19937_64 gen(2510);
  std::uniform_real_distribution<double> u(-1.0, 1.0);
  int failures = 0;
  auto check = [&](bool ok, const char* what, int m, double v) {
    if (!ok) {
      std::printf("FAIL %s m=%d value=%.3e\n", what, m, v);
      ++failures;
    }
  };
  for (int m = 1; m <= 64; ++m) {
    for (int rep = 0; rep < 4; ++rep) {
      std::vector<double> a(m), b(m > 1 ? m - 1 : 1), yr(m), yi(m);
      for (int i = 0; i < m; ++i) a[i] = 3.0 * u(gen);
      for (int i = 0; i + 1 < m; ++i) b[i] = std::abs(2.0 * u(gen)) + 1e-3;
      const double tau = 0.05 + 0.6 * std::abs(u(gen));
      std::vector<double> work(rsv::tridiag_work_doubles(m));
      check(rsv::tridiag_expm(m, a.data(), b.data(), tau, yr.data(), yi.data(), work.data()) == 0,
            "tridiag_expm status", m, 0.0);
      std::vector<cd> dense((size_t)m * m, 0.0), e((size_t)m * m);
      for (int i = 0; i < m; ++i) {
        dense[(size_t)i * m + i] = cd(0.0, -tau * a[i]);
        if (i + 1 < m) {
          dense[(size_t)i * m + i + 1] = cd(0.0, -tau * b[i]);
          dense[(size_t)(i + 1) * m + i] = cd(0.0, -tau * b[i]);
        }
      }
      check(rsv::dense_expm(m, dense.data(), e.data()) == 0, "dense_expm status", m, 0.0);
      double err = 0.0, nrm = 0.0;
      for (int i = 0; i < m; ++i) {
        const cd y(yr[i], yi[i]);
        err = std::max(err, std::abs(y - e[(size_t)i * m]));
        nrm += std::norm(y);
      }
      check(err < 1e-12, "qr vs pade", m, err);
      check(std::abs(nrm - 1.0) < 1e-13, "unit norm", m, nrm - 1.0);
      double last = -1.0;
      check(rsv::tridiag_expm_last(m, a.data(), b.data(), tau, &last, work.data()) == 0,
            "tridiag_expm_last status", m, 0.0);
      const double want = std::abs(cd(yr[m - 1], yi[m - 1]));
      check(std::abs(last - want) < 1e-12, "last element", m, last - want);
    }
  }
  {  // 1 x 1: exp(-i tau a) exactly
    const double a = 1.7, tau = 0.3;
    double yr = 0, yi = 0;
    std::vector<double> work(rsv::tridiag_work_doubles(1));
    rsv::tridiag_expm(1, &a, &a, tau, &yr, &yi, work.data());
    check(std::abs(cd(yr, yi) - std::exp(cd(0.0, -tau * a))) < 1e-15, "1x1 closed form", 1, 0.0);
  }
  if (failures) return 1;
  std::printf("host_expm ok\n");
  return 0;
}
