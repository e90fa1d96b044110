// exp(A) of a small dense complex matrix, host FP64: scaling and squaring with the diagonal
// [6/6] Pade approximant (Golub & Van Loan, "Matrix Computations", Sec. 11.3, Algorithm
// 11.3.1): A is scaled by 2^-j with j = max(0, 1 + floor(log2 |A|_inf)), so |A/2^j|_inf <= 1/2,
// where the [6/6] approximant's relative backward error is below 1e-16; N(A) and D(A) are
// summed term by term, D F = N is solved by Gaussian elimination with partial pivoting, and F
// is squared j times.  The Arnoldi exponential of the Lindblad and gradient paths applies it
// to its upper Hessenberg matrix (m <= 65).
#include <cmath>
#include <complex>
#include <vector>

#include "arnoldi.h"

namespace rsv {

using cd = std::complex<double>;

namespace {

void matmul(int m, const cd* a, const cd* b, cd* c) {
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) {
      cd s = 0.0;
      for (int k = 0; k < m; ++k) s += a[i * m + k] * b[k * m + j];
      c[i * m + j] = s;
    }
}

// Solves D X = B for X (both m x m, row-major) in place in B; D is destroyed.
int solve(int m, cd* d, cd* b) {
  for (int col = 0; col < m; ++col) {
    int piv = col;
    for (int r = col + 1; r < m; ++r)
      if (std::abs(d[r * m + col]) > std::abs(d[piv * m + col])) piv = r;
    if (std::abs(d[piv * m + col]) == 0.0) return -1;
    if (piv != col)
      for (int k = 0; k < m; ++k) {
        std::swap(d[piv * m + k], d[col * m + k]);
        std::swap(b[piv * m + k], b[col * m + k]);
      }
    for (int r = col + 1; r < m; ++r) {
      const cd f = d[r * m + col] / d[col * m + col];
      if (f == 0.0) continue;
      for (int k = col; k < m; ++k) d[r * m + k] -= f * d[col * m + k];
      for (int k = 0; k < m; ++k) b[r * m + k] -= f * b[col * m + k];
    }
  }
  for (int col = m - 1; col >= 0; --col) {
    for (int k = 0; k < m; ++k) b[col * m + k] /= d[col * m + col];
    for (int r = 0; r < col; ++r) {
      const cd f = d[r * m + col];
      if (f == 0.0) continue;
      for (int k = 0; k < m; ++k) b[r * m + k] -= f * b[col * m + k];
    }
  }
  return 0;
}

}  // namespace

int dense_expm(int m, const cd* a, cd* out) {
  if (m < 1) return -1;
  double norm = 0.0;  // infinity norm
  for (int i = 0; i < m; ++i) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) s += std::abs(a[i * m + j]);
    norm = std::max(norm, s);
  }
  if (!std::isfinite(norm)) return -1;
  int j = 0;
  if (norm > 0.0) j = std::max(0, 1 + (int)std::floor(std::log2(norm)));
  const double scale = std::ldexp(1.0, -j);
  const size_t mm = (size_t)m * m;
  std::vector<cd> as(mm), x(mm), t(mm), num(mm), den(mm);
  for (size_t i = 0; i < mm; ++i) as[i] = a[i] * scale;
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < m; ++k) {
      const cd e = (i == k) ? 1.0 : 0.0;
      x[i * m + k] = e;
      num[i * m + k] = e;
      den[i * m + k] = e;
    }
  const int q = 6;
  double c = 1.0;
  for (int k = 1; k <= q; ++k) {
    c = c * (q - k + 1) / ((2.0 * q - k + 1) * k);
    matmul(m, as.data(), x.data(), t.data());
    x.swap(t);
    const double sgn = (k % 2) ? -1.0 : 1.0;
    for (size_t i = 0; i < mm; ++i) {
      num[i] += c * x[i];
      den[i] += sgn * c * x[i];
    }
  }
  if (solve(m, den.data(), num.data()) != 0) return -1;
  for (int s = 0; s < j; ++s) {
    matmul(m, num.data(), num.data(), t.data());
    num.swap(t);
  }
  for (size_t i = 0; i < mm; ++i) out[i] = num[i];
  return 0;
}

}  // namespace rsv
