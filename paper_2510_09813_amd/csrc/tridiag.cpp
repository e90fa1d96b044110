// Host FP64 part of the Krylov exponential (Sec. III.A): exp(-i tau T) e_1 for the Lanczos
// tridiagonal T.
//
// T is diagonalised by implicit symmetric QR steps with a Wilkinson shift, chasing the bulge
// with Givens rotations (Golub & Van Loan, "Matrix Computations", Sec. 8.3).  T stays small
// (at most 64 x 64), so the active block is kept as a dense matrix and every rotation
// updates only the rows and columns it touches inside the band.  With T = Q diag(l) Q^T:
//   y = Q exp(-i tau diag(l)) Q^T e_1,  y_j = sum_k Q[j][k] exp(-i tau l_k) Q[0][k].
// The convergence test needs only y_{m-1}, i.e. rows 0 and m-1 of Q: the "last" variant
// accumulates just those two rows, O(m) per rotation less work.
#include <cfloat>
#include <cmath>

#include "rsv_internal.h"

namespace rsv {

size_t tridiag_work_doubles(int m) { return (size_t)2 * m * m + 2 * (size_t)m; }

namespace {

// c, s with  c*x - s*z = r  and  s*x + c*z = 0.
inline void givens(double x, double z, double& c, double& s) {
  if (z == 0.0) {
    c = 1.0;
    s = 0.0;
  } else if (std::fabs(z) > std::fabs(x)) {
    const double t = -x / z;
    s = 1.0 / std::sqrt(1.0 + t * t);
    c = s * t;
  } else {
    const double t = -z / x;
    c = 1.0 / std::sqrt(1.0 + t * t);
    s = c * t;
  }
}

inline bool negligible(double off, double d0, double d1) {
  return std::fabs(off) <= DBL_EPSILON * (std::fabs(d0) + std::fabs(d1)) ||
         std::fabs(off) < DBL_MIN;
}

// Eigenvalues into the diagonal of t (m x m), eigenvectors into the columns of q.  With
// all_rows false only rows 0 and m-1 of q are kept up to date.
int tridiag_eig(int m, const double* alpha, const double* beta, double* t, double* q,
                bool all_rows) {
  for (int i = 0; i < m * m; ++i) t[i] = q[i] = 0.0;
  for (int i = 0; i < m; ++i) {
    t[i * m + i] = alpha[i];
    q[i * m + i] = 1.0;
    if (i + 1 < m) t[i * m + i + 1] = t[(i + 1) * m + i] = beta[i];
  }
  auto T = [&](int i, int j) -> double& { return t[i * m + j]; };
  auto rotate_q = [&](int i, int k, double c, double s) {
    const double a0 = q[i * m + k], a1 = q[i * m + k + 1];
    q[i * m + k] = c * a0 - s * a1;
    q[i * m + k + 1] = s * a0 + c * a1;
  };

  int hi = m - 1, iter = 0;
  while (hi > 0) {
    if (negligible(T(hi, hi - 1), T(hi - 1, hi - 1), T(hi, hi))) {
      T(hi, hi - 1) = T(hi - 1, hi) = 0.0;
      --hi;
      iter = 0;
      continue;
    }
    int lo = hi - 1;
    while (lo > 0 && !negligible(T(lo, lo - 1), T(lo - 1, lo - 1), T(lo, lo))) --lo;
    if (lo > 0) T(lo, lo - 1) = T(lo - 1, lo) = 0.0;
    if (++iter > 100) return -2;

    // Wilkinson shift: eigenvalue of the trailing 2x2 block closer to T(hi, hi)
    const double d = 0.5 * (T(hi - 1, hi - 1) - T(hi, hi));
    const double b = T(hi, hi - 1);
    const double den = d + std::copysign(std::hypot(d, b), d == 0.0 ? 1.0 : d);
    const double mu = T(hi, hi) - b * b / den;

    double x = T(lo, lo) - mu, z = T(lo + 1, lo);
    for (int k = lo; k < hi; ++k) {
      double c, s;
      givens(x, z, c, s);
      const int j0 = k > lo ? k - 1 : lo;
      const int j1 = k + 2 < hi ? k + 2 : hi;
      for (int j = j0; j <= j1; ++j) {  // rows k, k+1 of G^T T
        const double a0 = T(k, j), a1 = T(k + 1, j);
        T(k, j) = c * a0 - s * a1;
        T(k + 1, j) = s * a0 + c * a1;
      }
      for (int i = j0; i <= j1; ++i) {  // columns k, k+1 of (G^T T) G
        const double a0 = T(i, k), a1 = T(i, k + 1);
        T(i, k) = c * a0 - s * a1;
        T(i, k + 1) = s * a0 + c * a1;
      }
      if (all_rows) {
        for (int i = 0; i < m; ++i) rotate_q(i, k, c, s);  // Q <- Q G
      } else {
        rotate_q(0, k, c, s);
        if (m > 1) rotate_q(m - 1, k, c, s);
      }
      if (k + 1 < hi) {
        x = T(k + 1, k);
        z = T(k + 2, k);
      }
    }
  }
  return 0;
}

}  // namespace

// work: 2*m*m + 2*m doubles.
int tridiag_expm(int m, const double* alpha, const double* beta, double tau, double* y_re,
                 double* y_im, double* work) {
  if (m <= 0 || m > kMaxKrylov) return -1;
  double* t = work;
  double* q = work + m * m;
  const int rc = tridiag_eig(m, alpha, beta, t, q, true);
  if (rc) return rc;
  double* er = work + 2 * m * m;  // Q[0][k] exp(-i tau l_k)
  double* ei = er + m;
  for (int k = 0; k < m; ++k) {
    const double ph = -tau * t[k * m + k];
    er[k] = q[k] * std::cos(ph);
    ei[k] = q[k] * std::sin(ph);
  }
  for (int j = 0; j < m; ++j) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < m; ++k) {
      sr += q[j * m + k] * er[k];
      si += q[j * m + k] * ei[k];
    }
    y_re[j] = sr;
    y_im[j] = si;
  }
  return 0;
}

int tridiag_expm_last(int m, const double* alpha, const double* beta, double tau,
                      double* last_abs, double* work) {
  if (m <= 0 || m > kMaxKrylov) return -1;
  double* t = work;
  double* q = work + m * m;
  const int rc = tridiag_eig(m, alpha, beta, t, q, false);
  if (rc) return rc;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < m; ++k) {
    const double ph = -tau * t[k * m + k];
    const double w = q[(m - 1) * m + k] * q[k];
    sr += w * std::cos(ph);
    si += w * std::sin(ph);
  }
  *last_abs = std::hypot(sr, si);
  return 0;
}

}  // namespace rsv
