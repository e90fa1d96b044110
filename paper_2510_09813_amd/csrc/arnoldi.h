// Arnoldi Krylov exponential x <- exp(tau Op) x for non-Hermitian operators on device vectors
// (the Lindblad equation's Liouvillian, the augmented operator of the pulse gradients), and
// the dense matrix exponential of its small Hessenberg matrix.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <functional>
#include <vector>

#include "engine.h"

namespace rsv {

// exp(a) of an m x m complex matrix (row-major), host FP64; 0 on success.
int dense_expm(int m, const std::complex<double>* a, std::complex<double>* out);

// Device vectors of 2^nb amplitudes (storage precision prec): the Krylov basis (kmax + 1
// vectors, kept unnormalised), two more vectors, partial sums and device scalars.
struct ArnoldiSpace {
  int prec = 0, nb = 0, kmax = 0;
  std::vector<void*> vec;  // kmax + 3 vectors: basis then two scratch
  double* partial = nullptr;
  double* dscal = nullptr;
  double* h_scal = nullptr;  // pinned host copy of dscal
};
size_t arnoldi_device_bytes(int prec, int nb, int kmax);
// Lays out the device block (arnoldi_device_bytes) and borrows pinned h_scal (>= 2 kMaxKrylov + 8
// doubles).
void arnoldi_carve(void* block, double* h_scal, int prec, int nb, int kmax, ArnoldiSpace* sp);

using OpFn = std::function<int(const void* in, void* out, hipStream_t s)>;

// x <- exp(tau Op) x with the Arnoldi process (classical Gram-Schmidt, a second pass when the
// first removes most of the new vector, FP64 inner products), y = exp(tau H_m) e_1 from the
// Hessenberg matrix, converged when
// |x| h_{m+1,m} |y_m| <= tol (the estimate of Saad 1992 used by the Lanczos path), x = |x| V_m y.
// Without convergence in kmax vectors the step is split in halves (exact for a constant
// operator), at most max_depth levels deep, else RSV_ENOTCONV.
int arnoldi_expm(const OpFn& op, ArnoldiSpace& sp, void* d_x, double tau, double tol,
                 int max_depth, hipStream_t s, rsv_stats* st);

}  // namespace rsv
