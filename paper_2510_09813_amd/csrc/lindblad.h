// Lindblad master equation on the vectorised density matrix (see lindblad.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "rsv_internal.h"

namespace rsv {

constexpr int kMaxLindbladAtoms = 14;  // 4^14 amplitudes: 4 GiB per complex128 vector

// H_k's drive coefficients and detunings by bit position (as StepCoef, per bit) and the
// dissipation rates (1/us).
struct LindbladCoef {
  int n;
  double up_re[kMaxLindbladAtoms], up_im[kMaxLindbladAtoms];
  double dn_re[kMaxLindbladAtoms], dn_im[kMaxLindbladAtoms];
  double delta[kMaxLindbladAtoms];
  double gamma_r, gamma_phi;
};

// y = L x for vectorised density matrices of 4^n amplitudes; e: the 2^n interaction energies
// (FP64, device).
hipError_t liouvillian_apply(int prec, const LindbladCoef& c, const double* e, const void* x,
                             void* y, hipStream_t s);
// out[r] = Re rho_rr for r < 2^n (device FP64).
hipError_t rho_diagonal(int prec, int n, const void* x, double* out, hipStream_t s);

}  // namespace rsv
