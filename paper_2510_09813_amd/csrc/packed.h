// Packed small-job evolution: one workgroup runs one whole job (see packed.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "rsv.h"
#include "rsv_internal.h"

namespace rsv {

constexpr int kMaxPackBits = 13;     // largest n in either precision
constexpr int kPackOccOffset = 8;    // out[8 + p]: sum |psi_b|^2 b_p

// One job of a packed launch; every pointer is device memory.
struct PackedJob {
  int n, dt_ns, kmax, max_depth, per_site;
  int init_zero;  // 1: start from |0...0> instead of reading psi
  int64_t first_step, n_steps, n_samples;
  double tol;
  const double* omega;
  const double* delta;
  const double* phi;  // may be null
  const void* diag;   // interaction diagonal E_b in the storage precision
  void* psi;          // state in / out
  void* basis;        // (kmax + 1) vectors
  double* out;        // [0] status, [1] H applications, [2] largest Krylov dimension,
                      // [3] sub-steps, [4] |psi|^2, [8 + p] occupation numerators
};

int packed_max_atoms(int prec);
hipError_t packed_evolve(int prec, const PackedJob* d_jobs, int count, hipStream_t s);

}  // namespace rsv
