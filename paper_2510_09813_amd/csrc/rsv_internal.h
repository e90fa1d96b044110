// Internal declarations shared by the HIP kernels, the host solver and the C ABI of librsv.
//
// Index convention: the amplitude index b of a 2^n state vector holds the level of atom i
// (0-based) in bit n-1-i, so atom 0 is the most significant bit (row-major c_{i1...iN},
// Sec. II.B).  Kernels work with BIT positions p = n-1-i; the host converts per-atom data.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace rsv {

constexpr int kMaxAtoms = 30;
constexpr int kBlock = 256;       // threads per workgroup for every streaming kernel
constexpr int kMaxKrylov = 64;

enum Prec : int { kC128 = 0, kC64 = 1 };

inline size_t amp_bytes(int prec) { return prec == kC128 ? 16 : 8; }
inline size_t real_bytes(int prec) { return prec == kC128 ? 8 : 4; }

// One constant Hamiltonian H_k of eq. (3) with the drive phase, by bit position p:
//   (H x)_b = (E_b - sum_p delta[p] b_p) x_b + sum_p c_p(b_p) x_{b ^ 2^p}
// with c_p(1) = up[p] = Omega/2 e^{-i phi} (= <1|h|0>) and c_p(0) = dn[p] = Omega/2 e^{+i phi}.
// site == 0 means every bit shares index 0 (a global drive).
struct StepCoef {
  int n;
  int site;
  double up_re[kMaxAtoms], up_im[kMaxAtoms];
  double dn_re[kMaxAtoms], dn_im[kMaxAtoms];
  double delta[kMaxAtoms];
};

// Krylov combination: out = sum_l (re_l + i im_l) * x_l, x_l device vectors.
struct CombineCoef {
  int m;
  double re[kMaxKrylov], im[kMaxKrylov];
  const void* x[kMaxKrylov];
};

// --------------------------------------------------------------------------- H|psi>
// Tile geometry of the H|psi> passes for a precision: the low pass covers bits [0, lo_bits);
// each high pass covers up to hi_bits - r_bits high bits plus r_bits contiguous low bits.
struct TilePlan {
  int n, lo_bits, hi_bits, r_bits;
  int n_hi_passes;
  int flip_lo[kMaxAtoms], flip_hi[kMaxAtoms], tile_a[kMaxAtoms];
};
TilePlan make_tile_plan(int prec, int n);

// Number of per-workgroup partial sums hpsi_apply writes (0 when no partials requested).
int64_t hpsi_num_partials(int prec, int n);

// out = sx * H x + (prev ? -cprev * prev : 0), optionally partial[wg] = Re<sx x, out> per
// workgroup of the low pass (FP64).  tbuf (one vector) is required when n > lo_bits.
hipError_t hpsi_apply(int prec, int n, const StepCoef& c, const void* diag, const void* x,
                      double sx, void* out, const void* prev, double cprev, void* tbuf,
                      double* partial, hipStream_t s);

// --------------------------------------------------------------------------- diagonal
// E_b = sum_{p<q} Ub[p][q] b_p b_q for all b < 2^n; Ub is 32x32 FP64, bit-indexed, on device.
hipError_t diag_build(int prec, int n, const double* d_ub, void* diag, hipStream_t s);

// --------------------------------------------------------------------------- vectors
int64_t vec_num_partials(int prec, int n);
// u = w - alpha * sv * v (alpha read from d_alpha[0]); partial ||u||^2.
hipError_t lanczos_update(int prec, int n, const void* w, const void* v, double sv,
                          const double* d_alpha, void* u, double* partial, hipStream_t s);
// out = sum_l coef_l x_l; partial ||out||^2.
hipError_t krylov_combine(int prec, int n, const CombineCoef& c, void* out, double* partial,
                          hipStream_t s);
// partial ||x||^2.
hipError_t norm2_partial(int prec, int n, const void* x, double* partial, hipStream_t s);
// dst[0] = sum of partial[0..count) in a fixed order (one workgroup).
hipError_t finalize_sum(const double* partial, int64_t count, double* dst, hipStream_t s);
// Precision conversion for state import/export: complex128 <-> storage precision.
hipError_t convert_from_c128(int prec, int n, const void* src_c128, void* dst, hipStream_t s);
hipError_t convert_to_c128(int prec, int n, const void* src, void* dst_c128, hipStream_t s);

// --------------------------------------------------------------------------- observables
int64_t occ_num_partials(int n);
// <n_i> numerators and the total, FP64: out[0] = sum |x|^2, out[1 + p] = sum |x_b|^2 b_p.
hipError_t occupations(int prec, int n, const void* x, double* partial, double* out,
                       hipStream_t s);
int64_t sample_scratch_doubles(int n);
// idx[s] for s < shots; scratch holds sample_scratch_doubles(n) doubles.
hipError_t sample(int prec, int n, const void* x, uint64_t seed, int shots, double* scratch,
                  uint64_t* idx, hipStream_t s);

// --------------------------------------------------------------------------- host FP64
// Eigendecomposition of the symmetric tridiagonal T (alpha: m diagonal, beta: m-1
// off-diagonal) and y = exp(-i tau T) e_1.  Returns 0 on success.
int tridiag_expm(int m, const double* alpha, const double* beta, double tau, double* y_re,
                 double* y_im, double* work);
size_t tridiag_work_doubles(int m);

}  // namespace rsv
