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
// mode kCoefUniform / kCoefReal: every bit shares index 0 (a global drive; kCoefReal when
// phi = 0 so that up = dn is real); kCoefSite: per-bit coefficients.
enum CoefMode : int { kCoefUniform = 0, kCoefReal = 1, kCoefSite = 2 };
struct StepCoef {
  int n;
  int mode;
  double up_re[kMaxAtoms], up_im[kMaxAtoms];
  double dn_re[kMaxAtoms], dn_im[kMaxAtoms];
  double delta[kMaxAtoms];
};

// Krylov combination: out = sum_l (re_l + i im_l) * x_l, x_l device vectors (up to the whole
// basis plus one more vector, for re-orthogonalisation).
constexpr int kMaxCombine = kMaxKrylov + 1;
struct CombineCoef {
  int m;
  double re[kMaxCombine], im[kMaxCombine];
  const void* x[kMaxCombine];
};

// Inner products <x_g, y> = sum_b conj(x_g[b]) y[b] of up to kDotGroup vectors with one y.
constexpr int kDotGroup = 8;
struct DotGroup {
  int g;
  const void* x[kDotGroup];
};

// --------------------------------------------------------------------------- H|psi>
// Tile geometry of the H|psi> passes for a precision: the low pass's tiles cover bits
// [0, lo_bits) and it also flips the lo_ext bits [lo_ext_bit, lo_ext_bit + lo_ext) (the top
// bits), reading those neighbours from other tiles in global memory; high pass i covers
// bits [tile_a, tile_a + hi_bits - run_bits) plus run_bits contiguous low bits and flips
// [flip_lo, flip_hi).
constexpr int kMaxLoExt = 7;
struct TilePlan {
  int n, lo_bits, hi_bits;
  int n_hi_passes;
  int flip_lo[kMaxAtoms], flip_hi[kMaxAtoms], tile_a[kMaxAtoms], run_bits[kMaxAtoms];
  int lo_ext, lo_ext_bit;
};
TilePlan make_tile_plan(int prec, int n);

// Input of one H sweep: u = a0 x0 + (a1 + dot_coef * dot[0]) x1 + a2 x2 (x1, x2, dot may
// be null).  With only x0 and a0 = 1 the sweep applies H to a stored vector.  When nrm1 is
// set the Lanczos coefficients come from device memory instead: with s1 = 1/sqrt(nrm1[0])
// and s2 = 1/sqrt(nrm2[0]) (0 without nrm2), a0 = s1, the x1 coefficient is
// -s1^3 dot[0] and a2 = -s2/s1 -- so a sweep can be queued before the host has read them.
struct SweepIn {
  const void* x0;
  const void* x1;
  const void* x2;
  double a0, a1, a2;
  const double* dot;
  double dot_coef;
  const double* nrm1 = nullptr;
  const double* nrm2 = nullptr;
};
// Optional outputs: u_out stores the formed u (required when the sweep forms u and has
// more than one pass); part_norm / part_dot receive per-workgroup FP64 partial sums of |u|^2
// and Re<u, H u>.
struct SweepOut {
  void* u_out;
  double* part_norm;
  double* part_dot;
};
enum SweepPart : int { kAllPasses = 0, kFirstPass = 1, kLaterPasses = 2 };

// out = H u over all passes of the tile plan (or only the first / only the later ones);
// dtab holds the interaction-diagonal tables (diag_tables_build); tbuf (one vector) holds
// the high-bit partial when n > lo_bits.
hipError_t hpsi_sweep(int prec, int n, const StepCoef& c, const double* dtab, const SweepIn& in,
                      void* out, void* tbuf, const SweepOut& so, int part, hipStream_t s);
int64_t sweep_num_partials(int prec, int n);   // the largest partial count of any pass
int64_t sweep_norm_partials(int prec, int n);  // partials of |u|^2 (first pass)
int64_t sweep_dot_partials(int prec, int n);   // partials of Re<u, H u> (low pass)
int sweep_passes(int prec, int n);

// --------------------------------------------------------------------------- diagonal
// E_b = sum_{p<q} Ub[p][q] b_p b_q for all b < 2^n; Ub is 32x32 FP64, bit-indexed, on device.
hipError_t diag_build(int prec, int n, const double* d_ub, void* diag, hipStream_t s);
// The low pass forms E_b from two FP64 tables instead of reading a stored diagonal
// (L = the plan's lo_bits, b = (t << L) | e):
//   elo[e]                   = sum over pairs of set bits inside [0, L)        (2^L values)
//   etile[t (L + 1)]         = sum over pairs of set bits of t << L, above L
//   etile[t (L + 1) + 1 + p] = sum over set bits q >= L of t << L of Ub[p][q]  (p < L)
// so E_b = elo[e] + etile[t (L+1)] + sum_{p < L, e_p = 1} etile[t (L+1) + 1 + p].
size_t diag_table_doubles(int prec, int n);
hipError_t diag_tables_build(int prec, int n, const double* d_ub, double* dtab, hipStream_t s);

// --------------------------------------------------------------------------- vectors
int64_t vec_num_partials(int prec, int n);
// out = sum_l coef_l x_l; partial ||out||^2.
hipError_t krylov_combine(int prec, int n, const CombineCoef& c, void* out, double* partial,
                          hipStream_t s);
// The same combination, also accumulating the occupation numerators of the new state in the
// same pass: occ_out[0] = sum |out|^2, occ_out[1 + p] = sum over amplitudes with bit p set
// (device, n + 1 doubles); occ_partial holds combine_occ_partial_doubles(n).
int64_t combine_occ_partial_doubles(int n);
hipError_t krylov_combine_occ(int prec, int n, const CombineCoef& c, void* out, double* partial,
                              double* occ_partial, double* occ_out, hipStream_t s);
// partial ||x||^2.
hipError_t norm2_partial(int prec, int n, const void* x, double* partial, hipStream_t s);
// dst[0] = sum of partial[0..count) in a fixed order (one workgroup).
hipError_t finalize_sum(const double* partial, int64_t count, double* dst, hipStream_t s);
// dst[r] = sum of partial[r * count .. (r + 1) * count) for r < rows, the same fixed order.
hipError_t finalize_rows(const double* partial, int64_t count, int rows, double* dst,
                         hipStream_t s);
// Partials of Re and Im <x_g, y>: partial[(2 g + c) * vec_num_partials + w], c = 0 re, 1 im.
hipError_t multi_dot(int prec, int n, const DotGroup& d, const void* y, double* partial,
                     hipStream_t s);
// Precision conversion for state import/export: complex128 <-> storage precision.
hipError_t convert_from_c128(int prec, int n, const void* src_c128, void* dst, hipStream_t s);
hipError_t convert_to_c128(int prec, int n, const void* src, void* dst_c128, hipStream_t s);

// --------------------------------------------------------------------------- observables
int64_t occ_num_partials(int n);
// <n_i> numerators and the total, FP64: out[0] = sum |x|^2, out[1 + p] = sum |x_b|^2 b_p.
hipError_t occupations(int prec, int n, const void* x, double* partial, double* out,
                       hipStream_t s);
// <n_p n_q> numerators by bit position: *out_dev (inside scratch) gets [0] = sum |x|^2 and
// [1 + p n + q] for p <= q; scratch holds corr_scratch_doubles(n) doubles.
int64_t corr_scratch_doubles(int n);
hipError_t correlations(int prec, int n, const void* x, double* scratch, double** out_dev,
                        hipStream_t s);
int64_t sample_scratch_doubles(int n);
// idx[s] for s < shots; scratch holds sample_scratch_doubles(n) doubles.
hipError_t sample(int prec, int n, const void* x, uint64_t seed, int shots, double* scratch,
                  uint64_t* idx, hipStream_t s);
// The allocation-free sampler's scratch: a file-scope device array of
// sample_scratch_doubles(kMaxAtoms) doubles followed by room for kStaticMaxShots indices.
// static_sample_scratch gives its address on `device` (which must be current), resolved once
// per device; 0 on success.
constexpr int kStaticMaxShots = 1 << 16;
int static_sample_scratch(int device, void** out);
size_t static_sample_idx_offset_bytes();

// --------------------------------------------------------------------------- host FP64
// Eigendecomposition of the symmetric tridiagonal T (alpha: m diagonal, beta: m-1
// off-diagonal) and y = exp(-i tau T) e_1.  Returns 0 on success.
int tridiag_expm(int m, const double* alpha, const double* beta, double tau, double* y_re,
                 double* y_im, double* work);
size_t tridiag_work_doubles(int m);
// |[exp(-i tau T) e_1]_{m-1}| only (rows 0 and m-1 of the eigenvectors): the convergence test.
int tridiag_expm_last(int m, const double* alpha, const double* beta, double tau,
                      double* last_abs, double* work);

}  // namespace rsv
