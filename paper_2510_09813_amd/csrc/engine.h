// Host engine of librsv: device memory sources, registers, evolution workspaces and the
// Lanczos time stepper, shared by the C ABI (capi.cpp) and the server (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "first_fit.h"
#include "rsv.h"
#include "rsv_internal.h"

namespace rsv {

// Records a thread-local error message and returns code.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
const char* last_error();

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return ::rsv::fail(RSV_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                         __FILE__, __LINE__);                                             \
  } while (0)

#define RSV_TRY(expr)            \
  do {                           \
    int r_ = (expr);             \
    if (r_ != RSV_OK) return r_; \
  } while (0)

// A source of device memory.
class Allocator {
 public:
  virtual ~Allocator() = default;
  virtual int alloc(size_t bytes, void** p) = 0;
  virtual void release(void* p, size_t bytes) = 0;
  virtual size_t in_use() const = 0;
};

// hipMalloc / hipFree under an optional byte budget.
class DeviceAllocator : public Allocator {
 public:
  explicit DeviceAllocator(size_t budget) : budget_(budget) {}
  int alloc(size_t bytes, void** p) override;
  void release(void* p, size_t bytes) override;
  size_t in_use() const override;

 private:
  size_t budget_, in_use_ = 0;
  mutable std::mutex mu_;
};

// First-fit sub-allocation of one device block (256-byte granules).  Nothing allocates or
// frees device memory while it serves, so sub-allocations never synchronise the device.
class ArenaAllocator : public Allocator {
 public:
  ArenaAllocator() = default;
  ~ArenaAllocator() override;
  int init(size_t bytes);
  int alloc(size_t bytes, void** p) override;  // RSV_ENOMEM when no gap is large enough
  void release(void* p, size_t bytes) override;
  size_t in_use() const override;
  size_t capacity() const { return ff_.size(); }

 private:
  char* base_ = nullptr;
  FirstFit ff_;
  mutable std::mutex mu_;
};

size_t vec_bytes(int n, int prec);
size_t partial_doubles(int n, int prec);
size_t workspace_bytes(int n, int kmax, int prec);
size_t register_bytes(int n, int prec);
int check_state_args(int n, int prec);
int check_pulses(const rsv_pulses* pl, int n);
int check_opts(const rsv_evolve_opts* o, const rsv_pulses* pl, int64_t* first, int64_t* count);
StepCoef step_coef(const rsv_pulses* pl, int n, int64_t k, int dt_ns);

struct Workspace {
  int kmax = 0;
  void* block = nullptr;  // (kmax + 3) vectors, partial sums, device scalars
  std::vector<void*> basis;
  void* z = nullptr;  // H u of the latest Krylov vector; also the combination target
  void* t = nullptr;  // high-bit partial of H u
  double* pnorm = nullptr;
  double* pdot = nullptr;
  double* dscal = nullptr;
  size_t bytes = 0;
};

// Shot-to-shot noise: standard normal variate c of the stream seeded with `seed`, and the
// perturbation of ensemble member s (factor of Omega, per-atom detuning offsets [n],
// displaced positions [n][3]).
double noise_gaussian(uint64_t seed, uint64_t c);
void noise_member(const rsv_noise& nz, uint64_t seed, int n, int64_t s, const double* xyz,
                  double* factor, double* offsets, double* xyz_out);

}  // namespace rsv

struct rsv_ctx {
  int device = 0;
  rsv::DeviceAllocator* dev = nullptr;
  void* static_scratch = nullptr;  // this device's copy of the allocation-free sampler's scratch
};

struct rsv_register {
  rsv_ctx* ctx = nullptr;
  rsv::Allocator* alloc = nullptr;  // where the diagonal and the workspace live
  int n = 0;
  int prec = 0;
  double c6 = 0;
  double* d_ub = nullptr;
  double* d_dtab = nullptr;  // interaction-diagonal tables of the H psi low pass
  void* d_hbuf = nullptr;  // high-bit partial of rsv_apply_hamiltonian
  double* d_efull = nullptr;  // the 2^N interaction energies (FP64) of the Lindblad path
  size_t bytes = 0;
  rsv::Workspace ws;
  double* h_scal = nullptr;  // pinned host scalars of the per-iteration exchange
  bool own_h_scal = false;
  hipEvent_t ev[rsv::kMaxKrylov + 1] = {};  // iteration k's scalars have reached h_scal
  bool have_ev = false;
};

struct rsv_result {
  rsv_ctx* ctx = nullptr;
  int n = 0;
  int prec = 0;
  void* d_psi = nullptr;
  size_t bytes = 0;
  rsv_stats stats{};
};

namespace rsv {

// U_ij = C / |r_i - r_j|^6 (eq. 3) by bit position p = n-1-i into ub[32 * 32];
// RSV_EINVAL for coincident atoms or non-finite input.
int build_interactions(int n, const double* xyz, double c6, double* ub);

// Builds U and the device diagonal tables on `stream`; memory from `alloc`; h_scal (>= 512 doubles
// of pinned memory) is borrowed when given, else allocated.
int register_create(rsv_ctx* ctx, Allocator* alloc, int n, const double* xyz, double c6,
                    int prec, hipStream_t stream, double* h_scal, rsv_register** out);
void register_destroy(rsv_register* reg, hipStream_t stream);
int workspace_acquire(rsv_register* reg, int kmax);

// Evolves d_psi (2^n amplitudes of the register's precision) in place on `stream`.
// With obs_out set, <n_i> of the state after every obs_every-th step are written to
// obs_out[(j / obs_every - 1) * n + i] (host), accumulated by the pass that forms the state.
int evolve(rsv_register* reg, const rsv_pulses* pl, const rsv_evolve_opts* o, void* d_psi,
           hipStream_t stream, rsv_stats* st, int obs_every = 0, double* obs_out = nullptr);

// d_psi <- exp(-i dir tau H_c) d_psi (dir = +1 forward, -1 backward in time) by the Lanczos
// exponential of one step (sub-steps without convergence), with the register's workspace.
int krylov_exp(rsv_register* reg, const StepCoef& c, double tau, double dir, double tol,
               int kmax, int max_depth, void* d_psi, hipStream_t s, rsv_stats* st);

// <n_i> and samples of a device state; d_scratch needs occupation_scratch_bytes /
// sample_scratch_bytes; h_tmp is pinned host memory of at least 64 doubles.
size_t occupation_scratch_bytes(int n);
size_t sample_scratch_bytes(int n, int shots);
int occupations_with(int n, int prec, const void* d_psi, void* d_scratch, double* h_tmp,
                     double* out, hipStream_t s);
int sample_with(int n, int prec, const void* d_psi, uint64_t seed, int shots, void* d_scratch,
                uint64_t* out, hipStream_t s);

}  // namespace rsv
