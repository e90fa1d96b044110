/* librsv -- Rydberg state-vector emulation on AMD Instinct MI355X (gfx950).
 *
 * Computes the emu-sv method of "Efficient Emulation of Neutral Atom Quantum Hardware"
 * (arXiv 2510.09813): time evolution psi(t_{k+1}) = exp(-i H_k dt) psi(t_k) (eq. 6) of the
 * Rydberg Hamiltonian (eq. 3, Sec. II.A)
 *
 *   H(t) = sum_i Omega_i/2 (cos phi_i sigma^x_i - sin phi_i sigma^y_i) - sum_i delta_i n_i
 *          + sum_{i>j} C / |r_i - r_j|^6 n_i n_j
 *
 * on a 2^N state vector.  The pulse is piecewise constant with midpoint sampling
 * (Sec. III): step k uses the mean of the 1 ns samples at floor(m) and ceil(m),
 * m = (k + 1/2) dt.  exp(-i H_k dt) psi is the Lanczos Krylov exponential of Sec. III.A,
 * grown until its a-posteriori error estimate is below the tolerance.  H psi is
 * matrix-free: the diagonal (interaction energies from tables built once per register,
 * detuning added from the bit pattern) plus one level swap per atom scaled by the drive
 * (Sec. III.A).
 *
 * Conventions
 *  - |1> is the Rydberg level, n = |1><1|; the default initial state is |0...0> (Sec. II.B).
 *  - Amplitude index b: atom i (0-based) is bit N-1-i, i.e. atom 0 is the most significant
 *    bit (row-major c_{i1...iN}, Sec. II.B).  Bitstring character i is atom i.
 *  - sigma^y = [[0,-i],[i,0]] in (|0>,|1>): <1|h_i|0> = Omega_i/2 e^{-i phi_i}.
 *  - Units: hbar = 1, positions in um, time in us (dt and samples on a 1 ns grid), Omega and
 *    delta in rad/us, phi in rad, C in rad us^-1 um^6.
 *  - State vectors are interleaved (re, im): complex128 (RSV_C128) or complex64 (RSV_C64).
 *    In RSV_C64 the state, the Krylov basis and H psi are complex64 while every inner
 *    product, norm and Lanczos coefficient is FP64 and the tridiagonal exponential is host
 *    FP64.
 *
 * Ownership and errors
 *  - Host input arrays are read during the call only (copied where kept).
 *  - Handles belong to the library until the matching *_destroy.
 *  - Device pointers passed to *_device calls and rsv_apply_hamiltonian stay owned by the
 *    caller, must hold 2^N amplitudes of the register's precision and must not overlap.
 *  - Every call returns RSV_OK or an error code; nothing throws across this boundary.
 *    rsv_last_error() returns a thread-local description of the last failure.
 *  - A context is used by one host thread at a time.  Work is issued on the given HIP stream
 *    (NULL = the default stream); calls return after the work finished unless stated.
 */
#ifndef RSV_H_
#define RSV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RSV_OK = 0,
  RSV_EINVAL = 1,      /* invalid argument: sizes, grid, non-finite values, coincident atoms */
  RSV_ENOMEM = 2,      /* the context's HBM budget or the device cannot hold the workspace */
  RSV_EDEVICE = 3,     /* a HIP runtime call failed */
  RSV_ENOTCONV = 4,    /* Krylov exponential not converged within kmax even after sub-steps */
  RSV_ENUMERIC = 5,    /* a Lanczos coefficient or norm became NaN or Inf */
  RSV_EBUSY = 6,       /* resource in use (server queue full) */
  RSV_ECANCELLED = 7   /* the job was cancelled */
};

typedef enum { RSV_C128 = 0, RSV_C64 = 1 } rsv_precision;

typedef struct rsv_ctx rsv_ctx;
typedef struct rsv_register rsv_register;
typedef struct rsv_result rsv_result;
typedef struct rsv_server rsv_server;

/* Pulses sampled on the 1 ns grid t_n = n ns, n = 0..n_samples-1 (Sec. III).
 * per_site = 0: each array has n_samples values shared by all atoms;
 * per_site = 1: arrays are [n_atoms][n_samples], row-major.  phi may be NULL (zero). */
typedef struct {
  int64_t n_samples;
  int per_site;
  const double* omega; /* rad/us */
  const double* delta; /* rad/us */
  const double* phi;   /* rad */
} rsv_pulses;

/* dt_ns:      step in ns (integer multiple of the sampling grid, Sec. III); the pulse must
 *             cover a whole number of steps: (n_samples - 1) % dt_ns == 0.
 * tol:        Krylov tolerance on the a-posteriori estimate beta_m |[exp(-i dt T_m) e_1]_m|
 *             times |psi| (the "precision" of Sec. III.A), > 0.
 * kmax:       maximum Krylov dimension, 2..64.  Without convergence the step is split into
 *             sub-steps with the same H_k (exact), at most max_substep_depth halvings deep.
 * first_step, n_steps: evolve steps [first_step, first_step + n_steps); n_steps < 0 means up
 *             to the end of the pulse.  Stepping is Markov, so (k, psi_k) is a checkpoint.
 * reorth:     0 = the three-term Lanczos recurrence (default); 1 = every new Krylov vector is
 *             also orthogonalised against all stored ones (classical Gram-Schmidt, FP64
 *             inner products), at the cost of reading the basis once more per iteration.
 *             The paper leaves orthogonalisation open; the loss of orthogonality found is
 *             reported in rsv_stats.ortho_loss. */
typedef struct {
  int dt_ns;
  double tol;
  int kmax;
  int max_substep_depth;
  int64_t first_step;
  int64_t n_steps;
  int reorth;
} rsv_evolve_opts;

typedef struct {
  int64_t steps;          /* time steps taken */
  int64_t krylov_iters;   /* Lanczos iterations (H psi applications), summed */
  int64_t krylov_max;     /* largest Krylov dimension used */
  int64_t substeps;       /* extra sub-steps taken after non-convergence */
  double norm_final;      /* |psi| after the last step (1 up to rounding) */
  double seconds;         /* wall time of the evolution, entry to final synchronisation */
  double bytes_hpsi;      /* algorithmic HBM bytes of the H psi passes */
  double ortho_loss;      /* reorth = 1: largest |<v_l, u>| / |u| removed from a new vector */
} rsv_stats;

/* ------------------------------------------------------------------ context */
const char* rsv_version(void);
const char* rsv_last_error(void);
/* hbm_budget_bytes = 0: no budget beyond the device's free memory. */
int rsv_ctx_create(int hip_device, size_t hbm_budget_bytes, rsv_ctx** out);
void rsv_ctx_destroy(rsv_ctx* ctx);
/* Bytes of device memory currently held by the context's registers and results. */
size_t rsv_ctx_bytes_in_use(const rsv_ctx* ctx);

/* ------------------------------------------------------------------ register
 * Builds U_ij = C/|r_i - r_j|^6 on the host (eq. 3) and, on the device, the tables from
 * which the H psi kernels form the interaction diagonal E_b = sum_{i>j} U_ij n_i n_j
 * (Sec. III.A keeps only the diagonal of H): the pair sums of the low bits and, per tile of
 * high bits, their pair sum and couplings -- about 2^12 + 13 * 2^(N-12) FP64 values instead
 * of 2^N.  n_atoms in 1..30; xyz_um is [n_atoms][3]; coincident atoms give RSV_EINVAL. */
int rsv_register_create(rsv_ctx* ctx, int n_atoms, const double* xyz_um, double c6,
                        rsv_precision prec, rsv_register** out);
void rsv_register_destroy(rsv_register* reg);
/* Writes E (2^N reals: FP64 for RSV_C128, FP32 for RSV_C64) into a caller device buffer;
 * returns after the stream has finished. */
int rsv_register_diagonal(rsv_register* reg, void* d_out, void* hip_stream);

/* Device bytes rsv_evolve needs for a register of n_atoms: (kmax + 3) vectors (Krylov basis
 * of kmax + 1, the Lanczos residual, the high-bit H psi partial) plus U and the diagonal
 * tables, the state and the reduction buffers -- the admission formula of the server. */
size_t rsv_workspace_bytes(int n_atoms, int kmax, rsv_precision prec);

/* ------------------------------------------------------------------ hot path
 * One H_k psi: d_out = H_k d_in with the parameters of step `step` for the given dt
 * (Sec. III.A).  d_in, d_out: caller device buffers of 2^N amplitudes.  The kernels are
 * enqueued on hip_stream and the call returns without waiting for them. */
int rsv_apply_hamiltonian(rsv_register* reg, const rsv_pulses* pulses, int64_t step, int dt_ns,
                          const void* d_in, void* d_out, void* hip_stream);

/* Evolves the caller's device state in place through the requested steps (eq. 6). */
int rsv_evolve_device(rsv_register* reg, const rsv_pulses* pulses, const rsv_evolve_opts* opts,
                      void* d_psi_inout, void* hip_stream, rsv_stats* stats_out);

/* rsv_evolve_device that also records <n_i> along the way (observables at intermediate
 * times, Sec. IV): after every `every`-th step j (j = every, 2 every, ... <= the steps
 * taken) the occupations of the new state go to occ_out[(j / every - 1) * n_atoms + i],
 * accumulated (FP64) by the same pass that forms the state from the Krylov basis, so they
 * cost no extra read of it.  occ_out: host, floor(steps / every) * n_atoms doubles. */
int rsv_evolve_device_observed(rsv_register* reg, const rsv_pulses* pulses,
                               const rsv_evolve_opts* opts, void* d_psi_inout, void* hip_stream,
                               int every, double* occ_out, rsv_stats* stats_out);

/* Host-level form: psi0_host is 2^N complex128 values (NULL = |0...0>); the result keeps
 * the evolved state on the device until rsv_result_destroy. */
int rsv_evolve(rsv_register* reg, const rsv_pulses* pulses, const rsv_evolve_opts* opts,
               const void* psi0_host, rsv_result** out);
int rsv_result_state(const rsv_result* res, void* psi_host_c128);
/* <n_i> for i = 0..N-1 (FP64 accumulation, normalised by |psi|^2). */
int rsv_result_occupations(const rsv_result* res, double* n_out);
/* n_shots basis indices drawn from |psi_b|^2 / |psi|^2 in shot order.  Shot s uses the s-th
 * output x_s of SplitMix64 seeded with `seed`, u_s = (x_s >> 11) 2^-53, and returns the
 * smallest b with CDF(b) > u_s CDF(2^N - 1) (the largest b of nonzero mass if rounding
 * leaves none). */
int rsv_result_sample(const rsv_result* res, uint64_t seed, int n_shots, uint64_t* idx_out);
int rsv_result_stats(const rsv_result* res, rsv_stats* out);
void rsv_result_destroy(rsv_result* res);

/* <H_k> = <psi|H_k|psi> / <psi|psi> for the Hamiltonian of step `step` (eq. 3 with the
 * midpoint parameters of Sec. III), from one H psi (the kernels of rsv_apply_hamiltonian)
 * with FP64 inner products.  d_psi: 2^N amplitudes of the register's precision. */
int rsv_energy_device(rsv_register* reg, const rsv_pulses* pulses, int64_t step, int dt_ns,
                      const void* d_psi, double* energy_out, void* hip_stream);

/* The same outputs for a caller device state of n_atoms in precision prec. */
int rsv_occupations_device(rsv_ctx* ctx, int n_atoms, rsv_precision prec, const void* d_psi,
                           double* n_out, void* hip_stream);
int rsv_sample_device(rsv_ctx* ctx, int n_atoms, rsv_precision prec, const void* d_psi,
                      uint64_t seed, int n_shots, uint64_t* idx_out, void* hip_stream);
/* Correlators <n_i n_j> = sum_b |psi_b|^2 n_i(b) n_j(b) / |psi|^2 (Sec. IV's expectation
 * values), FP64: out[i * n_atoms + j], symmetric, diagonal <n_i>. */
int rsv_correlations_device(rsv_ctx* ctx, int n_atoms, rsv_precision prec, const void* d_psi,
                            double* out, void* hip_stream);

/* Allocation-free form of rsv_sample_device, for callers that cannot allocate device or
 * pinned memory (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, outputs and errors; the block sums, their scan and the drawn
 * indices live in a device array inside the library (4.7 MB on every device it runs on,
 * kept until the process ends) instead of memory taken from the context.  n_shots at most
 * 65536 (RSV_EINVAL beyond).  Every call on a device shares that device's array: calls that
 * overlap in time on one device (other host threads, other streams) race and must be
 * serialised by the caller.  idx_out is host memory; returns after the stream finished. */
int rsv_sample_device_static(rsv_ctx* ctx, int n_atoms, rsv_precision prec, const void* d_psi,
                             uint64_t seed, int n_shots, uint64_t* idx_out, void* hip_stream);

/* ------------------------------------------------------------------ open systems
 * The Lindblad master equation (Sec. III.A: open-system dynamics by the full master
 * equation, evolved with a Krylov method) on the vectorised density matrix:
 *   d rho/dt = -i [H_k, rho] + sum_i (L_i rho L_i^+ - {L_i^+ L_i, rho}/2)
 * with, per atom, relaxation of the Rydberg level L_i = sqrt(relax_rate) |0><1|_i and
 * dephasing L_i = sqrt(2 dephasing_rate) n_i (an atom's coherences then decay at
 * dephasing_rate; equivalently sqrt(dephasing_rate/2) sigma^z_i).  Rates in 1/us.
 * rho is 2^N x 2^N, stored row-major as 4^N amplitudes of the register's precision,
 * element (r, c) at index (r << N) | c with the state-vector bit order; N <= 14. */
typedef struct {
  double relax_rate;
  double dephasing_rate;
} rsv_lindblad;

/* d_out = L_k d_in for step `step` (test and benchmark hook).  The kernel is enqueued on
 * hip_stream and the call returns without waiting (the register's interaction energies are
 * built on its first Lindblad call and kept). */
int rsv_lindblad_apply(rsv_register* reg, const rsv_pulses* pulses, int64_t step, int dt_ns,
                       const rsv_lindblad* rates, const void* d_in, void* d_out, void* hip_stream);
/* rho <- exp(dt L_{k}) rho for the requested steps (opts as for rsv_evolve_device; reorth is
 * ignored, kmax <= 63), each exponential by the Arnoldi process (classical Gram-Schmidt with
 * a second pass when the first removes most of the new vector, FP64 inner products, host
 * FP64 exponential of the Hessenberg matrix) to the
 * estimate |rho| h_{m+1,m} |[exp(dt H_m) e_1]_m| <= tol, halving the step without
 * convergence.  stats->norm_final is the Frobenius norm of the final rho. */
int rsv_lindblad_evolve_device(rsv_register* reg, const rsv_pulses* pulses,
                               const rsv_evolve_opts* opts, const rsv_lindblad* rates,
                               void* d_rho_inout, void* hip_stream, rsv_stats* stats_out);
/* <n_i> = sum_r rho_rr n_i(r) / Tr rho and Tr rho (trace_out may be NULL). */
int rsv_lindblad_occupations(rsv_ctx* ctx, int n_atoms, rsv_precision prec, const void* d_rho,
                             double* occ_out, double* trace_out, void* hip_stream);

/* ------------------------------------------------------------------ gradients
 * Derivatives of an output with respect to the pulse (Sec. IV: the emulator is
 * differentiable): C = <psi_K| sum_i w_i n_i |psi_K> after the requested steps of eq. (6)
 * from psi0_host (2^N complex128 values, NULL = |0...0>), and dC/dOmega_j, dC/ddelta_j for
 * every sample j of GLOBAL pulses (per_site = 0; phi, if given, is held fixed).  Adjoint
 * method: the forward sweep to psi_K, then backwards step by step psi_k and the adjoint
 * lambda_k by the Lanczos exponential run backwards in time, and the derivative of each
 * step's exponential from the Arnoldi exponential of the block operator
 * -i [[H_k, dH/dtheta], [0, H_k]] applied to (0, psi_k); the midpoint rule of Sec. III
 * hands half of a step's derivative to each of its two samples.  grad_omega and grad_delta
 * have n_samples entries (zero for samples no step uses); kmax <= 63.  Cost: about
 * (1 + 2 + 2 x 6) times the Krylov work of the forward evolution. */
int rsv_gradient_occupations(rsv_register* reg, const rsv_pulses* pulses,
                             const rsv_evolve_opts* opts, const double* weights,
                             const void* psi0_host, double* value, double* grad_omega,
                             double* grad_delta, rsv_stats* stats_out);

/* ------------------------------------------------------------------ serving
 * A server evolves a stream of independent jobs (each a register, its pulses and options)
 * on one device with continuous batching: n_lanes jobs run at once, each on its own HIP
 * stream, so their kernels overlap on the device; a queued job is admitted as soon as a
 * lane is free and its device footprint (rsv_server_job_bytes: the Krylov workspace of
 * kmax + 3 vectors, the diagonal, the state and output scratch) fits in the server's
 * arena, first fit in arrival order.  The arena is allocated once at creation, so serving
 * never allocates or frees device memory.  A job's result does not depend on what else
 * runs: every reduction has a fixed order.
 *
 * Small jobs (n_atoms <= pack_max_atoms, at most 12 for RSV_C128 and 13 for RSV_C64) are
 * packed: a free lane takes the queued small jobs of the first one's precision (up to
 * pack_max_jobs) and runs them in ONE launch, one workgroup per job, each workgroup carrying
 * its job's whole evolution with the state on chip.  The method is that of Sec. III.A with
 * the small exponential evaluated on the device (a Chebyshev expansion), so a packed result
 * agrees with the plain path to the tolerance, not bit for bit; it is still independent of
 * the batch it ran in.  With packing on, the server runs one lane more than n_lanes that
 * takes only packed batches, so small jobs do not wait for lanes held by long jobs. */
typedef struct {
  int n_lanes;        /* concurrent jobs, 1..16 */
  size_t arena_bytes; /* device memory reserved for jobs; 0 = three quarters of free memory */
  int max_queue;      /* queued jobs beyond this make rsv_server_submit return RSV_EBUSY; 0 = no limit */
  int pack_max_atoms; /* 0 = never pack; else jobs with n_atoms <= this (<= 13) run packed */
  int pack_max_jobs;  /* jobs per packed launch, 0 = 256 */
} rsv_server_opts;

typedef struct {
  int n_atoms;
  const double* xyz_um; /* [n_atoms][3] */
  double c6;
  rsv_precision prec;
  rsv_pulses pulses;
  rsv_evolve_opts opts;
  const void* psi0_host; /* 2^N complex128 values, NULL = |0...0> */
  int n_shots;           /* bitstring samples to draw from the final state (seeded by seed) */
  uint64_t seed;
  int return_state;      /* 1: the completion carries the final state as complex128 */
  uint64_t tag;          /* caller's label, returned unchanged */
  int verify_fp64;       /* RSV_C64 jobs: 1 = also evolve the job in complex128 (tol at most
                            1e-10) and report the complex64 result's infidelity and largest
                            occupation error against it; the job then runs on the plain path
                            and occupies both workspaces */
} rsv_job_desc;

typedef struct {
  uint64_t job_id, tag;
  int status; /* RSV_OK, or the error the job ended with (RSV_ECANCELLED when cancelled) */
  int n_atoms, n_shots;
  double t_submit, t_start, t_end; /* seconds since rsv_server_create */
  rsv_stats stats;
  double* occupations; /* [n_atoms]; these arrays stay valid until rsv_server_release */
  uint64_t* samples;   /* [n_shots] or NULL */
  void* state;         /* [2^N] complex128 or NULL */
  char error[160];
  /* verify_fp64 jobs: 1 - |<psi_128|psi>|^2 / (|psi_128|^2 |psi|^2) (FP64, so resolved to
   * about 1e-16) and max_i |<n_i> - <n_i>_128| against the complex128 evolution of the same
   * job; -1 otherwise */
  double infidelity_fp64;
  double max_occ_err_fp64;
} rsv_completion;

/* Shot-to-shot parameter noise (Sec. III.A: open-system effects by varying the Hamiltonian's
 * parameters from shot to shot).  Ensemble member s perturbs a job by standard normal
 * variates g: the drive amplitude by one factor for all atoms, Omega_i(t) -> (1 +
 * omega_rel_sigma g_0) Omega_i(t); each atom's detuning by a constant offset, delta_i(t) ->
 * delta_i(t) + delta_sigma g_{1+i} (rad/us); each atom's position on each axis, r_{i,a} ->
 * r_{i,a} + position_sigma_um g_{1+N+3i+a}.  Variate c = s (4N + 1) + j is the Box-Muller
 * transform sqrt(-2 ln u1) cos(2 pi u2) of u1 = ((x_{2c} >> 11) + 1) 2^-53 and
 * u2 = (x_{2c+1} >> 11) 2^-53, x_k the k-th output of SplitMix64 seeded with noise_seed. */
typedef struct {
  double omega_rel_sigma;   /* relative standard deviation of the drive amplitude */
  double delta_sigma;       /* standard deviation of each atom's detuning offset, rad/us */
  double position_sigma_um; /* standard deviation of each position coordinate, um */
} rsv_noise;

/* The perturbation of member s of an ensemble of n_atoms (host only): *omega_factor,
 * delta_offset[n_atoms] (rad/us) and xyz_out[n_atoms][3] = xyz_um displaced (um). */
int rsv_noise_member(const rsv_noise* noise, uint64_t noise_seed, int n_atoms, int64_t member,
                     const double* xyz_um, double* omega_factor, double* delta_offset,
                     double* xyz_out);

int rsv_server_create(rsv_ctx* ctx, const rsv_server_opts* opts, rsv_server** out);
/* Device bytes one job occupies in the arena. */
size_t rsv_server_job_bytes(int n_atoms, int kmax, rsv_precision prec, int n_shots);
/* Copies the job (all arrays) and queues it.  RSV_ENOMEM if it can never fit the arena,
 * RSV_EBUSY if the queue is full, RSV_EINVAL for invalid input. */
int rsv_server_submit(rsv_server* srv, const rsv_job_desc* job, uint64_t* job_id);
/* Waits up to timeout_ms (< 0: forever) for at least one completion and moves up to max of
 * them to out[0..*n_out). */
int rsv_server_poll(rsv_server* srv, rsv_completion* out, int max, int* n_out, int timeout_ms);
/* Queues n_members jobs, member s being `job` perturbed as rsv_noise_member(noise,
 * noise_seed, n_atoms, s) describes (with delta_sigma > 0 the member's pulses become
 * per-site).  Member s samples with seed job->seed + s and carries tag job->tag + s; its id
 * goes to job_ids[s].  The members are queued together, in member order, so that small
 * ones share packed launches; each is an ordinary job (alone == in the mix).  All or none
 * are queued: RSV_EBUSY if the queue cannot take them all. */
int rsv_server_submit_ensemble(rsv_server* srv, const rsv_job_desc* job, const rsv_noise* noise,
                               uint64_t noise_seed, int n_members, uint64_t* job_ids);
/* Frees the arrays of a polled completion. */
void rsv_server_release(rsv_server* srv, rsv_completion* c);
/* Cancels a queued job (it completes with RSV_ECANCELLED); RSV_EBUSY if it already runs,
 * RSV_EINVAL if unknown or finished. */
int rsv_server_cancel(rsv_server* srv, uint64_t job_id);
/* Jobs queued, running and completed-but-not-polled; arena bytes in use. */
int rsv_server_status(rsv_server* srv, int* queued, int* running, int* done, size_t* arena_used);
/* Cancels queued jobs, waits for the running ones and frees everything; completions not
 * polled are discarded. */
void rsv_server_destroy(rsv_server* srv);

/* Host FP64 tridiagonal exponential used by every Lanczos step (Sec. III.A):
 * y = exp(-i tau T) e_1 for T = tridiag(beta, alpha, beta), m in 1..64.  Host only. */
int rsv_tridiag_expm(int m, const double* alpha, const double* beta, double tau, double* y_re,
                     double* y_im);

#ifdef __cplusplus
}
#endif

#endif /* RSV_H_ */
