// Continuous-batching server: a stream of independent emulation jobs on one device.
//
// n_lanes worker threads each own a HIP stream and pinned host scalars.  A lane takes the
// first queued job (arrival order) whose device footprint fits in the arena, runs the
// whole job (diagonal, evolution, occupations, samples, optional state) on its stream and
// releases the footprint; kernels of concurrent jobs overlap on the device, and the host
// round trip of one job's Lanczos iteration is hidden behind the others' kernels.  Each
// job's memory is one arena block split by a bump allocator, so admission is exactly
// "the footprint fits" and nothing is allocated or freed on the device while serving.
//
// Small jobs are packed: a lane takes every queued small job of one precision (up to the
// batch limit and its pinned staging size) as one arena block, uploads all their inputs
// with one copy, builds each diagonal, runs them in one launch of the packed kernel (one
// workgroup per job) and downloads all outputs with one copy.  With packing on, one lane
// beyond n_lanes takes only packed batches, so small jobs never queue behind long jobs that
// hold every regular lane.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "engine.h"
#include "packed.h"

using namespace rsv;

namespace {

constexpr size_t kGranule = 256;
inline size_t granule(size_t b) { return (b + kGranule - 1) / kGranule * kGranule; }

// Sequential sub-allocation of one job's arena block; release is a no-op.
class BumpAllocator : public Allocator {
 public:
  BumpAllocator(void* base, size_t size) : base_((char*)base), size_(size) {}
  int alloc(size_t bytes, void** p) override {
    bytes = granule(bytes);
    if (used_ + bytes > size_) {
      *p = nullptr;
      return fail(RSV_ENOMEM, "job block exhausted (%zu + %zu > %zu)", used_, bytes, size_);
    }
    *p = base_ + used_;
    used_ += bytes;
    return RSV_OK;
  }
  void release(void*, size_t) override {}
  size_t in_use() const override { return used_; }

 private:
  char* base_;
  size_t size_, used_ = 0;
};

size_t job_bytes(int n, int kmax, int prec, int shots) {
  return granule(register_bytes(n, prec)) + granule(workspace_bytes(n, kmax, prec)) +
         granule(vec_bytes(n, prec)) + granule(occupation_scratch_bytes(n)) +
         granule(sample_scratch_bytes(n, shots > 0 ? shots : 0)) + 4 * kGranule;
}

constexpr size_t kPackStage = size_t(32) << 20;  // pinned staging per lane, each direction
constexpr int kPackDefaultJobs = 256;
constexpr int kPackOutDoubles = 64;

struct Job {
  uint64_t id = 0, tag = 0;
  int n = 0, prec = 0, shots = 0, return_state = 0, verify = 0;
  int64_t first_step = 0, n_steps = 0;
  bool packed = false, taken = false;
  size_t up = 0, down = 0, work = 0;  // packed footprint: uploaded, downloaded, device-only
  double c6 = 0;
  uint64_t seed = 0;
  std::vector<double> xyz, omega, delta, phi;
  std::vector<double> psi0;  // interleaved complex128, empty = |0...0>
  rsv_pulses pulses{};
  rsv_evolve_opts opts{};
  size_t bytes = 0;
  double t_submit = 0;
  void* block = nullptr;  // arena block while admitted
};

}  // namespace

struct rsv_server {
  rsv_ctx* ctx = nullptr;
  rsv_server_opts opts{};
  ArenaAllocator arena;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job*> queue;
  std::deque<rsv_completion> done;
  std::vector<std::thread> lanes;
  int running = 0;
  bool stop = false;
  uint64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
};

namespace {

void fill_error(rsv_completion& c, int status) {
  c.status = status;
  if (status != RSV_OK) {
    std::strncpy(c.error, last_error(), sizeof c.error - 1);
    c.error[sizeof c.error - 1] = 0;
  }
}

// The precision report of a complex64 job: the same job evolved in complex128 (tolerance at
// most 1e-10) in the rest of the job's block, then 1 - |<a|b>|^2 / (|a|^2 |b|^2) and the
// largest occupation difference, all sums FP64 on the device.
int verify_fp64(rsv_server* srv, Job* job, const void* d_psi64,
                BumpAllocator& bump, hipStream_t stream, double* h_pinned, rsv_completion& c) {
  const int n = job->n;
  rsv_register* reg = nullptr;
  RSV_TRY(register_create(srv->ctx, &bump, n, job->xyz.data(), job->c6, kC128, stream, h_pinned,
                          &reg));
  struct Guard {
    rsv_register* r;
    hipStream_t s;
    ~Guard() { register_destroy(r, s); }
  } guard{reg, stream};
  RSV_TRY(workspace_acquire(reg, job->opts.kmax));
  void *d_psi = nullptr, *occ_scratch = nullptr;
  RSV_TRY(bump.alloc(vec_bytes(n, kC128), &d_psi));
  RSV_TRY(bump.alloc(occupation_scratch_bytes(n), &occ_scratch));
  const size_t b128 = (size_t(1) << n) * 16;
  if (!job->psi0.empty()) {
    HIP_TRY(hipMemcpyAsync(d_psi, job->psi0.data(), b128, hipMemcpyHostToDevice, stream));
  } else {
    HIP_TRY(hipMemsetAsync(d_psi, 0, b128, stream));
    h_pinned[0] = 1.0;
    h_pinned[1] = 0.0;
    HIP_TRY(hipMemcpyAsync(d_psi, h_pinned, 16, hipMemcpyHostToDevice, stream));
    HIP_TRY(hipStreamSynchronize(stream));
  }
  rsv_evolve_opts o = job->opts;
  o.tol = std::min(o.tol, 1e-10);
  rsv_stats st{};
  RSV_TRY(evolve(reg, &job->pulses, &o, d_psi, stream, &st));
  std::vector<double> occ(n);
  RSV_TRY(occupations_with(n, kC128, d_psi, occ_scratch, h_pinned, occ.data(), stream));
  double err = 0.0;
  for (int i = 0; i < n; ++i) err = std::max(err, std::abs(occ[i] - c.occupations[i]));
  // the complex64 state widened into the complex128 register's workspace vector z, then
  // <a, b>, |a|^2, |b|^2 with the two-stage FP64 sums
  void* wide = reg->ws.z;
  HIP_TRY(convert_to_c128(kC64, n, d_psi64, wide, stream));
  double* part = reg->ws.pnorm;
  double* res = reg->ws.dscal;
  const int64_t nw = vec_num_partials(kC128, n);
  DotGroup d{};
  d.g = 1;
  d.x[0] = d_psi;
  HIP_TRY(multi_dot(kC128, n, d, wide, part, stream));
  HIP_TRY(finalize_rows(part, nw, 2, res, stream));
  HIP_TRY(norm2_partial(kC128, n, d_psi, part, stream));
  HIP_TRY(finalize_sum(part, nw, res + 2, stream));
  HIP_TRY(norm2_partial(kC128, n, wide, part, stream));
  HIP_TRY(finalize_sum(part, nw, res + 3, stream));
  HIP_TRY(hipMemcpyAsync(h_pinned, res, 4 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  const double ab2 = h_pinned[0] * h_pinned[0] + h_pinned[1] * h_pinned[1];
  c.infidelity_fp64 = std::max(0.0, 1.0 - ab2 / (h_pinned[2] * h_pinned[3]));
  c.max_occ_err_fp64 = err;
  return RSV_OK;
}

// Runs one admitted job on `stream`; the job's memory is job->block.
int run_job(rsv_server* srv, Job* job, hipStream_t stream, double* h_pinned, rsv_completion& c) {
  BumpAllocator bump(job->block, job->bytes);
  const int n = job->n, prec = job->prec;
  rsv_register* reg = nullptr;
  RSV_TRY(register_create(srv->ctx, &bump, n, job->xyz.data(), job->c6, prec, stream, h_pinned,
                          &reg));
  struct Guard {
    rsv_register* r;
    hipStream_t s;
    ~Guard() { register_destroy(r, s); }
  } guard{reg, stream};
  RSV_TRY(workspace_acquire(reg, job->opts.kmax));
  void *d_psi = nullptr, *occ_scratch = nullptr, *smp_scratch = nullptr;
  RSV_TRY(bump.alloc(vec_bytes(n, prec), &d_psi));
  RSV_TRY(bump.alloc(occupation_scratch_bytes(n), &occ_scratch));
  RSV_TRY(bump.alloc(sample_scratch_bytes(n, job->shots), &smp_scratch));
  // z and t of the workspace are adjacent: 2^N complex128 of staging for conversions
  void* staging = reg->ws.z;
  const size_t b128 = (size_t(1) << n) * 16;
  if (!job->psi0.empty()) {
    void* dst = prec == kC128 ? d_psi : staging;
    HIP_TRY(hipMemcpyAsync(dst, job->psi0.data(), b128, hipMemcpyHostToDevice, stream));
    if (prec != kC128) HIP_TRY(convert_from_c128(prec, n, staging, d_psi, stream));
  } else {
    HIP_TRY(hipMemsetAsync(d_psi, 0, vec_bytes(n, prec), stream));
    if (prec == kC128) {
      h_pinned[0] = 1.0;
      h_pinned[1] = 0.0;
      HIP_TRY(hipMemcpyAsync(d_psi, h_pinned, 16, hipMemcpyHostToDevice, stream));
    } else {
      float* f = (float*)h_pinned;
      f[0] = 1.0f;
      f[1] = 0.0f;
      HIP_TRY(hipMemcpyAsync(d_psi, f, 8, hipMemcpyHostToDevice, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));  // the pinned scalars are reused below
  }
  RSV_TRY(evolve(reg, &job->pulses, &job->opts, d_psi, stream, &c.stats));
  c.occupations = new double[n];
  RSV_TRY(occupations_with(n, prec, d_psi, occ_scratch, h_pinned, c.occupations, stream));
  if (job->shots > 0) {
    c.samples = new uint64_t[job->shots];
    c.n_shots = job->shots;
    RSV_TRY(sample_with(n, prec, d_psi, job->seed, job->shots, smp_scratch, c.samples, stream));
  }
  if (job->return_state) {
    c.state = new double[(size_t(1) << n) * 2];
    const void* src = d_psi;
    if (prec != kC128) {
      HIP_TRY(convert_to_c128(prec, n, d_psi, staging, stream));
      src = staging;
    }
    HIP_TRY(hipMemcpyAsync(c.state, src, b128, hipMemcpyDeviceToHost, stream));
  }
  HIP_TRY(hipStreamSynchronize(stream));
  if (job->verify) RSV_TRY(verify_fp64(srv, job, d_psi, bump, stream, h_pinned, c));
  return RSV_OK;
}

void free_completion(rsv_completion& c) {
  delete[] c.occupations;
  delete[] c.samples;
  delete[] (double*)c.state;
  c.occupations = nullptr;
  c.samples = nullptr;
  c.state = nullptr;
}

// ---------------------------------------------------------------------- packed batches

size_t pulse_count(const Job& j) {
  return (size_t)j.pulses.n_samples * (j.pulses.per_site ? (size_t)j.n : 1);
}

// Footprint of a packed job: uploaded (U, pulses, initial state), downloaded (status and
// occupations, samples, final state) and device-only (diagonal, state, Krylov basis,
// sampling scratch).
void packed_sizes(Job& j) {
  const size_t dim = size_t(1) << j.n, cnt = pulse_count(j);
  j.up = granule(32 * 32 * 8) + 2 * granule(cnt * 8) + (j.phi.empty() ? 0 : granule(cnt * 8)) +
         (j.psi0.empty() ? 0 : granule(dim * 16));
  j.down = granule(kPackOutDoubles * 8) + granule((size_t)j.shots * 8) +
           (j.return_state ? granule(dim * 16) : 0);
  j.work = granule(dim * (j.prec == kC128 ? 8 : 4)) + granule(vec_bytes(j.n, j.prec)) +
           granule((size_t)j.opts.kmax * vec_bytes(j.n, j.prec)) +
           (j.shots > 0 ? granule((size_t)sample_scratch_doubles(j.n) * 8) : 0);
}

size_t batch_bytes(size_t count, size_t up, size_t down, size_t work) {
  return granule(count * sizeof(PackedJob)) + up + down + work;
}

struct Work {
  std::vector<Job*> jobs;  // one plain job, or a packed batch
  bool packed = false;
  void* block = nullptr;
  size_t bytes = 0;
};

// Packed batch starting at queue position `first`: that job and the later packed jobs of
// its precision, in arrival order, within the batch limit and the staging size; shrunk
// from the end until its block fits the arena.
bool take_batch(rsv_server* srv, size_t first, Work& w) {
  const Job* lead = srv->queue[first];
  const size_t max_jobs = srv->opts.pack_max_jobs > 0 ? srv->opts.pack_max_jobs : kPackDefaultJobs;
  std::vector<Job*> cand;
  std::vector<size_t> up{0}, down{0}, work{0};  // prefix sums
  for (size_t q = first; q < srv->queue.size() && cand.size() < max_jobs; ++q) {
    Job* j = srv->queue[q];
    if (!j->packed || j->prec != lead->prec) continue;
    const size_t u = up.back() + j->up, d = down.back() + j->down;
    if (granule((cand.size() + 1) * sizeof(PackedJob)) + u > kPackStage || d > kPackStage) break;
    cand.push_back(j);
    up.push_back(u);
    down.push_back(d);
    work.push_back(work.back() + j->work);
  }
  for (size_t k = cand.size(); k >= 1; k = k / 2) {
    const size_t bytes = batch_bytes(k, up[k], down[k], work[k]);
    void* block = nullptr;
    if (srv->arena.alloc(bytes, &block) == RSV_OK) {
      w.jobs.assign(cand.begin(), cand.begin() + k);
      w.packed = true;
      w.block = block;
      w.bytes = bytes;
      return true;
    }
  }
  return false;
}

// First queued work (arrival order) whose memory fits: a plain job, or a packed batch led
// by the first packed job that fits (packed_only: the small-job lane takes only those).
bool take_work(rsv_server* srv, std::unique_lock<std::mutex>& lk, Work& w, bool packed_only) {
  for (;;) {
    if (srv->stop) return false;
    for (size_t q = 0; q < srv->queue.size(); ++q) {
      Job* j = srv->queue[q];
      bool got = false;
      if (packed_only && !j->packed) continue;
      if (j->packed) {
        got = take_batch(srv, q, w);
      } else {
        void* block = nullptr;
        if (srv->arena.alloc(j->bytes, &block) == RSV_OK) {
          j->block = block;
          w.jobs.assign(1, j);
          w.packed = false;
          w.block = block;
          w.bytes = j->bytes;
          got = true;
        }
      }
      if (got) {
        for (Job* t : w.jobs) t->taken = true;
        srv->queue.erase(std::remove_if(srv->queue.begin(), srv->queue.end(),
                                        [](Job* x) { return x->taken; }),
                         srv->queue.end());
        srv->running += (int)w.jobs.size();
        return true;
      }
    }
    srv->cv_work.wait(lk);
  }
}

struct LaneBuffers {
  hipStream_t stream = nullptr;
  double* h_pinned = nullptr;  // 512 doubles of per-iteration scalars
  char* h_up = nullptr;        // packed staging, kPackStage bytes each
  char* h_down = nullptr;
};

// Device and staging addresses of one packed job inside its batch block.
struct PackedSlot {
  size_t up_off, down_off;  // offsets within the upload / download regions
  double *ub, *omega, *delta, *phi;
  void* psi0;  // complex128 initial state or null
  double* out;
  uint64_t* idx;
  void* state;  // complex128 final state or null
  void *diag, *psi, *basis;
  double* scratch;
  int status;  // RSV_OK, or an input error found on the host
};

// Runs a packed batch: one upload, per-job diagonal builds, one packed launch, per-job
// samples and state exports, one download.  Completions are appended to `out`.
int run_batch(rsv_server* srv, Work& w, LaneBuffers& lb, std::vector<rsv_completion>& out,
              double t_start) {
  const size_t count = w.jobs.size();
  const int prec = w.jobs[0]->prec;
  hipStream_t s = lb.stream;
  size_t up_total = granule(count * sizeof(PackedJob)), down_total = 0, work_total = 0;
  for (Job* j : w.jobs) {
    up_total += j->up;
    down_total += j->down;
    work_total += j->work;
  }
  char* up_base = (char*)w.block;  // [descriptors | per-job inputs]
  char* down_base = up_base + up_total;
  char* work_base = down_base + down_total;
  std::vector<PackedSlot> slot(count);
  PackedJob* desc = (PackedJob*)lb.h_up;
  size_t uo = granule(count * sizeof(PackedJob)), dw = 0, wo = 0;
  int launched = 0;
  for (size_t i = 0; i < count; ++i) {
    Job* j = w.jobs[i];
    PackedSlot& sl = slot[i];
    const size_t dim = size_t(1) << j->n, cnt = pulse_count(*j);
    auto take_up = [&](size_t bytes, const void* src) {
      std::memcpy(lb.h_up + uo, src, bytes);
      void* dev = up_base + uo;
      uo += granule(bytes);
      return dev;
    };
    sl.up_off = uo;
    sl.status = build_interactions(j->n, j->xyz.data(), j->c6, (double*)(lb.h_up + uo));
    sl.ub = (double*)(up_base + uo);
    uo += granule(32 * 32 * 8);
    sl.omega = (double*)take_up(cnt * 8, j->omega.data());
    sl.delta = (double*)take_up(cnt * 8, j->delta.data());
    sl.phi = j->phi.empty() ? nullptr : (double*)take_up(cnt * 8, j->phi.data());
    sl.psi0 = j->psi0.empty() ? nullptr : take_up(dim * 16, j->psi0.data());
    sl.down_off = dw;
    sl.out = (double*)(down_base + dw);
    dw += granule(kPackOutDoubles * 8);
    sl.idx = (uint64_t*)(down_base + dw);
    dw += granule((size_t)j->shots * 8);
    sl.state = j->return_state ? down_base + dw : nullptr;
    dw += j->return_state ? granule(dim * 16) : 0;
    sl.diag = work_base + wo;
    wo += granule(dim * (prec == kC128 ? 8 : 4));
    sl.psi = work_base + wo;
    wo += granule(vec_bytes(j->n, prec));
    sl.basis = work_base + wo;
    wo += granule((size_t)j->opts.kmax * vec_bytes(j->n, prec));
    sl.scratch = (double*)(work_base + wo);
    wo += j->shots > 0 ? granule((size_t)sample_scratch_doubles(j->n) * 8) : 0;
    if (sl.status != RSV_OK) continue;
    PackedJob& d = desc[launched++];
    d.n = j->n;
    d.dt_ns = j->opts.dt_ns;
    d.kmax = j->opts.kmax;
    d.max_depth = j->opts.max_substep_depth;
    d.per_site = j->pulses.per_site;
    d.init_zero = j->psi0.empty() ? 1 : 0;
    d.first_step = j->first_step;
    d.n_steps = j->n_steps;
    d.n_samples = j->pulses.n_samples;
    d.tol = j->opts.tol;
    d.omega = sl.omega;
    d.delta = sl.delta;
    d.phi = sl.phi;
    d.diag = sl.diag;
    d.psi = sl.psi;
    d.basis = sl.basis;
    d.out = sl.out;
  }
  HIP_TRY(hipMemcpyAsync(up_base, lb.h_up, up_total, hipMemcpyHostToDevice, s));
  for (size_t i = 0; i < count; ++i) {
    const PackedSlot& sl = slot[i];
    const Job* j = w.jobs[i];
    if (sl.status != RSV_OK) continue;
    HIP_TRY(diag_build(prec, j->n, sl.ub, sl.diag, s));
    if (sl.psi0) {
      if (prec == kC128)
        HIP_TRY(hipMemcpyAsync(sl.psi, sl.psi0, (size_t(1) << j->n) * 16, hipMemcpyDeviceToDevice, s));
      else
        HIP_TRY(convert_from_c128(prec, j->n, sl.psi0, sl.psi, s));
    }
  }
  HIP_TRY(packed_evolve(prec, (const PackedJob*)up_base, launched, s));
  for (size_t i = 0; i < count; ++i) {
    const PackedSlot& sl = slot[i];
    const Job* j = w.jobs[i];
    if (sl.status != RSV_OK) continue;
    if (j->shots > 0) HIP_TRY(sample(prec, j->n, sl.psi, j->seed, j->shots, sl.scratch, sl.idx, s));
    if (sl.state) {
      if (prec == kC128)
        HIP_TRY(hipMemcpyAsync(sl.state, sl.psi, (size_t(1) << j->n) * 16, hipMemcpyDeviceToDevice, s));
      else
        HIP_TRY(convert_to_c128(prec, j->n, sl.psi, sl.state, s));
    }
  }
  if (down_total) HIP_TRY(hipMemcpyAsync(lb.h_down, down_base, down_total, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double t_end = srv->now();
  for (size_t i = 0; i < count; ++i) {
    const PackedSlot& sl = slot[i];
    Job* j = w.jobs[i];
    rsv_completion c;
    std::memset(&c, 0, sizeof c);
    c.infidelity_fp64 = c.max_occ_err_fp64 = -1.0;
    c.job_id = j->id;
    c.tag = j->tag;
    c.n_atoms = j->n;
    c.t_submit = j->t_submit;
    c.t_start = t_start;
    c.t_end = t_end;
    int status = sl.status;
    const double* o = (const double*)(lb.h_down + sl.down_off);
    if (status == RSV_OK) {
      status = (int)o[0];
      if (status == RSV_ENOTCONV)
        fail(status, "Krylov estimate above tolerance at the deepest sub-step");
      else if (status != RSV_OK)
        fail(status, "non-finite Lanczos coefficients or zero state");
      else if (!(o[4] > 0.0))
        status = fail(RSV_ENUMERIC, "state has zero norm");
    }
    if (status == RSV_OK) {
      const int n = j->n;
      c.stats.steps = j->n_steps;
      c.stats.krylov_iters = (int64_t)o[1];
      c.stats.krylov_max = (int64_t)o[2];
      c.stats.substeps = (int64_t)o[3];
      c.stats.norm_final = std::sqrt(o[4]);
      c.stats.seconds = t_end - t_start;
      c.occupations = new double[n];
      for (int a = 0; a < n; ++a) c.occupations[a] = o[kPackOccOffset + (n - 1 - a)] / o[4];
      if (j->shots > 0) {
        c.n_shots = j->shots;
        c.samples = new uint64_t[j->shots];
        std::memcpy(c.samples, lb.h_down + sl.down_off + granule(kPackOutDoubles * 8),
                    (size_t)j->shots * 8);
      }
      if (j->return_state) {
        const size_t b = (size_t(1) << n) * 16;
        c.state = new double[(size_t(1) << n) * 2];
        std::memcpy(c.state, (char*)sl.state - down_base + lb.h_down, b);
      }
    }
    fill_error(c, status);
    out.push_back(c);
  }
  return RSV_OK;
}

void lane_main(rsv_server* srv, bool packed_only) {
  (void)hipSetDevice(srv->ctx->device);
  LaneBuffers lb;
  bool ok = hipStreamCreateWithFlags(&lb.stream, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc((void**)&lb.h_pinned, 512 * sizeof(double), hipHostMallocDefault) ==
                hipSuccess;
  if (ok && srv->opts.pack_max_atoms > 0)
    ok = hipHostMalloc((void**)&lb.h_up, kPackStage, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&lb.h_down, kPackStage, hipHostMallocDefault) == hipSuccess;
  for (;;) {
    Work w;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      if (!take_work(srv, lk, w, packed_only)) break;
    }
    std::vector<rsv_completion> comps;
    const double t_start = srv->now();
    if (w.packed) {
      const int rc = ok ? run_batch(srv, w, lb, comps, t_start)
                        : fail(RSV_EDEVICE, "lane could not allocate its buffers");
      if (rc != RSV_OK) {  // a device error ends the whole batch
        for (rsv_completion& c : comps) free_completion(c);
        comps.clear();
        const double t_end = srv->now();
        for (Job* j : w.jobs) {
          rsv_completion c;
          std::memset(&c, 0, sizeof c);
          c.infidelity_fp64 = c.max_occ_err_fp64 = -1.0;
          c.job_id = j->id;
          c.tag = j->tag;
          c.n_atoms = j->n;
          c.t_submit = j->t_submit;
          c.t_start = t_start;
          c.t_end = t_end;
          fill_error(c, rc);
          comps.push_back(c);
        }
      }
    } else {
      Job* job = w.jobs[0];
      rsv_completion c;
      std::memset(&c, 0, sizeof c);
      c.infidelity_fp64 = c.max_occ_err_fp64 = -1.0;
      c.job_id = job->id;
      c.tag = job->tag;
      c.n_atoms = job->n;
      c.t_submit = job->t_submit;
      c.t_start = t_start;
      const int rc = ok ? run_job(srv, job, lb.stream, lb.h_pinned, c)
                        : fail(RSV_EDEVICE, "lane could not allocate its buffers");
      c.t_end = srv->now();
      fill_error(c, rc);
      comps.push_back(c);
    }
    // a job that failed part-way may still have work queued on the lane's stream: let it
    // drain before its memory goes back to the arena
    bool failed = false;
    for (const rsv_completion& c : comps) failed |= c.status != RSV_OK;
    if (failed && lb.stream) (void)hipStreamSynchronize(lb.stream);
    srv->arena.release(w.block, w.bytes);
    for (Job* j : w.jobs) delete j;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      srv->running -= (int)w.jobs.size();
      for (rsv_completion& c : comps) srv->done.push_back(c);
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();  // memory was released: queued jobs may fit now
  }
  if (lb.stream) (void)hipStreamDestroy(lb.stream);
  if (lb.h_pinned) (void)hipHostFree(lb.h_pinned);
  if (lb.h_up) (void)hipHostFree(lb.h_up);
  if (lb.h_down) (void)hipHostFree(lb.h_down);
}

}  // namespace

namespace {

int check_noise(const rsv_noise* nz, int n, int64_t last_member) {
  if (!(std::isfinite(nz->omega_rel_sigma) && nz->omega_rel_sigma >= 0.0 &&
        std::isfinite(nz->delta_sigma) && nz->delta_sigma >= 0.0 &&
        std::isfinite(nz->position_sigma_um) && nz->position_sigma_um >= 0.0))
    return fail(RSV_EINVAL, "noise standard deviations must be finite and >= 0");
  if (last_member < 0 || (uint64_t)last_member > (UINT64_MAX / 2 - 1) / (4 * (uint64_t)n + 1))
    return fail(RSV_EINVAL, "member index out of range");
  return RSV_OK;
}

// Validates and copies one job description (every array) into a Job.
int make_job(rsv_server* srv, const rsv_job_desc* jd, std::unique_ptr<Job>* out) {
  const int n = jd->n_atoms;
  RSV_TRY(check_state_args(n, jd->prec));
  if (!jd->xyz_um) return fail(RSV_EINVAL, "positions are NULL");
  RSV_TRY(check_pulses(&jd->pulses, n));
  int64_t first = 0, count = 0;
  RSV_TRY(check_opts(&jd->opts, &jd->pulses, &first, &count));
  if (jd->n_shots < 0) return fail(RSV_EINVAL, "n_shots must be >= 0");
  std::unique_ptr<Job> j(new (std::nothrow) Job());
  if (!j) return fail(RSV_ENOMEM, "host allocation failed");
  j->tag = jd->tag;
  j->n = n;
  j->prec = jd->prec;
  j->shots = jd->n_shots;
  j->seed = jd->seed;
  j->return_state = jd->return_state;
  j->verify = jd->verify_fp64 && jd->prec == kC64;
  j->c6 = jd->c6;
  j->xyz.assign(jd->xyz_um, jd->xyz_um + 3 * n);
  const size_t cnt = (size_t)jd->pulses.n_samples * (jd->pulses.per_site ? (size_t)n : 1);
  j->omega.assign(jd->pulses.omega, jd->pulses.omega + cnt);
  j->delta.assign(jd->pulses.delta, jd->pulses.delta + cnt);
  if (jd->pulses.phi) j->phi.assign(jd->pulses.phi, jd->pulses.phi + cnt);
  j->pulses = jd->pulses;
  j->pulses.omega = j->omega.data();
  j->pulses.delta = j->delta.data();
  j->pulses.phi = jd->pulses.phi ? j->phi.data() : nullptr;
  j->opts = jd->opts;
  if (jd->psi0_host) {
    const double* p = (const double*)jd->psi0_host;
    j->psi0.assign(p, p + (size_t(2) << n));
  }
  j->first_step = first;
  j->n_steps = count;
  // the packed kernel runs the three-term recurrence only
  j->packed = !jd->opts.reorth && !j->verify &&
              n <= std::min(srv->opts.pack_max_atoms, packed_max_atoms(jd->prec));
  if (j->packed) {
    packed_sizes(*j);
    // too large for one staging buffer: the plain path takes it
    j->packed = granule(sizeof(PackedJob)) + j->up <= kPackStage && j->down <= kPackStage;
  }
  j->bytes = j->packed ? batch_bytes(1, j->up, j->down, j->work)
                       : job_bytes(n, jd->opts.kmax, jd->prec, jd->n_shots);
  if (j->verify) j->bytes += job_bytes(n, jd->opts.kmax, kC128, 0);  // the reference run
  if (j->bytes > srv->arena.capacity())
    return fail(RSV_ENOMEM, "job needs %zu bytes, the arena holds %zu", j->bytes,
                srv->arena.capacity());
  *out = std::move(j);
  return RSV_OK;
}

// Queues jobs together, in order, or none of them; ids[i] receives job i's id.
int enqueue(rsv_server* srv, std::vector<std::unique_ptr<Job>>& jobs, uint64_t* ids) {
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(RSV_EINVAL, "server is shutting down");
    if (srv->opts.max_queue > 0 &&
        srv->queue.size() + jobs.size() > (size_t)srv->opts.max_queue)
      return fail(RSV_EBUSY, "queue full (%d jobs)", srv->opts.max_queue);
    const double t = srv->now();
    for (size_t i = 0; i < jobs.size(); ++i) {
      jobs[i]->id = srv->next_id++;
      jobs[i]->t_submit = t;
      if (ids) ids[i] = jobs[i]->id;
      srv->queue.push_back(jobs[i].release());
    }
  }
  // every idle lane looks: one woken lane may not be able to take the job (the small-job
  // lane takes packed jobs only, and a job may not fit the arena beside another lane's)
  srv->cv_work.notify_all();
  return RSV_OK;
}

}  // namespace

extern "C" {

size_t rsv_server_job_bytes(int n, int kmax, rsv_precision prec, int shots) {
  if (n < 1 || n > kMaxAtoms || kmax < 2 || kmax > kMaxKrylov || shots < 0) return 0;
  return job_bytes(n, kmax, prec, shots);
}

int rsv_server_create(rsv_ctx* ctx, const rsv_server_opts* opts, rsv_server** out) {
  if (!out) return fail(RSV_EINVAL, "out is NULL");
  *out = nullptr;
  if (!ctx || !opts) return fail(RSV_EINVAL, "NULL argument");
  if (opts->n_lanes < 1 || opts->n_lanes > 16) return fail(RSV_EINVAL, "n_lanes must be in 1..16");
  if (opts->max_queue < 0) return fail(RSV_EINVAL, "max_queue must be >= 0");
  if (opts->pack_max_atoms < 0 || opts->pack_max_atoms > kMaxPackBits)
    return fail(RSV_EINVAL, "pack_max_atoms must be in 0..%d", kMaxPackBits);
  if (opts->pack_max_jobs < 0) return fail(RSV_EINVAL, "pack_max_jobs must be >= 0");
  HIP_TRY(hipSetDevice(ctx->device));
  size_t bytes = opts->arena_bytes;
  if (bytes == 0) {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    bytes = free_b / 4 * 3;
  }
  std::unique_ptr<rsv_server> s(new (std::nothrow) rsv_server());
  if (!s) return fail(RSV_ENOMEM, "host allocation failed");
  s->ctx = ctx;
  s->opts = *opts;
  RSV_TRY(s->arena.init(bytes));
  s->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < opts->n_lanes; ++i) s->lanes.emplace_back(lane_main, s.get(), false);
  // with packing, one more lane runs only packed batches: a small job then never waits for a
  // lane held by a long plain job
  if (opts->pack_max_atoms > 0) s->lanes.emplace_back(lane_main, s.get(), true);
  *out = s.release();
  return RSV_OK;
}

int rsv_server_submit(rsv_server* srv, const rsv_job_desc* jd, uint64_t* job_id) {
  if (!srv || !jd) return fail(RSV_EINVAL, "NULL argument");
  std::vector<std::unique_ptr<Job>> one(1);
  RSV_TRY(make_job(srv, jd, &one[0]));
  return enqueue(srv, one, job_id);
}

int rsv_noise_member(const rsv_noise* nz, uint64_t seed, int n, int64_t s, const double* xyz,
                     double* factor, double* offsets, double* xyz_out) {
  if (!nz || !xyz || !factor || !offsets || !xyz_out) return fail(RSV_EINVAL, "NULL argument");
  RSV_TRY(check_noise(nz, n, s));
  noise_member(*nz, seed, n, s, xyz, factor, offsets, xyz_out);
  return RSV_OK;
}

int rsv_server_submit_ensemble(rsv_server* srv, const rsv_job_desc* jd, const rsv_noise* nz,
                               uint64_t noise_seed, int n_members, uint64_t* job_ids) {
  if (!srv || !jd || !nz) return fail(RSV_EINVAL, "NULL argument");
  if (n_members < 1) return fail(RSV_EINVAL, "n_members must be >= 1");
  const int n = jd->n_atoms;
  RSV_TRY(check_state_args(n, jd->prec));
  if (!jd->xyz_um) return fail(RSV_EINVAL, "positions are NULL");
  RSV_TRY(check_pulses(&jd->pulses, n));
  RSV_TRY(check_noise(nz, n, n_members - 1));
  const int64_t ns = jd->pulses.n_samples;
  const bool site_in = jd->pulses.per_site != 0;
  // detuning offsets make the pulses per-site; without them the member keeps the job's layout
  const bool site_out = site_in || nz->delta_sigma != 0.0;
  const size_t rows = site_out ? (size_t)n : 1;
  std::vector<std::unique_ptr<Job>> jobs(n_members);
  std::vector<double> xyz(3 * n), off(n), om(rows * ns), de(rows * ns), ph;
  if (jd->pulses.phi) ph.resize(rows * ns);
  for (int s = 0; s < n_members; ++s) {
    double factor = 1.0;
    noise_member(*nz, noise_seed, n, s, jd->xyz_um, &factor, off.data(), xyz.data());
    for (size_t r = 0; r < rows; ++r) {
      const size_t src = site_in ? r * ns : 0;
      for (int64_t k = 0; k < ns; ++k) {
        om[r * ns + k] = factor * jd->pulses.omega[src + k];
        de[r * ns + k] = jd->pulses.delta[src + k] + (site_out ? off[r] : 0.0);
        if (jd->pulses.phi) ph[r * ns + k] = jd->pulses.phi[src + k];
      }
    }
    rsv_job_desc m = *jd;
    m.xyz_um = xyz.data();
    m.pulses.per_site = site_out ? 1 : 0;
    m.pulses.omega = om.data();
    m.pulses.delta = de.data();
    m.pulses.phi = jd->pulses.phi ? ph.data() : nullptr;
    m.seed = jd->seed + (uint64_t)s;
    m.tag = jd->tag + (uint64_t)s;
    RSV_TRY(make_job(srv, &m, &jobs[s]));  // copies every array
  }
  return enqueue(srv, jobs, job_ids);
}

int rsv_server_poll(rsv_server* srv, rsv_completion* out, int max, int* n_out, int timeout_ms) {
  if (!srv || !n_out || (max > 0 && !out)) return fail(RSV_EINVAL, "NULL argument");
  *n_out = 0;
  std::unique_lock<std::mutex> lk(srv->mu);
  auto ready = [&] { return !srv->done.empty(); };
  if (timeout_ms < 0) srv->cv_done.wait(lk, ready);
  else srv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
  int k = 0;
  while (k < max && !srv->done.empty()) {
    out[k++] = srv->done.front();
    srv->done.pop_front();
  }
  *n_out = k;
  return RSV_OK;
}

void rsv_server_release(rsv_server*, rsv_completion* c) {
  if (c) free_completion(*c);
}

int rsv_server_cancel(rsv_server* srv, uint64_t job_id) {
  if (!srv) return fail(RSV_EINVAL, "NULL argument");
  Job* victim = nullptr;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
      if ((*it)->id == job_id) {
        victim = *it;
        srv->queue.erase(it);
        break;
      }
    }
    if (!victim) {
      if (job_id > 0 && job_id < srv->next_id)
        return fail(RSV_EBUSY, "job %llu is running or finished", (unsigned long long)job_id);
      return fail(RSV_EINVAL, "unknown job %llu", (unsigned long long)job_id);
    }
    rsv_completion c;
    std::memset(&c, 0, sizeof c);
    c.infidelity_fp64 = c.max_occ_err_fp64 = -1.0;
    c.job_id = victim->id;
    c.tag = victim->tag;
    c.n_atoms = victim->n;
    c.t_submit = victim->t_submit;
    c.t_start = c.t_end = srv->now();
    c.status = RSV_ECANCELLED;
    std::strncpy(c.error, "cancelled", sizeof c.error - 1);
    srv->done.push_back(c);
  }
  delete victim;
  srv->cv_done.notify_all();
  return RSV_OK;
}

int rsv_server_status(rsv_server* srv, int* queued, int* running, int* done, size_t* arena_used) {
  if (!srv) return fail(RSV_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(srv->mu);
  if (queued) *queued = (int)srv->queue.size();
  if (running) *running = srv->running;
  if (done) *done = (int)srv->done.size();
  if (arena_used) *arena_used = srv->arena.in_use();
  return RSV_OK;
}

void rsv_server_destroy(rsv_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    srv->stop = true;
    for (Job* j : srv->queue) delete j;
    srv->queue.clear();
  }
  srv->cv_work.notify_all();
  for (auto& t : srv->lanes) t.join();
  for (auto& c : srv->done) free_completion(c);
  delete srv;
}

}  // extern "C"
