// Continuous-batching server: a stream of independent emulation jobs on one device.
//
// n_lanes worker threads each own a HIP stream and pinned host scalars.  A lane takes the
// first queued job (arrival order) whose device footprint fits in the arena, runs the
// whole job (diagonal, evolution, occupations, samples, optional state) on its stream and
// releases the footprint; kernels of concurrent jobs overlap on the device, and the host
// round trip of one job's Lanczos iteration is hidden behind the others' kernels.  Each
// job's memory is one arena block split by a bump allocator, so admission is exactly
// "the footprint fits" and nothing is allocated or freed on the device while serving.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <new>
#include <thread>
#include <vector>

#include "engine.h"

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

struct Job {
  uint64_t id = 0, tag = 0;
  int n = 0, prec = 0, shots = 0, return_state = 0;
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
  return RSV_OK;
}

Job* take_job(rsv_server* srv, std::unique_lock<std::mutex>& lk) {
  for (;;) {
    if (srv->stop) return nullptr;
    for (auto it = srv->queue.begin(); it != srv->queue.end(); ++it) {
      Job* j = *it;
      void* block = nullptr;
      if (srv->arena.alloc(j->bytes, &block) == RSV_OK) {
        j->block = block;
        srv->queue.erase(it);
        ++srv->running;
        return j;
      }
    }
    srv->cv_work.wait(lk);
  }
}

void lane_main(rsv_server* srv) {
  (void)hipSetDevice(srv->ctx->device);
  hipStream_t stream = nullptr;
  double* h_pinned = nullptr;
  const bool ok = hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) == hipSuccess &&
                  hipHostMalloc((void**)&h_pinned, 512 * sizeof(double), hipHostMallocDefault) ==
                      hipSuccess;
  for (;;) {
    Job* job = nullptr;
    {
      std::unique_lock<std::mutex> lk(srv->mu);
      job = take_job(srv, lk);
    }
    if (!job) break;
    rsv_completion c;
    std::memset(&c, 0, sizeof c);
    c.job_id = job->id;
    c.tag = job->tag;
    c.n_atoms = job->n;
    c.t_submit = job->t_submit;
    c.t_start = srv->now();
    const int rc = ok ? run_job(srv, job, stream, h_pinned, c)
                      : fail(RSV_EDEVICE, "lane could not create its stream");
    c.t_end = srv->now();
    fill_error(c, rc);
    srv->arena.release(job->block, job->bytes);
    delete job;
    {
      std::lock_guard<std::mutex> lk(srv->mu);
      --srv->running;
      srv->done.push_back(c);
    }
    srv->cv_done.notify_all();
    srv->cv_work.notify_all();  // memory was released: queued jobs may fit now
  }
  if (stream) (void)hipStreamDestroy(stream);
  if (h_pinned) (void)hipHostFree(h_pinned);
}

void free_completion(rsv_completion& c) {
  delete[] c.occupations;
  delete[] c.samples;
  delete[] (double*)c.state;
  c.occupations = nullptr;
  c.samples = nullptr;
  c.state = nullptr;
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
  for (int i = 0; i < opts->n_lanes; ++i) s->lanes.emplace_back(lane_main, s.get());
  *out = s.release();
  return RSV_OK;
}

int rsv_server_submit(rsv_server* srv, const rsv_job_desc* jd, uint64_t* job_id) {
  if (!srv || !jd) return fail(RSV_EINVAL, "NULL argument");
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
  j->bytes = job_bytes(n, jd->opts.kmax, jd->prec, jd->n_shots);
  if (j->bytes > srv->arena.capacity())
    return fail(RSV_ENOMEM, "job needs %zu bytes, the arena holds %zu", j->bytes,
                srv->arena.capacity());
  {
    std::lock_guard<std::mutex> lk(srv->mu);
    if (srv->stop) return fail(RSV_EINVAL, "server is shutting down");
    if (srv->opts.max_queue > 0 && (int)srv->queue.size() >= srv->opts.max_queue)
      return fail(RSV_EBUSY, "queue full (%d jobs)", srv->opts.max_queue);
    j->id = srv->next_id++;
    j->t_submit = srv->now();
    if (job_id) *job_id = j->id;
    srv->queue.push_back(j.release());
  }
  srv->cv_work.notify_one();
  return RSV_OK;
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
