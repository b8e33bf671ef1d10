// Serving: a scheduler thread admits cross-comparison jobs into resident
// device arenas, runs every admitted job that has not run yet in one bounded
// persistent launch (the aggregator stage of Section 4.1: small tile tasks
// grouped into one launch, one launcher for the device), and hands each
// job's counts and set sums back to the host.
//
// Per launch, on the compute stream: wait for the uploads, sccg_area_pairs
// (BATCHED) over the launch's contiguous pair range, sccg_jaccard_sets with
// one set per job, copies of the counts, sums and error word to pinned host
// memory, a clear of the error word, and an event.  Uploads (DMA of the
// job's host CSR and pairs, then a kernel that moves offsets and pair
// indices into arena coordinates) run on a second stream.
//
// Migration (Section 4.2, GPU to CPU): when jobs wait for admission because
// the arenas are full, the scheduler hands the smallest waiting job to a
// migration thread, which runs it with the host PixelBox and sums it on the
// host with the same exact arithmetic as the device.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fix192.h"
#include "host_pixelbox.h"
#include "sccg_common.h"
#include "serve_core.h"

using namespace sccg;
using namespace sccg::serve;

namespace {

constexpr int kMaxInflight = 4;
constexpr int kStepJobs = 1024;  // most jobs in one launch (size of the per-launch sum arrays)
constexpr int kServerStats = 12;
constexpr int kMaxCpuThreads = 256;

// Offsets of A and B move by their vertex shift; pair indices by the slot of
// their set's first polygon.
__global__ void k_serve_rebase(int64_t* offA, int64_t nA1, int64_t dA, int64_t* offB, int64_t nB1, int64_t dB,
                               int32_t* pa, int32_t* pb, int64_t np, int32_t sA, int32_t sB) {
  const int64_t total = nA1 + nB1 + np;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total; k += stride) {
    if (k < nA1) {
      offA[k] += dA;
    } else if (k < nA1 + nB1) {
      offB[k - nA1] += dB;
    } else {
      const int64_t q = k - nA1 - nB1;
      pa[q] += sA;
      pb[q] += sB;
    }
  }
}

__global__ void k_serve_clear_word(uint32_t* w) {
  if (threadIdx.x == 0) *w = 0u;
}

struct Job {
  uint64_t id = 0;
  sccg_polys A{}, B{};  // host
  int64_t n_pairs = 0;
  const int32_t* pa = nullptr;
  const int32_t* pb = nullptr;
  int64_t* out_i = nullptr;
  int64_t* out_u = nullptr;
  int64_t vA = 0, vB = 0;
  Footprint f{};
  Placement pl{};
  bool counted_wait = false;
  double t_submit = 0, t_admit = 0, t_launch = 0;
};

struct Slot {
  int64_t* d_setoff = nullptr;  // [kStepJobs + 1]
  int64_t* d_sums = nullptr;    // [3][kStepJobs]: sum_i, sum_u, n_contrib
  double* d_j = nullptr;        // [2][kStepJobs]: J, J'
  int64_t* h_setoff = nullptr;  // pinned mirrors
  int64_t* h_sums = nullptr;
  double* h_j = nullptr;
  uint32_t* h_err = nullptr;
  hipEvent_t uploaded = nullptr;
  hipEvent_t done = nullptr;
};

}  // namespace

struct sccg_server {
  explicit sccg_server(const sccg_server_config& c)
      : cfg(c),
        pipe(c.vertex_cap, c.slot_cap, c.pair_cap, c.max_step_pairs, c.max_inflight, kStepJobs),
        t0(std::chrono::steady_clock::now()) {}

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }

  int device = 0;
  sccg_server_config cfg;
  sccg_ctx* ctx = nullptr;
  hipStream_t stream = nullptr;  // launches and result copies
  hipStream_t copy = nullptr;    // uploads
  int32_t* d_xy = nullptr;       // [2 * vertex_cap]
  int64_t* d_off = nullptr;      // [slot_cap]
  int32_t* d_pa = nullptr;       // [pair_cap]
  int32_t* d_pb = nullptr;
  int64_t* d_i = nullptr;
  int64_t* d_u = nullptr;
  // pinned mirrors of the offset and pair arenas: a job's offsets and pair
  // indices are copied there first, so that their DMA is asynchronous (an
  // asynchronous copy from pageable memory waits for the copy stream)
  int64_t* h_off = nullptr;  // pinned [slot_cap]
  int32_t* h_pa = nullptr;   // pinned [pair_cap]
  int32_t* h_pb = nullptr;
  int64_t* h_i = nullptr;  // pinned [pair_cap]
  int64_t* h_u = nullptr;
  Slot slots[kMaxInflight];
  Pipeline<Job> pipe;  // scheduler thread only (too_big reads fixed capacities)
  std::chrono::steady_clock::time_point t0;
  std::thread thread;
  std::thread migrator;  // only with cfg.cpu_threads > 0
  // host worker pool: cpu_threads - 1 helpers that join the migration
  // thread on each migrated job
  std::vector<std::thread> helpers;
  std::mutex pmu;
  std::condition_variable pcv_go, pcv_done;
  HostWork* pwork = nullptr;  // guarded by pmu
  uint64_t pgen = 0;          // guarded by pmu: bumped for each job
  int pbusy = 0;              // guarded by pmu: helpers still on the current job
  bool pstop = false;         // guarded by pmu
  std::atomic<uint32_t> perr{0};

  std::mutex mu;
  std::condition_variable cv_work;
  std::condition_variable cv_done;
  std::condition_variable cv_host;
  // guarded by mu
  std::deque<Job*> incoming;
  std::deque<Job*> to_host;  // migrated jobs not started yet
  int host_jobs = 0;         // migrated jobs not finished yet
  bool host_stop = false;    // the migration thread may end
  std::deque<sccg_job_result> results;
  bool stop = false;
  int fatal = 0;
  std::string msg;
  uint64_t next_id = 1;
  int64_t stats[kServerStats] = {};
};

namespace {

sccg_job_result result_of(const Job* j, int status) {
  sccg_job_result r{};
  r.job_id = j->id;
  r.status = status;
  r.n_pairs = j->n_pairs;
  r.t_submit = j->t_submit;
  r.t_admit = j->t_admit;
  r.t_launch = j->t_launch;
  return r;
}

// Record a fatal HIP failure; every job still held completes with SCCG_E_HIP.
void set_fatal(sccg_server* s, const std::string& what) {
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->fatal) {
    s->fatal = SCCG_E_HIP;
    s->msg = what;
  }
}

#define SERVE_TRY(s, expr)                                                      \
  do {                                                                          \
    hipError_t e_ = (expr);                                                     \
    if (e_ != hipSuccess) {                                                     \
      set_fatal(s, std::string(#expr) + ": " + hipGetErrorString(e_));          \
      return false;                                                             \
    }                                                                           \
  } while (0)

// Device side of the pipeline (scheduler thread).
struct HipExec {
  sccg_server* s;

  int poll(int slot) {
    const hipError_t q = hipEventQuery(s->slots[slot].done);
    if (q == hipErrorNotReady) return 0;
    if (q != hipSuccess) {
      set_fatal(s, std::string("launch event: ") + hipGetErrorString(q));
      return -1;
    }
    return 1;
  }

  void admission_wait(Job*) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats[7] += 1;
  }

  // Copy one admitted job into its arena ranges (copy stream).
  bool upload(Job* j) {
    const int64_t nA = j->A.n_polys, nB = j->B.n_polys;
    const int64_t v = j->pl.vert_off, sl = j->pl.slot_off, p = j->pl.pair_off;
    if (j->vA > 0)
      SERVE_TRY(s, hipMemcpyAsync(s->d_xy + 2 * v, j->A.xy + 2 * j->A.offsets[0], (size_t)j->vA * 8,
                                  hipMemcpyHostToDevice, s->copy));
    if (j->vB > 0)
      SERVE_TRY(s, hipMemcpyAsync(s->d_xy + 2 * (v + j->vA), j->B.xy + 2 * j->B.offsets[0], (size_t)j->vB * 8,
                                  hipMemcpyHostToDevice, s->copy));
    memcpy(s->h_off + sl, j->A.offsets, (size_t)(nA + 1) * 8);
    memcpy(s->h_off + sl + nA + 1, j->B.offsets, (size_t)(nB + 1) * 8);
    memcpy(s->h_pa + p, j->pa, (size_t)j->n_pairs * 4);
    memcpy(s->h_pb + p, j->pb, (size_t)j->n_pairs * 4);
    SERVE_TRY(s, hipMemcpyAsync(s->d_off + sl, s->h_off + sl, (size_t)(nA + nB + 2) * 8, hipMemcpyHostToDevice,
                                s->copy));
    SERVE_TRY(s, hipMemcpyAsync(s->d_pa + p, s->h_pa + p, (size_t)j->n_pairs * 4, hipMemcpyHostToDevice, s->copy));
    SERVE_TRY(s, hipMemcpyAsync(s->d_pb + p, s->h_pb + p, (size_t)j->n_pairs * 4, hipMemcpyHostToDevice, s->copy));
    const int64_t total = nA + 1 + nB + 1 + j->n_pairs;
    const int blocks = (int)std::min<int64_t>((total + 255) / 256, 1024);
    hipLaunchKernelGGL(k_serve_rebase, dim3(blocks), dim3(256), 0, s->copy, s->d_off + sl, nA + 1,
                       v - j->A.offsets[0], s->d_off + sl + nA + 1, nB + 1, v + j->vA - j->B.offsets[0],
                       s->d_pa + p, s->d_pb + p, j->n_pairs, (int32_t)sl, (int32_t)(sl + nA + 1));
    SERVE_TRY(s, hipGetLastError());
    j->t_admit = s->now();
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats[4] = std::max(s->stats[4], s->pipe.arenas().vertices().used());
    s->stats[5] = std::max(s->stats[5], s->pipe.arenas().slots().used());
    s->stats[6] = std::max(s->stats[6], s->pipe.arenas().pairs().used());
    return true;
  }

  bool launch(const Step& st, Job* const* jobs, int si) {
    Slot& sl = s->slots[si];
    SERVE_TRY(s, hipEventRecord(sl.uploaded, s->copy));
    SERVE_TRY(s, hipStreamWaitEvent(s->stream, sl.uploaded, 0));
    sccg_polys arena{s->cfg.slot_cap - 1, s->d_off, s->d_xy};
    const int64_t off = st.pair_off;
    int r = sccg_area_pairs(s->ctx, &arena, &arena, st.n_pairs, s->d_pa + off, s->d_pb + off, s->d_i + off,
                            s->d_u + off, SCCG_BATCHED);
    if (r) {
      set_fatal(s, std::string("area pairs: ") + sccg_last_error(s->ctx));
      return false;
    }
    sl.h_setoff[0] = 0;
    for (int c = 0; c < st.count; ++c) sl.h_setoff[c + 1] = sl.h_setoff[c] + jobs[c]->n_pairs;
    SERVE_TRY(s, hipMemcpyAsync(sl.d_setoff, sl.h_setoff, (size_t)(st.count + 1) * 8, hipMemcpyHostToDevice,
                                s->stream));
    r = sccg_jaccard_sets(s->ctx, st.count, sl.d_setoff, s->d_i + off, s->d_u + off, s->cfg.jaccard_flags,
                          sl.d_sums, sl.d_sums + kStepJobs, sl.d_sums + 2 * kStepJobs, sl.d_j, sl.d_j + kStepJobs);
    if (r) {
      set_fatal(s, std::string("jaccard: ") + sccg_last_error(s->ctx));
      return false;
    }
    SERVE_TRY(s, hipMemcpyAsync(s->h_i + off, s->d_i + off, (size_t)st.n_pairs * 8, hipMemcpyDeviceToHost,
                                s->stream));
    SERVE_TRY(s, hipMemcpyAsync(s->h_u + off, s->d_u + off, (size_t)st.n_pairs * 8, hipMemcpyDeviceToHost,
                                s->stream));
    SERVE_TRY(s, hipMemcpyAsync(sl.h_sums, sl.d_sums, (size_t)3 * kStepJobs * 8, hipMemcpyDeviceToHost, s->stream));
    SERVE_TRY(s, hipMemcpyAsync(sl.h_j, sl.d_j, (size_t)2 * kStepJobs * 8, hipMemcpyDeviceToHost, s->stream));
    uint32_t* err = ctx_error_word(s->ctx);
    SERVE_TRY(s, hipMemcpyAsync(sl.h_err, err, 4, hipMemcpyDeviceToHost, s->stream));
    hipLaunchKernelGGL(k_serve_clear_word, dim3(1), dim3(64), 0, s->stream, err);
    SERVE_TRY(s, hipGetLastError());
    SERVE_TRY(s, hipEventRecord(sl.done, s->stream));
    const double t = s->now();
    for (int c = 0; c < st.count; ++c) jobs[c]->t_launch = t;
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats[2] += 1;
    s->stats[8] = std::max<int64_t>(s->stats[8], st.count);
    return true;
  }

  // The status one job's pairs give alone: run them again (they are still
  // resident) and read the error word they latch.
  int alone_status(int64_t off, int64_t n) {
    if (n <= 0) return SCCG_OK;
    sccg_polys arena{s->cfg.slot_cap - 1, s->d_off, s->d_xy};
    if (sccg_area_pairs(s->ctx, &arena, &arena, n, s->d_pa + off, s->d_pb + off, s->d_i + off, s->d_u + off,
                        SCCG_BATCHED) != SCCG_OK)
      return SCCG_E_HIP;
    uint32_t* errw = ctx_error_word(s->ctx);
    uint32_t e = 0;
    if (hipMemcpyAsync(&e, errw, 4, hipMemcpyDeviceToHost, s->stream) != hipSuccess) return SCCG_E_HIP;
    hipLaunchKernelGGL(k_serve_clear_word, dim3(1), dim3(64), 0, s->stream, errw);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess) return SCCG_E_HIP;
    return (e & kErrWatchdog) ? SCCG_E_DEVICE : (e ? SCCG_E_RANGE : SCCG_OK);
  }

  // Results of a finished launch: counts to the callers' arrays, sums to
  // the result queue.  The pipeline retires the jobs afterwards.
  void finish(const Step& st, Job* const* jobs, int si) {
    const Slot& sl = s->slots[si];
    const uint32_t err = *sl.h_err;
    const int status = (err & kErrWatchdog) ? SCCG_E_DEVICE : (err ? SCCG_E_RANGE : SCCG_OK);
    // A launch of several jobs that latched an error runs each job's pairs
    // again alone to learn which jobs the error belongs to, so that a job
    // reports the same status alone and in a mix (the counts are per pair
    // and do not change).  Should no job reproduce it, every job keeps the
    // launch's status.
    std::vector<int> job_status((size_t)st.count, status);
    if (err && st.count > 1) {
      int64_t p = st.pair_off;
      bool any = false;
      for (int c = 0; c < st.count; ++c) {
        job_status[(size_t)c] = alone_status(p, jobs[c]->n_pairs);
        any |= job_status[(size_t)c] != SCCG_OK;
        p += jobs[c]->n_pairs;
      }
      if (!any) std::fill(job_status.begin(), job_status.end(), status);
    }
    std::vector<sccg_job_result> out;
    out.reserve(st.count);
    int64_t pos = st.pair_off;
    for (int c = 0; c < st.count; ++c) {
      Job* j = jobs[c];
      if (j->out_i) memcpy(j->out_i, s->h_i + pos, (size_t)j->n_pairs * 8);
      if (j->out_u) memcpy(j->out_u, s->h_u + pos, (size_t)j->n_pairs * 8);
      pos += j->n_pairs;
      sccg_job_result r = result_of(j, job_status[(size_t)c]);
      r.jobs_in_launch = st.count;
      r.sum_i = sl.h_sums[c];
      r.sum_u = sl.h_sums[kStepJobs + c];
      r.n_contrib = sl.h_sums[2 * kStepJobs + c];
      r.j = sl.h_j[c];
      r.jprime = sl.h_j[kStepJobs + c];
      r.t_done = s->now();
      out.push_back(r);
      delete j;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (const sccg_job_result& r : out) s->results.push_back(r);
      s->stats[1] += (int64_t)out.size();
      s->stats[3] += st.n_pairs;
    }
    s->cv_done.notify_all();
  }
};

// One migrated job on the host: the host PixelBox for the counts, then the
// set sums of sccg_jaccard_sets (the same integer sums, the same binary64
// divisions and the same exact ratio sum, so the same bits).
sccg_job_result run_on_host(sccg_server* s, Job* j) {
  j->t_launch = s->now();
  std::vector<int64_t> bi, bu;
  int64_t* oi = j->out_i;
  int64_t* ou = j->out_u;
  if (!oi) {
    bi.resize((size_t)j->n_pairs);
    oi = bi.data();
  }
  if (!ou) {
    bu.resize((size_t)j->n_pairs);
    ou = bu.data();
  }
  // the job's pairs are shared by this thread and the pool's helpers
  HostWork w{&j->A, &j->B, j->pa, j->pb, oi, ou, j->n_pairs};
  const int nh = (int)s->helpers.size();
  if (nh > 0 && j->n_pairs > 64) {
    std::lock_guard<std::mutex> lk(s->pmu);
    s->pwork = &w;
    s->pgen += 1;
    s->pbusy = nh;
  }
  if (nh > 0 && j->n_pairs > 64) s->pcv_go.notify_all();
  uint32_t e = host_area_worker(w);
  if (nh > 0 && j->n_pairs > 64) {
    std::unique_lock<std::mutex> lk(s->pmu);
    s->pcv_done.wait(lk, [s] { return s->pbusy == 0; });
    s->pwork = nullptr;
    e |= s->perr.exchange(0);
  }
  const bool include_zero = (s->cfg.jaccard_flags & SCCG_J_INCLUDE_ZERO) != 0;
  uint64_t si = 0, su = 0, nn = 0;
  Fix192 acc;
  for (int64_t k = 0; k < j->n_pairs; ++k) {
    const int64_t I = oi[k], U = ou[k];
    if (!include_zero && I == 0) continue;
    si += (uint64_t)I;
    su += (uint64_t)U;
    nn += 1;
    if (U > 0) acc.add_ratio((double)I / (double)U);
  }
  sccg_job_result r = result_of(j, e ? SCCG_E_RANGE : SCCG_OK);
  r.jobs_in_launch = 0;
  r.sum_i = (int64_t)si;
  r.sum_u = (int64_t)su;
  r.n_contrib = (int64_t)nn;
  r.j = r.sum_u > 0 ? (double)r.sum_i / (double)r.sum_u : 0.0;
  r.jprime = nn > 0 ? acc.to_double() / (double)r.n_contrib : 0.0;
  r.t_done = s->now();
  return r;
}

// Scheduler thread: while the migration thread is idle and at least
// cpu_trigger jobs wait for admission, move the smallest waiting job to it.
int migrate(sccg_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->host_jobs > 0) return 0;
  }
  if ((int64_t)s->pipe.waiting() < s->cfg.cpu_trigger) return 0;
  Job* j = s->pipe.take_smallest(s->cfg.cpu_max_pairs);
  if (!j) return 0;
  j->t_admit = s->now();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->to_host.push_back(j);
    s->host_jobs += 1;
  }
  s->cv_host.notify_one();
  return 1;
}

// A helper of the host pool: takes part in every job the migration thread
// posts, until the pool stops.
void pool_helper(sccg_server* s) {
  uint64_t seen = 0;
  std::unique_lock<std::mutex> lk(s->pmu);
  for (;;) {
    s->pcv_go.wait(lk, [&] { return s->pstop || s->pgen != seen; });
    if (s->pstop) break;
    seen = s->pgen;
    HostWork* w = s->pwork;
    lk.unlock();
    const uint32_t e = host_area_worker(*w);
    if (e) s->perr.fetch_or(e);
    lk.lock();
    if (--s->pbusy == 0) s->pcv_done.notify_one();
  }
}

void migration_thread(sccg_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_host.wait(lk, [s] { return !s->to_host.empty() || s->host_stop; });
    if (s->to_host.empty()) break;
    Job* j = s->to_host.front();
    s->to_host.pop_front();
    lk.unlock();
    const sccg_job_result r = run_on_host(s, j);
    delete j;
    lk.lock();
    s->results.push_back(r);
    s->stats[1] += 1;
    s->stats[3] += r.n_pairs;
    s->stats[10] += 1;
    s->stats[11] += r.n_pairs;
    s->host_jobs -= 1;
    s->cv_done.notify_all();
    s->cv_work.notify_one();
  }
}

// After a failure: wait for the streams, then complete every held job with
// the error.
void fail_all(sccg_server* s) {
  (void)hipStreamSynchronize(s->stream);
  (void)hipStreamSynchronize(s->copy);
  std::vector<sccg_job_result> out;
  int code;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    code = s->fatal;
  }
  s->pipe.drain([&](Job* j) {
    out.push_back(result_of(j, code));
    delete j;
  });
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (sccg_job_result& r : out) {
      r.t_done = s->now();
      s->results.push_back(r);
    }
    s->stats[1] += (int64_t)out.size();
  }
  s->cv_done.notify_all();
}

void scheduler(sccg_server* s) {
  (void)hipSetDevice(s->device);
  HipExec ex{s};
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    while (!s->incoming.empty()) {
      s->pipe.push(s->incoming.front());
      s->incoming.pop_front();
    }
    const bool stopping = s->stop;
    const bool failed = s->fatal != 0;
    lk.unlock();
    int moved = 0;
    if (failed) {
      if (!s->pipe.empty()) fail_all(s);
    } else {
      moved = s->pipe.pump(ex);
      if (moved < 0) {
        fail_all(s);  // the executor recorded the failure
        moved = 1;
      } else if (s->cfg.cpu_threads > 0) {
        moved += migrate(s);
      }
    }
    lk.lock();
    if (stopping && s->incoming.empty() && s->pipe.empty() && s->host_jobs == 0) break;
    if (moved > 0 || !s->incoming.empty()) continue;
    if (!s->pipe.in_flight() && (s->pipe.empty() || s->fatal)) {
      if (!s->stop)
        s->cv_work.wait(lk, [s] { return !s->incoming.empty() || s->stop; });
      else
        s->cv_work.wait(lk, [s] { return !s->incoming.empty() || s->host_jobs == 0; });
    } else {
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    }
  }
}

int server_fail(sccg_server* s, int code, const std::string& m) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->msg = m;
  return code;
}

void free_server(sccg_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.d_setoff) (void)hipFree(sl.d_setoff);
    if (sl.d_sums) (void)hipFree(sl.d_sums);
    if (sl.d_j) (void)hipFree(sl.d_j);
    if (sl.h_setoff) (void)hipHostFree(sl.h_setoff);
    if (sl.h_sums) (void)hipHostFree(sl.h_sums);
    if (sl.h_j) (void)hipHostFree(sl.h_j);
    if (sl.h_err) (void)hipHostFree(sl.h_err);
    if (sl.uploaded) (void)hipEventDestroy(sl.uploaded);
    if (sl.done) (void)hipEventDestroy(sl.done);
  }
  void* dev[] = {s->d_xy, s->d_off, s->d_pa, s->d_pb, s->d_i, s->d_u};
  for (void* p : dev)
    if (p) (void)hipFree(p);
  if (s->h_i) (void)hipHostFree(s->h_i);
  if (s->h_off) (void)hipHostFree(s->h_off);
  if (s->h_pa) (void)hipHostFree(s->h_pa);
  if (s->h_pb) (void)hipHostFree(s->h_pb);
  if (s->h_u) (void)hipHostFree(s->h_u);
  if (s->ctx) (void)sccg_destroy(s->ctx);
  if (s->stream) (void)hipStreamDestroy(s->stream);
  if (s->copy) (void)hipStreamDestroy(s->copy);
  delete s;
}

bool check_host_polys(const sccg_polys* P, int64_t* verts) {
  if (!P || P->n_polys < 0 || P->n_polys >= ((int64_t)1 << 31) || !P->offsets) return false;
  if (P->offsets[0] < 0) return false;
  for (int64_t k = 0; k < P->n_polys; ++k)
    if (P->offsets[k + 1] < P->offsets[k]) return false;
  *verts = P->offsets[P->n_polys] - P->offsets[0];
  return *verts == 0 || P->xy != nullptr;
}

}  // namespace

extern "C" {

int sccg_server_create(sccg_server** out, int hip_device, const sccg_server_config* config,
                       const sccg_params* params) {
  if (!out) return SCCG_E_ARG;
  *out = nullptr;
  sccg_server_config c{};
  if (config) c = *config;
  if (c.vertex_cap == 0) c.vertex_cap = (int64_t)1 << 28;
  if (c.slot_cap == 0) c.slot_cap = (int64_t)1 << 24;
  if (c.pair_cap == 0) c.pair_cap = (int64_t)1 << 23;
  if (c.max_step_pairs == 0) c.max_step_pairs = (int64_t)1 << 21;
  if (c.max_inflight == 0) c.max_inflight = 2;
  if (c.cpu_trigger == 0) c.cpu_trigger = 1;
  if (c.cpu_max_pairs == 0) c.cpu_max_pairs = (int64_t)1 << 20;
  if (c.vertex_cap < 1 || c.vertex_cap > ((int64_t)1 << 36) || c.slot_cap < 3 || c.slot_cap > INT32_MAX ||
      c.pair_cap < 1 || c.pair_cap >= ((int64_t)1 << 31) || c.max_step_pairs < 1 || c.max_inflight < 1 ||
      c.max_inflight > kMaxInflight || (c.jaccard_flags & ~SCCG_J_INCLUDE_ZERO) || c.cpu_threads < 0 ||
      c.cpu_threads > kMaxCpuThreads || c.cpu_trigger < 0 || c.cpu_max_pairs < 0)
    return SCCG_E_ARG;
  sccg_params p{};
  if (params) p = *params;
  p.flags |= SCCG_F_NO_GRAPH;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) return SCCG_E_ARG;
  if (hipSetDevice(hip_device) != hipSuccess) return SCCG_E_HIP;
  sccg_server* s = new sccg_server(c);
  s->device = hip_device;
  int r = SCCG_OK;
  if (hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&s->copy, hipStreamNonBlocking) != hipSuccess) {
    free_server(s);
    return SCCG_E_HIP;
  }
  if ((r = sccg_create(&s->ctx, hip_device, s->stream, &p)) != SCCG_OK) {
    free_server(s);
    return r;
  }
  if ((r = sccg_reserve(s->ctx, 0, 0, c.pair_cap)) != SCCG_OK) {
    free_server(s);
    return r;
  }
  bool ok = hipMalloc((void**)&s->d_xy, (size_t)c.vertex_cap * 8) == hipSuccess &&
            hipMalloc((void**)&s->d_off, (size_t)c.slot_cap * 8) == hipSuccess &&
            hipMalloc((void**)&s->d_pa, (size_t)c.pair_cap * 4) == hipSuccess &&
            hipMalloc((void**)&s->d_pb, (size_t)c.pair_cap * 4) == hipSuccess &&
            hipMalloc((void**)&s->d_i, (size_t)c.pair_cap * 8) == hipSuccess &&
            hipMalloc((void**)&s->d_u, (size_t)c.pair_cap * 8) == hipSuccess &&
            hipHostMalloc((void**)&s->h_i, (size_t)c.pair_cap * 8, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&s->h_off, (size_t)c.slot_cap * 8, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&s->h_pa, (size_t)c.pair_cap * 4, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&s->h_pb, (size_t)c.pair_cap * 4, hipHostMallocDefault) == hipSuccess &&
            hipHostMalloc((void**)&s->h_u, (size_t)c.pair_cap * 8, hipHostMallocDefault) == hipSuccess;
  for (int k = 0; ok && k < c.max_inflight; ++k) {
    Slot& sl = s->slots[k];
    ok = hipMalloc((void**)&sl.d_setoff, (kStepJobs + 1) * 8) == hipSuccess &&
         hipMalloc((void**)&sl.d_sums, 3 * kStepJobs * 8) == hipSuccess &&
         hipMalloc((void**)&sl.d_j, 2 * kStepJobs * 8) == hipSuccess &&
         hipHostMalloc((void**)&sl.h_setoff, (kStepJobs + 1) * 8, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&sl.h_sums, 3 * kStepJobs * 8, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&sl.h_j, 2 * kStepJobs * 8, hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc((void**)&sl.h_err, 8, hipHostMallocDefault) == hipSuccess &&
         hipEventCreateWithFlags(&sl.uploaded, hipEventDisableTiming) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess;
  }
  if (!ok) {
    free_server(s);
    return SCCG_E_NOMEM;
  }
  if (c.cpu_threads > 0) {
    for (int t = 1; t < c.cpu_threads; ++t) s->helpers.emplace_back(pool_helper, s);
    s->migrator = std::thread(migration_thread, s);
  }
  s->thread = std::thread(scheduler, s);
  *out = s;
  return SCCG_OK;
}

int sccg_server_submit(sccg_server* s, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs,
                       const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter, int64_t* out_union,
                       uint64_t* out_job_id) {
  if (!s) return SCCG_E_ARG;
  if (!out_job_id) return server_fail(s, SCCG_E_ARG, "out_job_id is NULL");
  int64_t vA = 0, vB = 0;
  if (!check_host_polys(A, &vA)) return server_fail(s, SCCG_E_ARG, "A: bad host CSR (NULL, negative or decreasing offsets)");
  if (!check_host_polys(B, &vB)) return server_fail(s, SCCG_E_ARG, "B: bad host CSR (NULL, negative or decreasing offsets)");
  if (n_pairs < 0 || n_pairs >= ((int64_t)1 << 31)) return server_fail(s, SCCG_E_ARG, "n_pairs outside [0, 2^31)");
  if (n_pairs > 0 && (!pair_a || !pair_b)) return server_fail(s, SCCG_E_ARG, "NULL pair array");
  for (int64_t k = 0; k < n_pairs; ++k)
    if (pair_a[k] < 0 || pair_a[k] >= A->n_polys || pair_b[k] < 0 || pair_b[k] >= B->n_polys)
      return server_fail(s, SCCG_E_ARG, "pair " + std::to_string(k) + " indexes outside its set");
  Job* j = new Job();
  j->A = *A;
  j->B = *B;
  j->n_pairs = n_pairs;
  j->pa = pair_a;
  j->pb = pair_b;
  j->out_i = out_inter;
  j->out_u = out_union;
  j->vA = vA;
  j->vB = vB;
  j->f = Footprint{vA + vB, A->n_polys + B->n_polys + 2, n_pairs};
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->fatal) {
    delete j;
    s->msg = "server failed earlier: " + s->msg;
    return SCCG_E_STATE;
  }
  if (n_pairs > 0 && s->pipe.too_big(j->f)) {
    delete j;
    s->stats[9] += 1;
    s->msg = "job larger than a server arena";
    return SCCG_E_NOMEM;
  }
  j->id = s->next_id++;
  j->t_submit = s->now();
  *out_job_id = j->id;
  s->stats[0] += 1;
  if (n_pairs == 0) {
    sccg_job_result r = result_of(j, SCCG_OK);
    r.t_admit = r.t_launch = r.t_done = j->t_submit;
    s->results.push_back(r);
    s->stats[1] += 1;
    delete j;
    lk.unlock();
    s->cv_done.notify_all();
    return SCCG_OK;
  }
  s->incoming.push_back(j);
  lk.unlock();
  s->cv_work.notify_one();
  return SCCG_OK;
}

int sccg_server_poll(sccg_server* s, sccg_job_result* out, int max_results, int64_t timeout_us) {
  if (!s || max_results < 0 || (max_results > 0 && !out)) return SCCG_E_ARG;
  std::unique_lock<std::mutex> lk(s->mu);
  if (s->results.empty() && timeout_us != 0 && max_results > 0) {
    auto ready = [s] { return !s->results.empty(); };
    if (timeout_us < 0)
      s->cv_done.wait(lk, ready);
    else
      s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  }
  int n = 0;
  while (n < max_results && !s->results.empty()) {
    out[n++] = s->results.front();
    s->results.pop_front();
  }
  return n;
}

int sccg_server_get_stats(sccg_server* s, int64_t* out, int n) {
  if (!s || !out || n < 0) return SCCG_E_ARG;
  std::lock_guard<std::mutex> lk(s->mu);
  const int m = std::min(n, kServerStats);
  for (int k = 0; k < m; ++k) out[k] = s->stats[k];
  return m;
}

double sccg_server_clock(const sccg_server* s) { return s ? s->now() : 0.0; }

const char* sccg_server_last_error(sccg_server* s) {
  if (!s) return "null server";
  std::lock_guard<std::mutex> lk(s->mu);
  return s->msg.c_str();
}

int sccg_server_destroy(sccg_server* s) {
  if (!s) return SCCG_E_ARG;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->host_stop = true;
  }
  s->cv_host.notify_all();
  if (s->migrator.joinable()) s->migrator.join();
  {
    std::lock_guard<std::mutex> lk(s->pmu);
    s->pstop = true;
  }
  s->pcv_go.notify_all();
  for (std::thread& t : s->helpers) t.join();
  (void)hipSetDevice(s->device);
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  if (s->copy) (void)hipStreamSynchronize(s->copy);
  free_server(s);
  return SCCG_OK;
}

}  // extern "C"
