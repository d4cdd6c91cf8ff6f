// ka_server.cpp -- job server with continuous batching (include/ka.h, "Serving").
//
// One worker thread owns a HIP stream and a batch.  Each pass of its loop:
//   1. takes newly submitted jobs into the FIFO queue;
//   2. admits queue heads while a slot is free and their device footprint fits the budget
//      (strict FIFO: a head that does not fit yet blocks the ones behind it, so big jobs
//      are not starved): initial-state kernels on a second stream, so that they overlap the
//      batch steps already queued; the batch stream waits for them (an event), and the job
//      joins the batch for the sweeps up to its next observation time;
//   3. enqueues a chunk of batch steps, keeping at most two chunks in flight;
//   4. detaches members whose segment completed, enqueues their observation (counts copied
//      into pinned host memory) and either re-adds them for the next segment or marks them
//      finishing;
//   5. retires finishing jobs whose last copy has landed (event): moves their counts out of
//      pinned memory, frees their device memory (a kept sim stays; it belongs to the caller
//      from then on and no longer counts against the budget, so that waiting for all jobs
//      before taking their sims cannot block admission) and publishes them to
//      ka_server_poll.
// HIP calls happen on the worker thread, except in ka_server_take_sim / ka_server_release,
// which touch only a completed job's own sim; the API functions share state under a mutex.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "ka_objects.h"

namespace {

using Clock = std::chrono::steady_clock;

int sfail(int code, const char *fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  ka_set_error(buf);
  return code;
}

struct Job {
  int64_t id = 0;
  const ka_graph *graph = nullptr;
  int m = 0;
  double rho = 0;
  uint64_t seed = 0;
  int R = 0;
  int64_t sweeps = 0;
  bool keep = false;
  std::vector<int64_t> obs;          // absolute sweep indices, non-decreasing
  size_t next = 0;                   // next observation to take
  size_t footprint = 0;
  double attempts = 0;               // N * R * sweeps
  ka_sim *sim = nullptr;
  unsigned long long *pinned = nullptr;  // [n_obs][3][R] while the job runs
  std::vector<int64_t> counts;           // [n_obs][3][R] once it is complete
  hipEvent_t done_ev = nullptr;
  int rc = KA_OK;
  Clock::time_point t_submit, t_admit, t_done;
};

constexpr int64_t kChunkSteps = 64;

}  // namespace

struct ka_server {
  size_t budget = 0;
  int max_active = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipStream_t init_stream = nullptr;   // initial states of admitted jobs
  ka_batch *batch = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_work;   // worker waits for submissions
  std::condition_variable cv_done;   // wait_idle waits for completions
  bool stop = false;
  int64_t next_id = 1;
  int64_t submitted = 0, completed = 0;
  std::deque<std::unique_ptr<Job>> incoming;   // guarded by mu
  std::vector<int64_t> done_ids;               // guarded by mu
  std::map<int64_t, std::unique_ptr<Job>> finished;  // guarded by mu
  // worker-only state
  std::deque<std::unique_ptr<Job>> queue;
  std::map<int, std::unique_ptr<Job>> active;  // by batch slot
  std::vector<std::unique_ptr<Job>> finishing;
  std::deque<hipEvent_t> inflight;
  size_t used = 0;                   // device bytes of admitted, unfinished jobs
  // statistics (guarded by mu)
  double attempts_done = 0;
  int peak_active = 0;
  size_t peak_bytes = 0;
  std::string worker_error;
};

namespace {

// A completed job: counts out of pinned memory, device memory freed unless the sim is kept.
void release_job_memory(Job *j)
{
  if (j->pinned) {
    if (j->rc == KA_OK) j->counts.assign(j->pinned, j->pinned + j->obs.size() * 3u * (size_t)j->R);
    (void)hipHostFree(j->pinned);
    j->pinned = nullptr;
  }
  if (j->sim && (!j->keep || j->rc != KA_OK)) {
    ka_free(j->sim);
    j->sim = nullptr;
  }
  if (j->done_ev) (void)hipEventDestroy(j->done_ev);
  j->done_ev = nullptr;
}

// Put a detached job back into the batch for the sweeps up to its next observation.
int rejoin(ka_server *sv, Job *j)
{
  const int64_t t = j->sim->t;
  const int64_t target = j->next < j->obs.size() ? j->obs[j->next] : j->sweeps;
  int slot = -1;
  int rc = ka_batch_add(sv->batch, j->sim, target - t, &slot);
  if (rc) return rc;
  return slot;
}

// Observe every observation due at the job's current t; returns true if the job is done.
bool observe_due(Job *j)
{
  while (j->next < j->obs.size() && j->obs[j->next] == j->sim->t) {
    unsigned long long *dst = j->pinned + j->next * 3u * (size_t)j->R;
    j->rc = ka_sim_observe_async(j->sim, dst);
    if (j->rc) return true;
    ++j->next;
  }
  return j->next >= j->obs.size();
}

void finish(ka_server *sv, std::unique_ptr<Job> j)
{
  if (!j->done_ev) {
    hipError_t e = hipEventCreateWithFlags(&j->done_ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(j->done_ev, sv->stream);
    if (e != hipSuccess) {
      // no event to poll: wait here, so that retire() never reads counts still in flight
      if (j->done_ev) (void)hipEventDestroy(j->done_ev);
      j->done_ev = nullptr;
      (void)hipStreamSynchronize(sv->stream);
    }
  }
  sv->finishing.push_back(std::move(j));
}

void admit(ka_server *sv)
{
  while (!sv->queue.empty() && (int)sv->active.size() < sv->max_active) {
    Job *j = sv->queue.front().get();
    if (sv->used + j->footprint > sv->budget) break;  // strict FIFO
    std::unique_ptr<Job> jp = std::move(sv->queue.front());
    sv->queue.pop_front();
    j->t_admit = Clock::now();
    j->rc = ka_init(j->graph, j->m, j->rho, j->seed, j->R, sv->init_stream, &j->sim);
    if (j->rc == KA_OK) {
      sv->used += j->footprint;  // returned in retire() while j->sim is set
      // everything after the init runs on the batch stream, ordered after it by an event
      hipEvent_t ev = nullptr;
      hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e == hipSuccess) e = hipEventRecord(ev, sv->init_stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(sv->stream, ev, 0);
      if (ev) (void)hipEventDestroy(ev);
      if (e != hipSuccess) (void)hipStreamSynchronize(sv->init_stream);
      ka_sim_rebind_stream(j->sim, sv->stream);
    }
    if (j->rc == KA_OK && hipHostMalloc((void **)&j->pinned, j->obs.size() * 3u * (size_t)j->R *
                                                                  sizeof(unsigned long long),
                                        hipHostMallocDefault) != hipSuccess)
      j->rc = KA_ENOMEM;
    if (j->rc != KA_OK) {
      finish(sv, std::move(jp));
      continue;
    }
    if (observe_due(j)) {
      finish(sv, std::move(jp));
      continue;
    }
    const int slot = rejoin(sv, j);
    if (slot < 0) {
      j->rc = slot;
      finish(sv, std::move(jp));
      continue;
    }
    sv->active[slot] = std::move(jp);
  }
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->peak_active = std::max(sv->peak_active, (int)sv->active.size());
  sv->peak_bytes = std::max(sv->peak_bytes, sv->used);
}

void collect(ka_server *sv)
{
  std::vector<int> slots(sv->active.size() + 1);
  int n = 0;
  if (ka_batch_poll(sv->batch, slots.data(), (int)slots.size(), &n) != KA_OK) return;
  for (int q = 0; q < n; ++q) {
    auto it = sv->active.find(slots[(size_t)q]);
    if (it == sv->active.end()) continue;
    std::unique_ptr<Job> jp = std::move(it->second);
    sv->active.erase(it);
    Job *j = jp.get();
    if (observe_due(j)) {
      finish(sv, std::move(jp));
      continue;
    }
    const int slot = rejoin(sv, j);
    if (slot < 0) {
      j->rc = slot;
      finish(sv, std::move(jp));
      continue;
    }
    sv->active[slot] = std::move(jp);
  }
}

void retire(ka_server *sv)
{
  std::vector<std::unique_ptr<Job>> keep;
  for (auto &jp : sv->finishing) {
    Job *j = jp.get();
    if (j->done_ev && hipEventQuery(j->done_ev) == hipErrorNotReady) {
      keep.push_back(std::move(jp));
      continue;
    }
    j->t_done = Clock::now();
    if (j->sim) sv->used -= std::min(sv->used, j->footprint);
    release_job_memory(j);
    std::lock_guard<std::mutex> lk(sv->mu);
    if (j->rc == KA_OK) sv->attempts_done += j->attempts;
    sv->done_ids.push_back(j->id);
    sv->completed += 1;
    sv->finished[j->id] = std::move(jp);
  }
  sv->finishing = std::move(keep);
  sv->cv_done.notify_all();
}

void worker_main(ka_server *sv)
{
  (void)hipSetDevice(sv->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      const bool idle = sv->queue.empty() && sv->active.empty() && sv->finishing.empty();
      if (idle && sv->incoming.empty()) {
        if (sv->stop) break;
        sv->cv_work.wait_for(lk, std::chrono::milliseconds(2));
      }
      while (!sv->incoming.empty()) {
        sv->queue.push_back(std::move(sv->incoming.front()));
        sv->incoming.pop_front();
      }
    }
    admit(sv);
    if (!sv->active.empty()) {
      // flow control: at most two chunks in flight
      while (sv->inflight.size() >= 2) {
        (void)hipEventSynchronize(sv->inflight.front());
        (void)hipEventDestroy(sv->inflight.front());
        sv->inflight.pop_front();
      }
      int64_t left = 0;
      (void)ka_batch_steps_left(sv->batch, &left);
      if (left > 0) {
        const int rc = ka_batch_run(sv->batch, std::min(left, kChunkSteps));
        if (rc != KA_OK) {
          {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->worker_error = ka_last_error();
          }
          // The batch cannot advance: its jobs end with the error instead of waiting for ever.
          for (auto &kv : sv->active) {
            kv.second->rc = rc;
            finish(sv, std::move(kv.second));
          }
          sv->active.clear();
        }
        hipEvent_t ev = nullptr;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess) {
          (void)hipEventRecord(ev, sv->stream);
          sv->inflight.push_back(ev);
        }
      } else if (!sv->inflight.empty()) {
        // everything is enqueued: wait for the oldest chunk to land before polling again
        (void)hipEventSynchronize(sv->inflight.front());
        (void)hipEventDestroy(sv->inflight.front());
        sv->inflight.pop_front();
      }
      collect(sv);
    } else {
      while (!sv->inflight.empty()) {
        (void)hipEventDestroy(sv->inflight.front());
        sv->inflight.pop_front();
      }
    }
    if (!sv->finishing.empty()) {
      if (sv->active.empty() && sv->queue.empty()) (void)hipStreamSynchronize(sv->stream);
      retire(sv);
    }
  }
  (void)hipStreamSynchronize(sv->stream);
  for (hipEvent_t ev : sv->inflight) (void)hipEventDestroy(ev);
  sv->inflight.clear();
}

}  // namespace

extern "C" int ka_server_create(size_t device_budget, int max_active, void *hip_stream, ka_server **out)
{
  return ka_guard([&]() -> int {
    if (!out) return sfail(KA_EINVAL, "out is NULL");
    *out = nullptr;
    if (max_active < 1 || max_active > ka::kBatchMaxMembers)
      return sfail(KA_EINVAL, "max_active must be in [1, %d]", ka::kBatchMaxMembers);
    if (device_budget == 0) return sfail(KA_EINVAL, "device budget is 0");
    ka_server *sv = new (std::nothrow) ka_server;
    if (!sv) return sfail(KA_ENOMEM, "host allocation failed");
    sv->budget = device_budget;
    sv->max_active = max_active;
    (void)hipGetDevice(&sv->device);
    hipError_t e = hipSuccess;
    if (hip_stream) {
      sv->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&sv->stream, hipStreamNonBlocking);
      sv->own_stream = e == hipSuccess;
    }
    if (e != hipSuccess) {
      delete sv;
      return sfail(KA_EDEVICE, "stream: %s", hipGetErrorString(e));
    }
    e = hipStreamCreateWithFlags(&sv->init_stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
      delete sv;
      return sfail(KA_EDEVICE, "stream: %s", hipGetErrorString(e));
    }
    int rc = ka_batch_create(max_active, sv->stream, &sv->batch);
    if (rc != KA_OK) {
      (void)hipStreamDestroy(sv->init_stream);
      if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
      delete sv;
      return rc;
    }
    // members come and go, so tuning on the first job's steps would not be representative
    (void)ka_batch_set_option(sv->batch, KA_BOPT_AUTOTUNE, 0);
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return KA_OK;
  });
}

extern "C" int ka_server_submit(ka_server *sv, const ka_job_desc *job, int64_t *job_id)
{
  return ka_guard([&]() -> int {
    if (!sv || !job || !job->graph) return sfail(KA_EINVAL, "NULL argument");
    if (job->n_sweeps < 0 || job->n_sweeps >= (1ll << 32)) return sfail(KA_EINVAL, "n_sweeps out of range");
    if (job->n_replicas <= 0 || job->n_replicas % 64 != 0) return sfail(KA_EINVAL, "n_replicas must be a positive multiple of 64");
    int64_t N = 0;
    int z = 0;
    ka_graph_info(job->graph, &N, &z, nullptr, nullptr);
    if (job->m < 0 || job->m > z - 1) return sfail(KA_EINVAL, "m out of range");
    if (!(job->rho >= 0.0 && job->rho <= 1.0)) return sfail(KA_EINVAL, "rho out of range");
    auto j = std::make_unique<Job>();
    j->graph = job->graph;
    j->m = job->m;
    j->rho = job->rho;
    j->seed = job->seed;
    j->R = job->n_replicas;
    j->sweeps = job->n_sweeps;
    j->keep = job->keep_sim != 0;
    if (job->obs_times && job->n_obs > 0) {
      int64_t prev = 0;
      for (int q = 0; q < job->n_obs; ++q) {
        const int64_t v = job->obs_times[q];
        if (v < prev || v > job->n_sweeps) return sfail(KA_EINVAL, "observation times must be non-decreasing in [0, n_sweeps]");
        j->obs.push_back(v);
        prev = v;
      }
    } else {
      j->obs.push_back(job->n_sweeps);
    }
    if (ka_footprint(job->graph, job->n_replicas, &j->footprint) != KA_OK) return KA_EINVAL;
    j->footprint += j->obs.size() * 3u * (size_t)job->n_replicas * 8u;
    if (j->footprint > sv->budget) return sfail(KA_EINVAL, "job needs %zu device bytes, budget is %zu", j->footprint, sv->budget);
    j->attempts = (double)N * (double)job->n_replicas * (double)job->n_sweeps;
    j->t_submit = Clock::now();
    std::lock_guard<std::mutex> lk(sv->mu);
    j->id = sv->next_id++;
    if (job_id) *job_id = j->id;
    sv->incoming.push_back(std::move(j));
    sv->submitted += 1;
    sv->cv_work.notify_one();
    return KA_OK;
  });
}

extern "C" int ka_server_poll(ka_server *sv, int64_t *job_ids, int max_ids, int *n)
{
  return ka_guard([&]() -> int {
    if (!sv) return sfail(KA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    int got = 0;
    while (got < max_ids && !sv->done_ids.empty()) {
      if (job_ids) job_ids[got] = sv->done_ids.front();
      sv->done_ids.erase(sv->done_ids.begin());
      ++got;
    }
    if (n) *n = got;
    return KA_OK;
  });
}

extern "C" int ka_server_result(ka_server *sv, int64_t job_id, int64_t *density, int64_t *overlap,
                                int64_t *persistence, double *wait_s, double *latency_s)
{
  return ka_guard([&]() -> int {
    if (!sv) return sfail(KA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->finished.find(job_id);
    if (it == sv->finished.end()) return sfail(KA_ESTATE, "job %lld is not complete", (long long)job_id);
    Job *j = it->second.get();
    if (j->rc != KA_OK) return sfail(j->rc, "job %lld failed", (long long)job_id);
    if (j->counts.size() != j->obs.size() * 3u * (size_t)j->R)
      return sfail(KA_ESTATE, "job %lld has no counts", (long long)job_id);
    const size_t R = (size_t)j->R;
    for (size_t q = 0; q < j->obs.size(); ++q)
      for (size_t b = 0; b < R; ++b) {
        const int64_t *row = j->counts.data() + q * 3u * R;
        if (density) density[q * R + b] = row[b];
        if (overlap) overlap[q * R + b] = row[R + b];
        if (persistence) persistence[q * R + b] = row[2 * R + b];
      }
    if (wait_s) *wait_s = std::chrono::duration<double>(j->t_admit - j->t_submit).count();
    if (latency_s) *latency_s = std::chrono::duration<double>(j->t_done - j->t_submit).count();
    return KA_OK;
  });
}

extern "C" int ka_server_take_sim(ka_server *sv, int64_t job_id, ka_sim **out)
{
  return ka_guard([&]() -> int {
    if (!sv || !out) return sfail(KA_EINVAL, "NULL argument");
    ka_sim *sim = nullptr;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      auto it = sv->finished.find(job_id);
      if (it == sv->finished.end()) return sfail(KA_ESTATE, "job %lld is not complete", (long long)job_id);
      Job *j = it->second.get();
      if (!j->keep || !j->sim) return sfail(KA_ESTATE, "job %lld kept no sim", (long long)job_id);
      sim = j->sim;
      j->sim = nullptr;
    }
    // The sim gets a stream of its own: the server's stream may end with the server, and the
    // worker may be capturing a graph on it, which the caller's thread must not synchronise.
    // The job is complete (its last copy has landed), so nothing of the sim is pending.
    const int rc = ka_sim_take_own_stream(sim, false);
    if (rc != KA_OK) {
      ka_free(sim);
      return rc;
    }
    *out = sim;
    return KA_OK;
  });
}

extern "C" int ka_server_release(ka_server *sv, int64_t job_id)
{
  return ka_guard([&]() -> int {
    if (!sv) return sfail(KA_EINVAL, "server is NULL");
    std::unique_ptr<Job> jp;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      auto it = sv->finished.find(job_id);
      if (it == sv->finished.end()) return sfail(KA_ESTATE, "job %lld is not complete", (long long)job_id);
      jp = std::move(it->second);
      sv->finished.erase(it);
      sv->done_ids.erase(std::remove(sv->done_ids.begin(), sv->done_ids.end(), job_id), sv->done_ids.end());
    }
    // The job is complete, so nothing of its sim is pending.  It moves to a stream of its own
    // before it is freed: the worker may be capturing a graph on the server's stream, which
    // another thread must not synchronise.
    if (jp->sim) {
      (void)ka_sim_take_own_stream(jp->sim, false);
      ka_free(jp->sim);
    }
    return KA_OK;
  });
}

extern "C" int ka_server_wait_idle(ka_server *sv)
{
  return ka_guard([&]() -> int {
    if (!sv) return sfail(KA_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->completed == sv->submitted; });
    if (!sv->worker_error.empty()) return sfail(KA_EDEVICE, "worker: %s", sv->worker_error.c_str());
    return KA_OK;
  });
}

extern "C" int ka_server_stats(ka_server *sv, int64_t *jobs_done, double *attempts, int *peak_active,
                               size_t *peak_bytes)
{
  return ka_guard([&]() -> int {
    if (!sv) return sfail(KA_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    if (jobs_done) *jobs_done = sv->completed;
    if (attempts) *attempts = sv->attempts_done;
    if (peak_active) *peak_active = sv->peak_active;
    if (peak_bytes) *peak_bytes = sv->peak_bytes;
    return KA_OK;
  });
}

extern "C" void ka_server_free(ka_server *sv)
{
  try {
    if (!sv) return;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->stop = true;
      sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    ka_batch_free(sv->batch);
    for (auto &kv : sv->finished) {
      Job *j = kv.second.get();
      if (j->sim) ka_free(j->sim);
      if (j->pinned) (void)hipHostFree(j->pinned);
      if (j->done_ev) (void)hipEventDestroy(j->done_ev);
    }
    (void)hipStreamSynchronize(sv->init_stream);
    (void)hipStreamDestroy(sv->init_stream);
    if (sv->own_stream) (void)hipStreamDestroy(sv->stream);
    delete sv;
  } catch (...) {
  }
}
