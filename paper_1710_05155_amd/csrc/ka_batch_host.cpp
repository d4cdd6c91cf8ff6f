// ka_batch_host.cpp -- host side of batched execution (include/ka.h, "Batches").
//
// A batch keeps a member table (host copy + device copy), a device step base, and per
// segment (a run of steps with a fixed set of active members) a tile table built on the
// device.  The host cuts the steps it enqueues into segments at the steps where members
// finish or join, enqueues whole captured graphs of "G step kernels + base += G" and single
// launches for the rest.  Progress events let ka_batch_poll detach finished members without
// blocking.  A slot is reused only after its member's last step has completed on the device.
// Each upload of the member table goes through one of a ring of pinned staging copies,
// which the host rewrites only after that copy's previous upload has completed (an event):
// the DMA reads pinned memory when it executes, not when it is enqueued, so the host table
// itself (changed by later adds and by workgroup-size changes) is never read by a pending
// upload.
// Tile tables alternate between two device buffers; stream order puts each rebuild after
// every step that read the buffer before.
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <deque>
#include <new>
#include <string>
#include <vector>

#include "ka_objects.h"

namespace {

thread_local std::string g_batch_err;

int bfail(int code, const char *fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  ka_set_error(buf);
  return code;
}

int bhip(hipError_t e, const char *what)
{
  return bfail(KA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct Guard {
  int prev = -1;
  explicit Guard(int dev)
  {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~Guard()
  {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

}  // namespace

struct ka_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  int capacity = 0;
  int cus = 256;
  std::vector<ka::BatchMember> tab;      // host member table, per slot
  static constexpr int kStages = 4;
  ka::BatchMember *stage[kStages] = {};   // pinned staging copies for uploads
  hipEvent_t stage_ev[kStages] = {};      // completion of each copy's last upload
  int stage_next = 0;
  ka::BatchMember *d_tab = nullptr;
  long long *d_base = nullptr;           // device step base
  int *d_total = nullptr;
  int *d_tmember[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [buffer][wpt-1]
  int *d_tlocal[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int tcap[2][2] = {{0, 0}, {0, 0}};
  std::vector<ka_sim *> sims;            // per slot (nullptr = free)
  std::vector<int64_t> sweeps;           // per slot
  std::vector<std::vector<int>> class_sizes;  // per slot, graphs only
  // Infinity-Cache-aware admission (KA_BOPT_CACHE_BUDGET): members whose working set (n and
  // f) is at least budget/8 are "large"; a large member starts only while the large members
  // running with it fit the budget, otherwise it waits (FIFO) and starts at the step where
  // enough of them have finished.
  int64_t cache_budget = 0;
  std::vector<int64_t> ws;               // per slot: bytes of n and f
  std::vector<char> waiting_flag;        // per slot: added but not started yet
  std::deque<int> waiting;               // slots in admission order
  // One-at-a-time members (KA_BOPT_SOLO_BYTES): a member whose n and f take at least
  // solo_bytes fills the device with its own class passes; run inside the step kernels next
  // to other members, it would only push their state and its own out of the Infinity Cache.
  // Such members skip the step kernel: they queue in the order added and run one at a time,
  // each step advancing the running one by one launch of its own pass kernels
  // (ka_sim_passes) on the batch's stream, so that a step still advances every started member
  // by one class.
  int64_t solo_bytes = (int64_t)32 << 20;
  std::vector<char> solo;                // per slot
  std::deque<int> solo_waiting;          // solo slots not started yet, in admission order
  int seg_solo = -1;                     // the solo member running in the current segment
  int n_members = 0;                     // highest used slot + 1
  int64_t step = 0;                      // steps enqueued
  int64_t done_step = 0;                 // steps known complete on the device
  std::deque<std::pair<hipEvent_t, int64_t>> progress;
  std::vector<hipEvent_t> event_pool;
  bool dirty = false;                    // member table changed since the last upload
  bool autotune = true, tuned = false;
  int block = 256;
  int graph_steps = 64;
  // current segment
  bool seg_valid = false;
  int64_t seg_end = 0;
  int buf = 0;
  int T[2] = {0, 0};
  // one captured graph per tile buffer
  struct Graph {
    hipGraph_t g = nullptr;
    hipGraphExec_t x = nullptr;
    int T0 = -1, T1 = -1, block = 0, steps = 0;
  } graphs[2];
};

namespace {

hipEvent_t take_event(ka_batch *b)
{
  if (!b->event_pool.empty()) {
    hipEvent_t e = b->event_pool.back();
    b->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
  return e;
}

int tiles_per_plane(const ka_batch *b, int k, int block)
{
  const ka::BatchMember &m = b->tab[(size_t)k];
  if (m.kind == 0) {
    const int nsub = m.d == 2 ? 4 : 16;
    const int threads = nsub * 64 * ((m.P + 63) / 64);
    return (threads + block - 1) / block;
  }
  if (m.C == 1 && m.classes > 1) return 1;   // the whole sweep is one merged run
  int biggest = 0;
  for (int c : b->class_sizes[(size_t)k]) biggest = std::max(biggest, c);
  return (biggest + block - 1) / block;
}

bool active_at(const ka_batch *b, int k, int64_t s)
{
  return b->sims[(size_t)k] && b->tab[(size_t)k].s_begin <= s && s < b->tab[(size_t)k].s_end;
}

bool large_member(const ka_batch *b, int k)
{
  return b->cache_budget > 0 && !b->solo[(size_t)k] && b->ws[(size_t)k] * 8 >= b->cache_budget;
}

// Last step of the started solo member still running at step s (s itself when none runs).
int64_t solo_busy_until(const ka_batch *b, int64_t s)
{
  int64_t until = s;
  for (int k = 0; k < b->n_members; ++k)
    if (b->sims[(size_t)k] && b->solo[(size_t)k] && !b->waiting_flag[(size_t)k])
      until = std::max<int64_t>(until, b->tab[(size_t)k].s_end);
  return until;
}

// Bytes of large started members that still run at or after step s.
int64_t large_bytes_from(const ka_batch *b, int64_t s)
{
  int64_t bytes = 0;
  for (int k = 0; k < b->n_members; ++k)
    if (b->sims[(size_t)k] && !b->waiting_flag[(size_t)k] && large_member(b, k) && b->tab[(size_t)k].s_end > s)
      bytes += b->ws[(size_t)k];
  return bytes;
}

// Whether a waiting large member of ws bytes may start at step s next to `running` bytes of
// large members (always, when none runs).
bool fits_budget(const ka_batch *b, int64_t running, int64_t ws)
{
  return running == 0 || running + ws <= b->cache_budget;
}

void start_member(ka_batch *b, int k, int64_t s)
{
  ka::BatchMember &m = b->tab[(size_t)k];
  m.s_begin = s;
  m.s_end = s + (int64_t)m.C * b->sweeps[(size_t)k];
  b->waiting_flag[(size_t)k] = 0;
  b->dirty = true;
}

// Start waiting members, in order, that fit next to the large members running at the
// current step, and the next solo member once none runs.
void admit_waiting(ka_batch *b)
{
  while (!b->waiting.empty()) {
    const int k = b->waiting.front();
    if (!fits_budget(b, large_bytes_from(b, b->step), b->ws[(size_t)k])) break;
    b->waiting.pop_front();
    start_member(b, k, b->step);
  }
  // (a member with no sweeps ends where it starts, and the next one starts with it)
  while (!b->solo_waiting.empty() && solo_busy_until(b, b->step) == b->step) {
    start_member(b, b->solo_waiting.front(), b->step);
    b->solo_waiting.pop_front();
  }
}

// Step at which every member, waiting ones included, will have finished: the admissions of
// admit_waiting replayed on the host.
int64_t projected_end(const ka_batch *b)
{
  int64_t end = b->step;
  std::vector<std::pair<int64_t, int64_t>> large;   // (end step, bytes) of started large members
  for (int k = 0; k < b->n_members; ++k) {
    if (!b->sims[(size_t)k] || b->waiting_flag[(size_t)k]) continue;
    end = std::max<int64_t>(end, b->tab[(size_t)k].s_end);
    if (large_member(b, k) && b->tab[(size_t)k].s_end > b->step) large.emplace_back(b->tab[(size_t)k].s_end, b->ws[(size_t)k]);
  }
  int64_t s = b->step;
  for (int k : b->waiting) {
    for (;;) {
      int64_t running = 0, next = INT64_MAX;
      for (const auto &e : large)
        if (e.first > s) {
          running += e.second;
          next = std::min(next, e.first);
        }
      if (fits_budget(b, running, b->ws[(size_t)k])) break;
      s = next;
    }
    const int64_t e = s + (int64_t)b->tab[(size_t)k].C * b->sweeps[(size_t)k];
    large.emplace_back(e, b->ws[(size_t)k]);
    end = std::max(end, e);
  }
  // solo members one after another, the first when the running one ends
  int64_t solo_at = solo_busy_until(b, b->step);
  for (int k : b->solo_waiting) {
    solo_at += (int64_t)b->tab[(size_t)k].C * b->sweeps[(size_t)k];
    end = std::max(end, solo_at);
  }
  return end;
}

void drop_graph(ka_batch::Graph &g)
{
  if (g.x) (void)hipGraphExecDestroy(g.x);
  if (g.g) (void)hipGraphDestroy(g.g);
  g = ka_batch::Graph();
}

hipError_t grow(ka_batch *b, int buf, int w, int need)
{
  if (need <= b->tcap[buf][w]) return hipSuccess;
  // grow-only; earlier steps may still read the old buffer
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return e;
  const int cap = std::max(need, 2 * b->tcap[buf][w]);
  drop_graph(b->graphs[buf]);
  (void)hipFree(b->d_tmember[buf][w]);
  (void)hipFree(b->d_tlocal[buf][w]);
  b->d_tmember[buf][w] = b->d_tlocal[buf][w] = nullptr;
  b->tcap[buf][w] = 0;
  e = hipMalloc((void **)&b->d_tmember[buf][w], sizeof(int) * (size_t)cap);
  if (e == hipSuccess) e = hipMalloc((void **)&b->d_tlocal[buf][w], sizeof(int) * (size_t)cap);
  if (e == hipSuccess) b->tcap[buf][w] = cap;
  return e;
}

// Start the segment beginning at the current step: upload the member table if it changed,
// build the tile tables of the active members, and find where the segment ends.
hipError_t new_segment(ka_batch *b)
{
  hipError_t e = hipSuccess;
  if (b->dirty) {
    for (int k = 0; k < b->n_members; ++k)
      if (b->sims[(size_t)k])
        b->tab[(size_t)k].tiles_per_plane = b->solo[(size_t)k] ? 0 : tiles_per_plane(b, k, b->block);
    const int q = b->stage_next;
    e = hipEventSynchronize(b->stage_ev[q]);   // this copy's previous upload has been read
    if (e != hipSuccess) return e;
    const size_t bytes = sizeof(ka::BatchMember) * (size_t)std::max(1, b->n_members);
    std::memcpy(b->stage[q], b->tab.data(), bytes);
    e = hipMemcpyAsync(b->d_tab, b->stage[q], bytes, hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess) e = hipEventRecord(b->stage_ev[q], b->stream);
    if (e != hipSuccess) return e;
    b->stage_next = (q + 1) % ka_batch::kStages;
    b->dirty = false;
  }
  const int64_t S = b->step;
  int T[2] = {0, 0};
  int64_t end = INT64_MAX;
  b->seg_solo = -1;
  for (int k = 0; k < b->n_members; ++k) {
    if (!active_at(b, k, S)) continue;
    const ka::BatchMember &m = b->tab[(size_t)k];
    T[m.wpt - 1] += m.planes * m.tiles_per_plane;
    end = std::min<int64_t>(end, m.s_end);
    if (b->solo[(size_t)k]) b->seg_solo = k;
  }
  b->buf ^= 1;
  for (int w = 0; w < 2 && e == hipSuccess; ++w) {
    b->T[w] = T[w];
    if (T[w] == 0) continue;
    e = grow(b, b->buf, w, T[w]);
    if (e == hipSuccess) {
      ka::BatchTiles tt{b->d_tmember[b->buf][w], b->d_tlocal[b->buf][w], T[w]};
      e = ka::launch_batch_prepare(b->d_tab, b->n_members, S, w + 1, tt, b->d_total, b->stream);
    }
  }
  b->seg_end = end;
  b->seg_valid = e == hipSuccess;
  return e;
}

hipError_t launch_steps(ka_batch *b, int count)
{
  hipError_t e = hipSuccess;
  for (int q = 0; q < count && e == hipSuccess; ++q)
    for (int w = 0; w < 2 && e == hipSuccess; ++w)
      if (b->T[w] > 0) {
        ka::BatchTiles tt{b->d_tmember[b->buf][w], b->d_tlocal[b->buf][w], b->T[w]};
        e = ka::launch_batch_step(b->d_tab, tt, b->T[w], b->d_base, q, b->block, w + 1, b->stream);
      }
  if (e == hipSuccess) e = ka::launch_batch_advance(b->d_base, count, b->stream);
  return e;
}

hipError_t launch_graph(ka_batch *b)
{
  ka_batch::Graph &g = b->graphs[b->buf];
  if (!(g.x && g.T0 == b->T[0] && g.T1 == b->T[1] && g.block == b->block && g.steps == b->graph_steps)) {
    drop_graph(g);
    hipError_t e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipError_t le = launch_steps(b, b->graph_steps);
    e = hipStreamEndCapture(b->stream, &g.g);
    if (le != hipSuccess) e = le;
    if (e == hipSuccess) e = hipGraphInstantiate(&g.x, g.g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      drop_graph(g);
      return e;
    }
    g.T0 = b->T[0];
    g.T1 = b->T[1];
    g.block = b->block;
    g.steps = b->graph_steps;
  }
  return hipGraphLaunch(g.x, b->stream);
}

// The running solo member's launches for steps [from, from + count) of the current segment,
// which lies inside that member's steps.
hipError_t solo_passes(ka_batch *b, int64_t from, int64_t count)
{
  const int k = b->seg_solo;
  if (k < 0 || count <= 0) return hipSuccess;
  return ka_sim_passes(b->sims[(size_t)k], from - b->tab[(size_t)k].s_begin, count, b->stream);
}

hipError_t enqueue_steps(ka_batch *b, int64_t n)
{
  hipError_t e = hipSuccess;
  while (n > 0 && e == hipSuccess) {
    if (!b->seg_valid || b->dirty || b->step >= b->seg_end) {
      admit_waiting(b);
      e = new_segment(b);
      if (e != hipSuccess) break;
    }
    int64_t chunk = std::min<int64_t>(n, b->seg_end - b->step);
    if (b->T[0] == 0 && b->T[1] == 0) {
      // no step kernel in this segment: the device step base still moves by the whole chunk
      for (int64_t left = chunk; left > 0 && e == hipSuccess; left -= 1 << 30)
        e = ka::launch_batch_advance(b->d_base, (int)std::min<int64_t>(left, 1 << 30), b->stream);
      if (e == hipSuccess) e = solo_passes(b, b->step, chunk);
    } else {
      // each run of step kernels is followed by the solo member's launches for the same
      // steps (independent sims: their order does not matter)
      int64_t left = chunk, at = b->step;
      while (e == hipSuccess && b->graph_steps > 0 && left >= b->graph_steps) {
        e = launch_graph(b);
        if (e != hipSuccess) {
          // Nothing of a failed capture, instantiation or graph launch has run (for instance,
          // another thread used the legacy stream during the capture): the same steps are
          // launched directly.
          (void)hipGetLastError();
          e = launch_steps(b, b->graph_steps);
        }
        if (e == hipSuccess) e = solo_passes(b, at, b->graph_steps);
        left -= b->graph_steps;
        at += b->graph_steps;
      }
      while (e == hipSuccess && left > 0) {
        const int r = (int)std::min<int64_t>(left, 1024);
        e = launch_steps(b, r);
        if (e == hipSuccess) e = solo_passes(b, at, r);
        left -= r;
        at += r;
      }
    }
    b->step += chunk;
    n -= chunk;
  }
  if (e != hipSuccess) return e;
  hipEvent_t ev = take_event(b);
  e = hipEventRecord(ev, b->stream);
  if (e != hipSuccess) return e;
  b->progress.emplace_back(ev, b->step);
  return hipSuccess;
}

int64_t max_classes(const ka_batch *b)
{
  int64_t c = 1;
  for (int k = 0; k < b->n_members; ++k)
    if (b->sims[(size_t)k] && b->tab[(size_t)k].s_end > b->step) c = std::max<int64_t>(c, b->tab[(size_t)k].C);
  return c;
}

// Time equal numbers of real steps with each workgroup size (tile size) and keep the
// fastest.  The steps are the batch's own work: results do not depend on the tile size.
hipError_t autotune(ka_batch *b, int64_t &n_steps)
{
  const int blocks[3] = {128, 256, 512};
  const int64_t probe = std::min<int64_t>(2 * max_classes(b), n_steps / 4);
  if (probe < 4) return hipSuccess;  // too little work to tune on; keep the default size
  float ms[3] = {0.f, 0.f, 0.f};
  std::vector<std::pair<hipEvent_t, hipEvent_t>> evs;
  for (int q = 0; q < 3; ++q) {
    if (b->block != blocks[q]) {
      b->block = blocks[q];
      b->dirty = true;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    if (e == hipSuccess) e = enqueue_steps(b, probe);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e != hipSuccess) return e;
    evs.emplace_back(e0, e1);
    n_steps -= probe;
  }
  hipError_t e = hipStreamSynchronize(b->stream);
  if (e != hipSuccess) return e;
  int best = 0;
  for (int q = 0; q < 3; ++q) {
    (void)hipEventElapsedTime(&ms[q], evs[q].first, evs[q].second);
    (void)hipEventDestroy(evs[q].first);
    (void)hipEventDestroy(evs[q].second);
    if (ms[q] < ms[best]) best = q;
  }
  if (b->block != blocks[best]) {
    b->block = blocks[best];
    b->dirty = true;
  }
  b->tuned = true;
  return hipSuccess;
}

void detach(ka_batch *b, int slot)
{
  ka_sim *s = b->sims[(size_t)slot];
  s->t += b->sweeps[(size_t)slot];
  s->batch = nullptr;
  b->sims[(size_t)slot] = nullptr;
  b->sweeps[(size_t)slot] = 0;
  // the slot's device entry is already inactive for every later step; leave it in place
}

void harvest(ka_batch *b)
{
  while (!b->progress.empty()) {
    hipError_t q = hipEventQuery(b->progress.front().first);
    if (q != hipSuccess) break;
    b->done_step = std::max(b->done_step, b->progress.front().second);
    b->event_pool.push_back(b->progress.front().first);
    b->progress.pop_front();
  }
}

}  // namespace

extern "C" int ka_batch_create(int capacity, void *hip_stream, ka_batch **out)
{
  return ka_guard([&]() -> int {
    if (!out) return bfail(KA_EINVAL, "out is NULL");
    *out = nullptr;
    if (capacity < 1 || capacity > ka::kBatchMaxMembers)
      return bfail(KA_EINVAL, "capacity must be in [1, %d]", ka::kBatchMaxMembers);
    ka_batch *b = new (std::nothrow) ka_batch;
    if (!b) return bfail(KA_ENOMEM, "host allocation failed");
    (void)hipGetDevice(&b->device);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, b->device) == hipSuccess && cus > 0)
      b->cus = cus;
    b->capacity = capacity;
    b->sims.assign((size_t)capacity, nullptr);
    b->sweeps.assign((size_t)capacity, 0);
    b->class_sizes.assign((size_t)capacity, std::vector<int>());
    b->ws.assign((size_t)capacity, 0);
    b->waiting_flag.assign((size_t)capacity, 0);
    b->solo.assign((size_t)capacity, 0);
    hipError_t e = hipSuccess;
    if (hip_stream) {
      b->stream = (hipStream_t)hip_stream;
    } else {
      e = hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking);
      b->own_stream = e == hipSuccess;
    }
    b->tab.assign((size_t)capacity, ka::BatchMember{});
    for (int q = 0; q < ka_batch::kStages && e == hipSuccess; ++q) {
      e = hipHostMalloc((void **)&b->stage[q], sizeof(ka::BatchMember) * (size_t)capacity, hipHostMallocDefault);
      if (e == hipSuccess) e = hipEventCreateWithFlags(&b->stage_ev[q], hipEventDisableTiming);
    }
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_tab, sizeof(ka::BatchMember) * (size_t)capacity);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_base, sizeof(long long));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_total, sizeof(int));
    if (e == hipSuccess) e = hipMemsetAsync(b->d_base, 0, sizeof(long long), b->stream);
    if (e == hipSuccess) e = hipMemsetAsync(b->d_tab, 0, sizeof(ka::BatchMember) * (size_t)capacity, b->stream);
    if (e != hipSuccess) {
      for (int q = 0; q < ka_batch::kStages; ++q) {
        if (b->stage[q]) (void)hipHostFree(b->stage[q]);
        if (b->stage_ev[q]) (void)hipEventDestroy(b->stage_ev[q]);
      }
      (void)hipFree(b->d_tab);
      (void)hipFree(b->d_base);
      (void)hipFree(b->d_total);
      if (b->own_stream) (void)hipStreamDestroy(b->stream);
      delete b;
      return bhip(e, "ka_batch_create");
    }
    b->dirty = true;
    *out = b;
    return KA_OK;
  });
}

extern "C" int ka_batch_add(ka_batch *b, ka_sim *s, int64_t n_sweeps, int *slot)
{
  return ka_guard([&]() -> int {
    if (!b || !s) return bfail(KA_EINVAL, "NULL argument");
    if (s->batch) return bfail(KA_ESTATE, "sim is already a batch member");
    if (!s->n) return bfail(KA_ESTATE, "sim has no device state");
    if (s->device != b->device) return bfail(KA_EINVAL, "sim and batch are on different devices");
    if (n_sweeps < 0) return bfail(KA_EINVAL, "n_sweeps < 0");
    if (s->t + n_sweeps >= (1ll << 32)) return bfail(KA_ESTATE, "sweep index would reach 2^32");
    int k = 0;
    while (k < b->capacity && b->sims[(size_t)k]) ++k;
    if (k == b->capacity) return bfail(KA_ESTATE, "batch is full (%d members)", b->capacity);
    Guard dg(b->device);
    // order the member's own earlier work (init, sweeps) before the batch's steps
    if (s->stream != b->stream) {
      hipEvent_t ev = take_event(b);
      hipError_t e = hipEventRecord(ev, s->stream);
      if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, ev, 0);
      b->event_pool.push_back(ev);
      if (e != hipSuccess) return bhip(e, "ka_batch_add ordering");
    }
    ka::BatchMember m{};
    m.n = s->n;
    m.f = s->f;
    m.edges = s->edges;
    m.nbr = s->nbr;
    m.stride = (long long)s->edges_total;
    m.class_start = s->class_start_d;
    m.fsat = s->fsat;
    m.kind = s->lattice ? 0 : 1;
    m.d = s->geom.d;
    m.L = s->geom.L;
    m.Q = s->geom.Q;
    m.P = s->geom.P;
    m.qinv = s->geom.qinv;
    m.N = (int)s->N;
    m.z = s->z;
    m.m = s->m;
    m.C = ka_sim_steps_per_sweep(s);   // below s->C when a graph's tiny tail is merged
    m.classes = s->C;
    m.planes = s->planes;
    m.wpt = s->wpt;
    m.key0 = (uint32_t)s->seed;
    m.key1 = (uint32_t)(s->seed >> 32);
    m.noise = s->noise;
    m.t0 = (uint32_t)s->t;
    b->class_sizes[(size_t)k].clear();
    if (!s->lattice)
      for (int c = 0; c < s->C; ++c) b->class_sizes[(size_t)k].push_back(s->plan->class_start[(size_t)c + 1] - s->plan->class_start[(size_t)c]);
    b->tab[(size_t)k] = m;
    b->sims[(size_t)k] = s;
    b->sweeps[(size_t)k] = n_sweeps;
    b->ws[(size_t)k] = (int64_t)2 * s->N * s->W * 8;
    b->solo[(size_t)k] = b->solo_bytes > 0 && b->ws[(size_t)k] >= b->solo_bytes;
    b->n_members = std::max(b->n_members, k + 1);
    if (b->solo[(size_t)k] && (!b->solo_waiting.empty() || solo_busy_until(b, b->step) > b->step)) {
      // runs when the solo members added before it have finished
      b->tab[(size_t)k].s_begin = INT64_MAX;
      b->tab[(size_t)k].s_end = INT64_MAX;
      b->waiting_flag[(size_t)k] = 1;
      b->solo_waiting.push_back(k);
    } else if (large_member(b, k) && (!b->waiting.empty() || !fits_budget(b, large_bytes_from(b, b->step), b->ws[(size_t)k]))) {
      // waits until enough of the large members already running have finished
      b->tab[(size_t)k].s_begin = INT64_MAX;
      b->tab[(size_t)k].s_end = INT64_MAX;
      b->waiting_flag[(size_t)k] = 1;
      b->waiting.push_back(k);
    } else {
      b->waiting_flag[(size_t)k] = 0;
      start_member(b, k, b->step);
    }
    b->dirty = true;
    s->batch = b;
    if (slot) *slot = k;
    return KA_OK;
  });
}

extern "C" int ka_batch_run(ka_batch *b, int64_t n_steps)
{
  return ka_guard([&]() -> int {
    if (!b) return bfail(KA_EINVAL, "batch is NULL");
    if (n_steps <= 0) return KA_OK;
    Guard dg(b->device);
    hipError_t e = hipSuccess;
    if (b->autotune && !b->tuned) e = autotune(b, n_steps);
    if (e == hipSuccess && n_steps > 0) e = enqueue_steps(b, n_steps);
    if (e != hipSuccess) return bhip(e, "ka_batch_run");
    return KA_OK;
  });
}

extern "C" int ka_batch_steps_left(const ka_batch *b, int64_t *steps_left)
{
  return ka_guard([&]() -> int {
    if (!b || !steps_left) return bfail(KA_EINVAL, "NULL argument");
    *steps_left = projected_end(b) - b->step;
    return KA_OK;
  });
}

extern "C" int ka_batch_poll(ka_batch *b, int *slots, int max_slots, int *n_done)
{
  return ka_guard([&]() -> int {
    if (!b) return bfail(KA_EINVAL, "batch is NULL");
    Guard dg(b->device);
    harvest(b);
    int got = 0;
    for (int k = 0; k < b->n_members; ++k) {
      if (!b->sims[(size_t)k] || b->tab[(size_t)k].s_end > b->done_step) continue;
      if (slots && got >= max_slots) break;
      detach(b, k);
      if (slots) slots[got] = k;
      ++got;
    }
    if (n_done) *n_done = got;
    return KA_OK;
  });
}

extern "C" int ka_batch_wait_all(ka_batch *b)
{
  return ka_guard([&]() -> int {
    if (!b) return bfail(KA_EINVAL, "batch is NULL");
    int64_t left = 0;
    ka_batch_steps_left(b, &left);
    int rc = ka_batch_run(b, left);
    if (rc) return rc;
    Guard dg(b->device);
    hipError_t e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) return bhip(e, "ka_batch_wait_all");
    harvest(b);
    b->done_step = b->step;
    for (int k = 0; k < b->n_members; ++k)
      if (b->sims[(size_t)k]) detach(b, k);
    return KA_OK;
  });
}

extern "C" int ka_batch_set_option(ka_batch *b, int option, int64_t value)
{
  return ka_guard([&]() -> int {
    if (!b) return bfail(KA_EINVAL, "batch is NULL");
    switch (option) {
      case KA_BOPT_AUTOTUNE:
        b->autotune = value != 0;
        return KA_OK;
      case KA_BOPT_BLOCK:
        if (value != 128 && value != 256 && value != 512) return bfail(KA_EINVAL, "block must be 128, 256 or 512");
        if (b->block != (int)value) b->dirty = true;
        b->block = (int)value;
        b->autotune = false;
        return KA_OK;
      case KA_BOPT_GRAPH_STEPS:
        if (value < 0 || value > 4096) return bfail(KA_EINVAL, "graph steps must be in [0, 4096]");
        b->graph_steps = (int)value;
        return KA_OK;
      case KA_BOPT_CACHE_BUDGET:
        if (value < 0) return bfail(KA_EINVAL, "cache budget must be >= 0");
        for (int k = 0; k < b->n_members; ++k)
          if (b->sims[(size_t)k]) return bfail(KA_ESTATE, "the cache budget is set while the batch has no members");
        b->cache_budget = value;
        return KA_OK;
      case KA_BOPT_SOLO_BYTES:
        if (value < 0) return bfail(KA_EINVAL, "solo bytes must be >= 0");
        for (int k = 0; k < b->n_members; ++k)
          if (b->sims[(size_t)k]) return bfail(KA_ESTATE, "the solo threshold is set while the batch has no members");
        b->solo_bytes = value;
        return KA_OK;
      default:
        return bfail(KA_EINVAL, "unknown batch option %d", option);
    }
  });
}

extern "C" int ka_batch_info(const ka_batch *b, int64_t *step, int *members, int *block, int *tiles)
{
  return ka_guard([&]() -> int {
    if (!b) return bfail(KA_EINVAL, "batch is NULL");
    int active = 0;
    for (int k = 0; k < b->n_members; ++k) active += b->sims[(size_t)k] != nullptr;
    if (step) *step = b->step;
    if (members) *members = active;
    if (block) *block = b->block;
    if (tiles) *tiles = b->T[0] + b->T[1];
    return KA_OK;
  });
}

extern "C" void ka_batch_free(ka_batch *b)
{
  try {
    if (!b) return;
    (void)ka_batch_wait_all(b);
    Guard dg(b->device);
    (void)hipStreamSynchronize(b->stream);
    drop_graph(b->graphs[0]);
    drop_graph(b->graphs[1]);
    for (auto &pr : b->progress) (void)hipEventDestroy(pr.first);
    for (hipEvent_t ev : b->event_pool) (void)hipEventDestroy(ev);
    for (int q = 0; q < 2; ++q)
      for (int w = 0; w < 2; ++w) {
        (void)hipFree(b->d_tmember[q][w]);
        (void)hipFree(b->d_tlocal[q][w]);
      }
    for (int q = 0; q < ka_batch::kStages; ++q) {
      (void)hipHostFree(b->stage[q]);
      (void)hipEventDestroy(b->stage_ev[q]);
    }
    (void)hipFree(b->d_tab);
    (void)hipFree(b->d_base);
    (void)hipFree(b->d_total);
    if (b->own_stream) (void)hipStreamDestroy(b->stream);
    delete b;
  } catch (...) {
  }
}

// Called by ka_free for a sim that is still a batch member.
int ka_batch_release_member(ka_batch *b, ka_sim *s)
{
  (void)s;
  return ka_batch_wait_all(b);
}
