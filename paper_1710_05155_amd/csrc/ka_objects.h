// ka_objects.h -- the opaque objects behind the C ABI (include/ka.h), shared by the host
// translation units of libka.
#pragma once

#include <stdint.h>

#include <exception>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "ka.h"
#include "ka_internal.h"

// Device schedule of a general graph, in device numbering: built once per graph on its first
// ka_init and copied to the device by every ka_init on that graph.
struct GraphPlan {
  std::vector<int32_t> label;     // device index of canonical vertex i
  std::vector<int32_t> site_of;   // canonical vertex of device index
  std::vector<int> class_start;   // [C+1]
  std::vector<int4> rec;          // class-sorted (u, v, e, class)
  std::vector<int32_t> nbr;       // [2(z-1)][E] neighbour lists of rec
};

struct ka_graph;

// The device schedule of a general graph (vertex numbering, class-sorted records, neighbour
// lists), built on first use and kept in the graph: later ka_init calls on the same graph only
// copy it to the device.  Null if host memory runs out.  ka_plan.cpp.
std::shared_ptr<const GraphPlan> graph_plan(const ka_graph *g);

struct ka_graph {
  int lattice = 0;  // 1: hypercubic lattice (d, L); 0: general z-regular graph
  int d = 0, L = 0;
  int64_t N = 0;
  int z = 0;
  int C = 0;
  std::vector<int32_t> adj;            // [N][z]
  std::vector<int32_t> eu, ev, ecls;   // canonical edges
  mutable std::mutex plan_mu;
  mutable std::shared_ptr<const GraphPlan> plan;   // general graphs, once built
};

struct ka_sim {
  // graph summary
  int lattice = 0;
  int z = 0, C = 0;
  int64_t N = 0;
  ka::LatticeGeom geom{};
  std::shared_ptr<const GraphPlan> plan;   // general graphs: schedule (label, class_start, ...)
  // parameters
  int m = 0;
  int64_t K = 0;
  uint64_t seed = 0;
  int R = 0, W = 0, wpt = 1, planes = 1;
  int64_t t = 0;
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // word planes on streams of their own (lattices, global path): even planes on
  // plane_stream[0], odd ones on plane_stream[1], forked from and joined to `stream`
  hipStream_t plane_stream[2] = {nullptr, nullptr};
  hipEvent_t fork_ev = nullptr;
  hipEvent_t join_ev[2] = {nullptr, nullptr};
  // device memory
  ka::u64 *n = nullptr, *n0 = nullptr, *f = nullptr;
  int32_t *nbr = nullptr;             // graphs: [2(z-1)][E] neighbour lists of the records
  size_t edges_total = 0;             // graphs: E
  int4 *edges = nullptr;
  int *class_start_d = nullptr;
  int32_t *site_of = nullptr;     // general graphs: canonical vertex of device index
  uint32_t *fsat = nullptr;       // general graphs: bit per (plane, element) set once f is all ones
  ka::u64 *thr_u = nullptr;
  long long *thr_i = nullptr;
  int *err = nullptr;
  unsigned long long *counts = nullptr;
  size_t counts_cap = 0;
  int64_t *obs_d = nullptr;
  size_t obs_cap = 0;
  // batch membership: while set, the sim is advanced by that batch only
  struct ka_batch *batch = nullptr;
  // options and timing
  bool init_checked = false;
  int path_opt = 0;
  int noise = 0;                  // KA_OPT_NOISE
  int plane_streams = 0;          // KA_OPT_PLANE_STREAMS
  int tail_opt = 1;               // KA_OPT_TAIL
  int plane_group = 0;            // lattices: planes per launch group chosen at init (0: all)
  int plane_group_opt = -1;       // KA_OPT_PLANE_GROUPS (-1: plane_group)
  int tail_first = 0;             // general graphs: first class of the trailing run of classes
                                  // of at most kTailEdges edges (C if that run is shorter than 2)
  size_t lds_bytes = 0;
  bool lds_fits = false;
  ka::u64 *lds_acc = nullptr;     // LDS lattice sweep: pre-generated acceptance words
  int64_t lds_acc_sweeps = 0;     // sweeps lds_acc holds (0: words drawn in the loop)
  bool lds_acc_tried = false;
  ka::u64 *lds_snap = nullptr;    // LDS sweep: snapshots of n and f taken at observation times
  size_t lds_snap_rows = 0;       // snapshot rows lds_snap holds
  int64_t timing_every = 0;
  int64_t launches = 0;
  int64_t timed = 0;
  double timed_ms = 0.0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
  std::vector<hipEvent_t> event_pool;
};

// Error message of the calling thread (ka_last_error), shared by the host sources.
void ka_set_error(const char *msg);
// Finish the batch work of a member that is being freed.
int ka_batch_release_member(ka_batch *b, ka_sim *s);
// Launches per sweep of the sim's global path: its classes, with the merged run of tiny
// trailing classes of a general graph counted as one.
int ka_sim_steps_per_sweep(const ka_sim *s);
// Launches p0 .. p0 + count - 1 of the sim's global path counted from sweep s->t (launch p:
// step p mod P of sweep s->t + p / P, P = ka_sim_steps_per_sweep), on `stream`, with the word
// planes in the sim's groups as ka_sweep runs them (each group through all `count` launches
// before the next); s->t is left as it is.  A batch runs its one-at-a-time members with it.
hipError_t ka_sim_passes(ka_sim *s, int64_t p0, int64_t count, hipStream_t stream);
// Counts of ka_observe enqueued on the sim's stream into pinned host memory (3 * R values).
int ka_sim_observe_async(ka_sim *s, unsigned long long *host_out);
// Move a sim onto a new stream that it owns (its old stream may then be destroyed).  With
// wait = false the caller guarantees that no work of the sim is pending on the old stream.
int ka_sim_take_own_stream(ka_sim *s, bool wait);
// Bind the sim to `stream`, which the caller has already ordered after the sim's pending work.
void ka_sim_rebind_stream(ka_sim *s, hipStream_t stream);

// Runs the body of a C entry point: an exception thrown inside (a failed host allocation, or
// anything else from the standard library) becomes an error code and a message instead of
// crossing the C boundary.
template <typename F>
int ka_guard(F &&body) noexcept
{
  try {
    return body();
  } catch (const std::bad_alloc &) {
    ka_set_error("host allocation failed");
    return KA_ENOMEM;
  } catch (const std::exception &e) {
    ka_set_error(e.what());
    return KA_EDEVICE;
  } catch (...) {
    ka_set_error("unexpected exception");
    return KA_EDEVICE;
  }
}
