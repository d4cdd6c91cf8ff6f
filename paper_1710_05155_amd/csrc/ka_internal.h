// ka_internal.h -- launch descriptors shared by the libka host code and its HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ka {

typedef unsigned long long u64;

// Device layout of a word plane of a lattice sim: sites are grouped by their coordinate
// residues a_nu = x_nu mod 4 ("sublattice" sub = sum_nu a_nu 4^nu); inside a sublattice by
// their block coordinates p_nu = x_nu / 4 (pos = sum_nu p_nu Q^nu, Q = L/4).  Element index
// = sub * P + pos with P = Q^d.  Every edge class is a union of whole sublattices (its lower
// endpoints), so one pass writes exactly half of the sublattices and threads that walk pos
// read and write consecutive addresses.  General graphs number vertices in breadth-first
// order (neighbours of nearby vertices land near each other); random counters and initial
// keys keep the canonical edge and vertex ids.
// An element holds wpt consecutive 64-bit words (wpt = 2 when the replica count is a
// multiple of 128: word pair p = words 2p, 2p+1; else 1); plane p covers words
// p*wpt .. p*wpt+wpt-1.

struct LatticeGeom {
  int d;        // 2 or 3
  int L;        // side
  int Q;        // L / 4
  int P;        // Q^d, elements per sublattice
  int N;        // L^d
  unsigned long long qinv;   // lattice_qinv(Q): division by Q as a multiply
};

// ceil(2^63 / Q).  For 0 <= n < 2^31 and 1 <= Q < 2^31, n / Q = high 64 bits of
// (2n) * qinv: with qinv = 2^63/Q + e, 0 <= e < 1, the product over 2^64 is n/Q + n e / 2^63
// and n e / 2^63 < 1/Q, which is below the distance from n/Q up to the next integer.
inline unsigned long long lattice_qinv(int Q)
{
  return ((1ull << 63) + (unsigned long long)Q - 1ull) / (unsigned long long)Q;
}

struct PassLattice {
  u64 *n;
  u64 *f;
  LatticeGeom g;
  int mu;
  int noise;                 // 0: acceptance bit per replica, 1: shared by all replicas
  int planes;                // planes in this launch
  int plane0;                // first plane of this launch
  int blocks_per_plane;
  uint32_t t, c, key0, key1;
  // 3D, Q a power of two >= 64: chunks visited in tiles of 2^row_tile_log2 rows (0 = in
  // order); q_log2 = log2(Q)
  int row_tile_log2;
  int q_log2;
};

struct PassGraph {
  u64 *n;
  u64 *f;
  const int4 *edges;         // all edges sorted by class: (u, v, e, class)
  const int32_t *nbr;        // [2(z-1)][E] neighbour lists of the records above
  size_t stride;             // E
  int first;                 // first edge of the class
  int count;                 // edges in the class
  int noise;                 // 0: acceptance bit per replica, 1: shared by all replicas
  int N;
  int plane0;                // first plane of this launch
  int planes;
  int blocks_per_plane;
  uint32_t t, c, key0, key1;
  // summary of full moved-ever elements: bit plane*N + i set once every word of f at
  // element i of plane `plane` is all ones (null: f always read where an exchange happens)
  uint32_t *fsat;
  // merged run of small classes (launch_tail_graph): classes c .. c_end - 1, bounds from
  // class_start ([C+1], device); first, count and blocks_per_plane are not used there
  const int *class_start;
  uint32_t c_end;
};

// Whole sweep loop inside one workgroup per plane (plane in LDS).
struct SweepLds {
  u64 *n;
  u64 *f;
  const u64 *n0;
  // lattice
  LatticeGeom g;
  // graph
  const int4 *edges;         // all edges sorted by class: (u, v, e, class)
  const int32_t *nbr;        // [2(z-1)][E]
  size_t stride;             // E
  const int *class_start;    // [C+1]
  int N;
  int C;
  int noise;                 // 0: acceptance bit per replica, 1: shared by all replicas
  uint32_t t0;
  int n_sweeps;
  // observations: absolute sweep indices (non-decreasing), rows of out [n_obs][3][R]
  const int64_t *obs_times;
  int n_obs;
  unsigned long long *obs_out;
  int R;
  uint32_t key0, key1;
  // acceptance words of these sweeps generated beforehand (null: drawn in the loop).
  // Lattices: element (((plane * n_sweeps + s) * C + c) * acc_slots + j) * 1024 + thread.
  // Graphs: element (plane * n_sweeps + s) * E + k for class-sorted edge k (E = stride), and
  // acc_slots is the most edges any class gives one of the 1024 threads.
  u64 *acc;
  int acc_slots;
  // observations as state snapshots (null: counted in the loop): row q holds n of every plane,
  // then f of every plane, each in the global layout ([planes][N][wpt]); counted afterwards by
  // the observation kernel
  u64 *snap;
};

struct InitArgs {
  int N;
  int64_t K;
  uint32_t key0, key1;
  u64 *thr_u;         // [R]
  long long *thr_i;   // [R]
  int *err;
  // fill
  u64 *n;
  u64 *n0;
  u64 *f;
  int planes;
  int is_lattice;
  LatticeGeom g;
  const int32_t *site_of;   // general graphs: canonical vertex of each device index
};

struct ObserveArgs {
  const u64 *n;
  const u64 *n0;
  const u64 *f;
  int N;
  int planes;
  int R;
  unsigned long long *out;   // [rows][3][R]: density, overlap, persistence (added to)
  int rows;                  // states counted by one launch (at least 1)
  size_t row_stride;         // elements from one row's n (and f) to the next; 0: one state
};

// Launchers (ka_kernels.hip).  Return hipSuccess or the launch error.
hipError_t launch_pass_lattice(const PassLattice &a, int m, int wpt, hipStream_t s);
hipError_t launch_pass_graph(const PassGraph &a, int z, int m, int wpt, hipStream_t s);
// Classes a.c .. a.c_end - 1 of a general graph, each of at most kTailEdges edges, in one
// launch of one workgroup per plane.
constexpr int kTailEdges = 512;
hipError_t launch_tail_graph(const PassGraph &a, int z, int m, int wpt, hipStream_t s);
hipError_t launch_sweep_lds(const SweepLds &a, bool lattice, int zdeg, int m, int wpt,
                            size_t lds_bytes, hipStream_t s);
hipError_t launch_init(const InitArgs &a, int R, int wpt, hipStream_t s);
hipError_t launch_observe(const ObserveArgs &a, int wpt, hipStream_t s);
// Fixed device scratch of the observation entry point that allocates nothing: 3 counts per
// replica for up to kObserveScratchReplicas replicas.  observe_scratch_setup takes its address
// on the current device (once per device; called by ka_init); observe_scratch returns it
// (null before the setup).
constexpr int kObserveScratchReplicas = 8192;
constexpr int kObserveScratchWords = 3 * kObserveScratchReplicas;
hipError_t observe_scratch_setup(int device);
unsigned long long *observe_scratch(int device);
hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s);
size_t sweep_lds_bytes(int N, int wpt);
// Edge slots per thread of the LDS lattice sweep (edges per class over its 1024 threads).
int lds_lattice_slots(int d, int P);
// Whether the LDS lattice sweep takes pre-generated acceptance words for this layout.
bool lds_accept_supported(int d, int wpt, int slots);
// Edge slots per thread of the LDS graph sweep for its largest class, and the most it takes
// pre-generated acceptance words for.
int lds_graph_slots(int max_class_edges);
constexpr int kLdsGraphAcceptSlots = 3;
bool lds_graph_accept_supported(int z, int wpt);
// Acceptance words of a.n_sweeps sweeps for the LDS lattice or graph sweep, into a.acc.
hipError_t launch_lds_accept(const SweepLds &a, bool lattice, int wpt, hipStream_t s);

// Spatial four-point sums (ka_pairs.hip).
constexpr int kMaxPairShells = 2049;   // r2_max <= 2048
struct PairArgs {
  const u64 *n;
  const u64 *n0;
  LatticeGeom g;
  int planes;
  const int4 *disp;                    // (dx, dy, dz, r2)
  int n_disp;
  int r2_max;
  unsigned long long *S2;              // [r2_max + 1]
  unsigned long long *S11;
};
hipError_t launch_pairs(const PairArgs &a, int wpt, hipStream_t s);
// Graphs without a geometry: out[0] += sum_i Q_i, out[1] += sum_i Q_i^2 with Q_i the number
// of replicas b with n_i^b(t) n_i^b(0) = 1.
struct PairGraphArgs {
  const u64 *n;
  const u64 *n0;
  int N;
  int planes;
  unsigned long long *out;             // [2]
};
hipError_t launch_pairs_graph(const PairGraphArgs &a, int wpt, hipStream_t s);
int max_lds_bytes();

}  // namespace ka

namespace ka {

// ------------------------------------------------------------------------------------
// Batched execution of many instances: one step kernel applies one class pass to every
// active member.  Member k is active for global steps s in [s_begin, s_end); at step s it
// runs class (s - s_begin) mod C of its sweep t0 + (s - s_begin) / C.
// ------------------------------------------------------------------------------------
constexpr int kBatchMaxMembers = 1024;

struct BatchMember {
  u64 *n;
  u64 *f;
  const int4 *edges;           // graphs: class-sorted (u, v, e, class)
  const int32_t *nbr;          // graphs: [2(z-1)][E] neighbour lists
  long long stride;            // graphs: E
  const int *class_start;      // graphs: [C+1]
  int kind;                    // 0 lattice, 1 graph
  int d, L, Q, P, N;           // lattice geometry (N for both)
  unsigned long long qinv;     // lattice: lattice_qinv(Q)
  int z, m, C, planes, wpt;    // C: steps per sweep
  int classes;                 // graphs: classes per sweep; when above C, the last step runs
                               // classes C-1 .. classes-1 in one workgroup per plane
  int noise;                   // 0: acceptance bit per replica, 1: shared by all replicas
  uint32_t key0, key1;
  uint32_t t0;
  int tiles_per_plane;         // tiles of BLOCK threads per plane (graphs: largest class)
  long long s_begin, s_end;
  uint32_t *fsat;              // graphs: summary of full moved-ever elements (PassGraph::fsat)
};

// Work list of one segment (steps between membership changes): tile q belongs to member
// member[q] as its tile local[q].  Built on the device by the prepare kernel; cap is the
// number of entries the host sized the buffers for and launches step kernels over (entries
// past the device's own total hold member -1, and none is written at or past cap).
struct BatchTiles {
  int *member;
  int *local;
  int cap;
};

hipError_t launch_batch_prepare(const BatchMember *mem, int n_members, long long step, int wpt,
                                BatchTiles tiles, int *total, hipStream_t s);
hipError_t launch_batch_step(const BatchMember *mem, BatchTiles tiles, int n_tiles, const long long *base,
                             int offset, int block, int wpt, hipStream_t s);
hipError_t launch_batch_advance(long long *base, int by, hipStream_t s);

}  // namespace ka
