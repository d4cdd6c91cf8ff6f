/*
 * ka.h -- C ABI of libka, the MI355X (gfx950) multispin Kob-Andersen Monte Carlo library.
 *
 * Method: Boccagna, "A Multispin Algorithm for the Kob-Andersen Stochastic Dynamics on
 * Regular Lattices" (arXiv 1710.05155).  Sec. 2.1 defines the model (hard-core particles
 * on a periodic hypercubic lattice or a random regular graph, activation number m <= z-1,
 * a particle at i may hop to an empty neighbour j iff i has at most m occupied neighbours
 * and j at most m+1); Sec. 3.1 the multispin coding (bit b of a site's word is the
 * occupation of independent replica b); Sec. 3.2 the bitwise exchange update; Sec. 2.2 and
 * Sec. 3.3 the overlap observables.
 *
 * Schedule (a reading of the paper, which updates one random pair at a time): one sweep
 * visits the edge classes c = 0..C-1 in order; the edges of one class are pairwise at
 * graph distance >= 2 and are updated together.  Every edge of the class is attempted
 * once per replica, accepted with an independent Bernoulli(1/2) bit:
 *     acceptance bit of replica b, edge e (canonical id), class c, sweep t
 *       = bit (b & 63) of half ((b >> 6) & 1) of Philox4x32-10(counter (t, c, e, b >> 7),
 *         key (seed & 0xffffffff, seed >> 32)),  half 0 = out0 | out1 << 32,
 *                                                half 1 = out2 | out3 << 32.
 * Classes: lattices 4*mu + ((x_mu + 2*sum_{nu != mu} x_nu) mod 4) for the edge
 * (x, x + e_mu), whose canonical id is e = i*d + mu with i = sum_nu x_nu L^nu; general
 * graphs: the greedy distance-2 edge colouring of the canonical edge list (all {u < v},
 * lexicographic, e = rank).
 * Initial state of replica b: the K sites with the smallest keys (u_i, i), u_i = half
 * (b & 1) of Philox4x32-10(counter (0, 0xFFFFFFFF, i, b >> 1), same key): a uniform sample
 * of the configurations with K particles (Sec. 3.1).
 *
 * Conventions
 *   - Every function returns KA_OK (0) or a negative error code; ka_last_error() gives a
 *     message for the calling thread.  No C++ exception crosses this boundary.
 *   - All pointer arguments are HOST pointers unless stated otherwise.  Inputs are copied;
 *     the caller keeps ownership of its buffers.  The library owns all device memory.
 *   - A ka_sim is bound to one device (the current one at ka_init) and one HIP stream.  No
 *     two host threads may use the same ka_sim at once.  ka_graph objects are immutable and
 *     may be shared and freed once the sims built from them exist.
 *   - Streams the library creates are non-blocking (hipStreamNonBlocking), and all device work
 *     of a call, copies included, runs on the object's stream; the library never uses the
 *     legacy default stream.
 *   - Canonical state export layout: uint64 [W][N], W = n_replicas / 64; bit (b & 63) of
 *     word [b >> 6][i] is replica b at site i.  The device layout is private.
 *   - The sweep index t counts sweeps since ka_init; it is part of the random counter, so a
 *     run split across calls equals the unsplit run.  t must stay below 2^32.
 */
#ifndef KA_H
#define KA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define KA_OK 0
#define KA_EINVAL (-1)  /* invalid argument (sizes, m, rho, replica count, graph)      */
#define KA_ENOMEM (-2)  /* host or device allocation failed                           */
#define KA_EDEVICE (-3) /* HIP runtime or kernel error                                */
#define KA_ESTATE (-4)  /* call not valid in the current state (e.g. t would overflow) */

typedef struct ka_graph ka_graph;
typedef struct ka_sim ka_sim;

/* Periodic hypercubic lattice Z_L^d (Sec. 2.1), d in {2, 3}, L >= 4, L % 4 == 0, z = 2d,
 * N = L^d <= 2^30.  Neighbour order in exports: +e_0, -e_0, +e_1, -e_1, ... */
int ka_graph_lattice(int d, int L, ka_graph **out);

/* Random z-regular simple graph on N vertices (Sec. 2.1, Bollobas' configuration model):
 * stubs s = 0..N*z-1 (stub s belongs to vertex s / z) are shuffled by Fisher-Yates
 * (k = S-1 down to 1, swap k with a uniform j in [0, k]) and positions (2q, 2q+1) paired;
 * a pairing with a self-loop or a repeated edge is rejected whole and attempt a+1 drawn.
 * 32-bit word s of attempt a is output s % 4 of Philox4x32-10(counter (a, 0xFFFFFFFE,
 * s/4 low, s/4 high), key graph_seed); uniform integers by Lemire's multiply-shift
 * rejection method.  z in [3, 6], z < N, N*z even, N <= 2^28.  Adjacency rows sorted.
 * Returns KA_ESTATE if no simple pairing is found within 10^6 attempts. */
int ka_graph_rrg(int64_t N, int z, uint64_t graph_seed, ka_graph **out);

/* Layered random graph (Sec. 5.2): M copies of the periodic lattice Z_L^d (d in {2, 3},
 * L >= 3); for every bond (x, x+e_mu) the M links (x, a)-(x+e_mu, a) become
 * (x, a)-(x+e_mu, P(a)) with P a uniform random permutation of the copies, independent per
 * bond.  Vertex (x, a) has id a*L^d + i(x); rows sorted.  P of the bond with lattice edge id
 * e = i*d + mu: Fisher-Yates (k = M-1 down to 1, swap k with U[0, k]) of 0..M-1 on the
 * 32-bit words of Philox4x32-10(counter (e, 0xFFFFFFFD, s/4, 0), key graph_seed), word s =
 * output s % 4, uniform integers by Lemire's method.  Canonical edges as for any graph;
 * classes: the lattice class of the lifted bond when L % 4 == 0 (C = 4d), else the greedy
 * distance-2 colouring.  M*L^d <= 2^28. */
int ka_graph_layered(int d, int L, int M, uint64_t graph_seed, ka_graph **out);

/* Any simple z-regular graph given as adjacency rows adj[N][z] (copied; z in [3, 6]).
 * KA_EINVAL if an entry is out of range, a self-loop, repeated, or not symmetric. */
int ka_graph_from_adjacency(int64_t N, int z, const int32_t *adj, ka_graph **out);

/* Sizes: N sites, degree z, number of edges (N*z/2), number of edge classes C. */
int ka_graph_info(const ka_graph *g, int64_t *N, int *z, int64_t *n_edges, int *n_classes);

/* Copies (any may be NULL): adj [N][z], and per canonical edge e its endpoints and its class
 * edge_class[e].  General graphs: edge_u[e] < edge_v[e]; lattices: edge_u = x and
 * edge_v = x + e_mu (the lattice lists are computed here, on the host, on each call). */
int ka_graph_export(const ka_graph *g, int32_t *adj, int32_t *edge_u, int32_t *edge_v,
                    int32_t *edge_class);

void ka_graph_free(ka_graph *g);

/* Device bytes a sim of this graph with n_replicas replicas allocates (serving admission).
 * No passage of the paper applies: this is library bookkeeping.
 * For an instance whose word plane fits in LDS this includes the buffer of acceptance words
 * that its LDS-resident sweeps generate ahead (at most 8 MiB, allocated on the first such
 * sweep; a layout whose words for a single sweep would exceed 8 MiB draws them in the loop
 * instead), and the state snapshots its ka_run observations are counted from (at most
 * 4 MiB, allocated by the first ka_run that takes them). */
int ka_footprint(const ka_graph *g, int n_replicas, size_t *device_bytes);

/* Create a simulation of n_replicas (a positive multiple of 64) independent replicas on the
 * current HIP device with activation number m (0 <= m <= z-1) and K = floor(rho*N + 1/2)
 * particles (rho in [0, 1], evaluated in IEEE double), and launch the initial-state
 * kernels on hip_stream (a hipStream_t; NULL = a stream the library creates and owns).
 * Returns once the kernels are enqueued; t = 0.  For a general graph the first ka_init
 * builds the device schedule (vertex numbering, class-sorted edges, neighbour lists) and
 * keeps a host copy in the graph, so later ka_init calls on it only upload it; the graph
 * may be freed while sims built from it still run.  Thread-safe on a shared graph. */
int ka_init(const ka_graph *g, int m, double rho, uint64_t seed, int n_replicas,
            void *hip_stream, ka_sim **out);

/* Same with the particle number given directly (0 <= K <= N). */
int ka_init_k(const ka_graph *g, int m, int64_t K, uint64_t seed, int n_replicas,
              void *hip_stream, ka_sim **out);

/* Enqueue n_sweeps sweeps (t -> t + n_sweeps) on the sim's stream; does not synchronise.
 * One sweep applies the exchange of Sec. 2.1 rules (a)-(c) to every edge once per replica,
 * class by class as described at the top of this file; for all 64 replicas of a word at
 * once it is the bitwise update of Sec. 3.2 (thresholds "at most m occupied neighbours
 * other than the partner" on both ends, then the exchange of the two occupations where
 * they differ), masked by the acceptance bits.  The moved-ever mask f gains the bits of
 * both endpoints wherever the exchange happens.  KA_EINVAL if n_sweeps < 0, KA_ESTATE if t
 * would reach 2^32 or the sim is a batch member. */
int ka_sweep(ka_sim *s, int64_t n_sweeps);

/* Per-replica counts at the current t (Sec. 2.2 overlap q_i(t) = n_i(t) n_i(0), summed
 * over sites as in Sec. 3.3): density[b] = sum_i n_i, overlap[b] = sum_i n_i(t) n_i(0),
 * persistence[b] = number of sites occupied at t = 0 whose occupation never changed since.
 * Each output is int64[n_replicas] (any may be NULL); t receives the sweep index.
 * Synchronises the sim's stream. */
int ka_observe(ka_sim *s, int64_t *t, int64_t *density, int64_t *overlap,
               int64_t *persistence);

/* ka_observe for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same counts, accumulated in a
 * fixed device scratch array of the library (3 x 8192 counts, 192 KiB, one per device, held
 * until the process ends) instead of the sim's own observation buffer, which ka_observe
 * allocates on first use.  Calls no hipMalloc or hipFree.  At most 8192 replicas (KA_EINVAL
 * beyond).  Every call on a device shares that scratch: calls that overlap on one device
 * (from several host threads, or on several streams) race and must be serialised by the
 * caller.  The scratch is cleared by a kernel at the start of each call.  Synchronises the
 * sim's stream. */
int ka_observe_noalloc(ka_sim *s, int64_t *t, int64_t *density, int64_t *overlap,
                       int64_t *persistence);

/* Spatial four-point sums at the current t (Sec. 2.2 g4 and chi4 = sum_r g4; Sec. 3.3
 * Phi(r, t) as the popcount of the AND of n_i(t), n_i(0), n_j(t), n_j(0)), with
 * q_i^b = n_i^b(t) n_i^b(0), over ordered site pairs (i, j) grouped in shells r2:
 *   S2[r2]    = sum over pairs in the shell of sum_b q_i^b q_j^b                 (= Phi)
 *   S11[r2]   = sum over pairs in the shell of (sum_b q_i^b) (sum_b q_j^b)
 *   count[r2] = number of partners j of one site i in the shell.
 * Lattices: j = i + delta for every displacement delta of the torus once (components in the
 * minimum image |c| <= L/2), shell r2 = |delta|^2.  Other graphs (random regular, layered,
 * any adjacency): the distance convention of Sec. 3.3 for graphs without a geometry, 0 for
 * j = i and 1 for every j != i, so shell 0 holds the pairs (i, i) (count 1) and shell 1 all
 * others (count N - 1); shells 2.. are 0.
 * Arrays of r2_max + 1 values (any may be NULL); r2_max <= 2048; up to 1024 replicas.
 * g4(r) = (S2/R - S11/R^2) / (N rho^2 (1-rho)^2) (ka_g4) then sums to chi4 over all shells.
 * KA_EINVAL if a sum would not fit int64.  Synchronises. */
int ka_observe_pairs(ka_sim *s, int r2_max, int64_t *S2, int64_t *S11, int64_t *count);

/* Run to each of the n_obs non-decreasing absolute sweep indices obs_times[q] (each >= the
 * current t) and record the counts of ka_observe there into row q of density/overlap/
 * persistence (int64 [n_obs][n_replicas], any may be NULL).  Observations stay on the
 * device until one synchronisation at the end. */
int ka_run(ka_sim *s, const int64_t *obs_times, int n_obs, int64_t *density,
           int64_t *overlap, int64_t *persistence);

/* Copy the state out / in, canonical layout [W][N] each (any output may be NULL).  No
 * passage of the paper applies: this is checkpoint/resume of (n, n(0), f, t); because the
 * random counters hold the absolute sweep t, a run resumed from a copy equals the unbroken
 * run.  ka_set_state requires f to be consistent with the dynamics only for the meaning of
 * persistence; it is not checked.  Both synchronise the stream. */
int ka_get_state(ka_sim *s, uint64_t *n, uint64_t *n0, uint64_t *f, int64_t *t);
int ka_set_state(ka_sim *s, const uint64_t *n, const uint64_t *n0, const uint64_t *f,
                 int64_t t);

/* N, replicas, K, m, current t, number of classes (any may be NULL). */
int ka_sim_info(const ka_sim *s, int64_t *N, int *n_replicas, int64_t *K, int *m,
                int64_t *t, int *n_classes);

/* Options:
 *   KA_OPT_PATH:   0 = automatic, 1 = one kernel per class pass over global memory,
 *                  2 = whole sweep loop inside one workgroup per word plane with the plane in
 *                      LDS (only if it fits; KA_EINVAL otherwise).  Results are identical.
 *   KA_OPT_TIMING: k > 0 brackets every k-th class-pass launch with HIP events on the sim's
 *                  stream (for per-kernel durations, read with ka_timing); 0 = off.
 *   KA_OPT_NOISE:  0 (default) = an independent acceptance bit per replica, edge and sweep;
 *                  1 = shared noise: one bit per (sweep t, class c, edge e) for every replica,
 *                      bit 0 of output word 0 of Philox(t, c, e, 0xFFFFFFFF).  This is the
 *                      paper's multispin step (Sec. 3.2), which applies one random choice to
 *                      all replicas of a word.  Replicas are then coupled: replicas started
 *                      equal stay equal.  Applies to the sweeps that follow.
 *   KA_OPT_PLANE_STREAMS: 0 (default) = every word plane in one launch per class pass on
 *                  the sim's stream; 1 = on the global-memory path, a lattice sim with two
 *                  or more word planes (independent replica chains) runs even planes on one
 *                  stream of its own and odd planes on another, forked from and joined back
 *                  to the sim's stream, so that one plane's pass overlaps the start and end
 *                  of the other's.  The overlap needs the runtime to place the two streams
 *                  on different hardware queues; on a shared queue the passes serialize and
 *                  run slower.  Not used while KA_OPT_TIMING is on.  Results are identical
 *                  either way.
 *   KA_OPT_TAIL:   general graphs on the global-memory path.  1 (default) = when the class
 *                  schedule ends in two or more classes of at most 512 edges each (greedy
 *                  colourings end in a few tiny classes) and one word plane takes at most
 *                  1 MiB (N * 8 * words per thread bytes), that run of classes is one launch
 *                  of one workgroup per word plane, classes in order with a barrier between
 *                  them; 0 = one launch per class.  Results are identical.
 *   KA_OPT_PLANE_GROUPS: the global-memory path.  -1 (default) = the choice made
 *                  at ka_init: when a lattice sim's n and f (16 bytes per site and 64 replicas)
 *                  exceed 256 MiB, its word planes run in groups whose n and f fit 256 MiB
 *                  (the MI355X Infinity Cache), each group through a whole ka_sweep call (or
 *                  the sweeps between two ka_run observations) before the next, so that its
 *                  class passes find n and f in the cache; ka_init then also stores one word
 *                  per plane when a group holds a single word (general graphs: all planes in
 *                  each launch).  0 = every plane in each launch; k >= 1 = groups of k planes
 *                  (lattices and graphs).  Not used while KA_OPT_PLANE_STREAMS is on.
 *                  Results are identical. */
#define KA_OPT_PATH 1
#define KA_OPT_TIMING 2
#define KA_OPT_NOISE 3
#define KA_OPT_PLANE_STREAMS 4
#define KA_OPT_TAIL 5
#define KA_OPT_PLANE_GROUPS 6
int ka_set_option(ka_sim *s, int option, int64_t value);

/* Class-pass kernel launches so far (one per class step, or one per word plane and class
 * step when the planes run on their own streams, or one per group of planes and class step
 * when they run group by group; a merged run of tiny graph classes counts once), and among them the number bracketed by
 * events and their summed duration in milliseconds (synchronises the stream). */
int ka_timing(ka_sim *s, int64_t *launches, int64_t *timed, double *timed_ms);

/* Path a ka_sweep would take now: 1 = global class passes, 2 = LDS-resident. */
int ka_sim_path(const ka_sim *s, int *path);

/* Release a sim.  If the sim is still a batch member, its batch is first run to completion
 * (as ka_batch_wait_all, which detaches every member), so the member's device work never
 * outlives its memory. */
void ka_free(ka_sim *s);

/* ------------------------------------------------------------------------------------ */
/* Batches: many sims advanced together.  One step kernel applies one class pass to every */
/* active member (a solo member, see KA_BOPT_SOLO_BYTES, takes its pass through its own   */
/* kernels in the same step); member k, added at global step s_k with n_k sweeps, runs    */
/* class (s - s_k) mod C_k of its sweep t_k + (s - s_k) / C_k at step s, for              */
/* s_k <= s < s_k + C_k*n_k.  The per-edge arithmetic and random counters are those of    */
/* ka_sweep, so a member ends in exactly the state ka_sweep(n_k) would give it alone.     */
/* Steps advance on the device, so the library replays a captured HIP graph of step       */
/* kernels.                                                                               */
/* ------------------------------------------------------------------------------------ */
typedef struct ka_batch ka_batch;

/* Batch with room for `capacity` members (1..1024), executing on hip_stream (NULL: a
 * stream the library creates).  Members' own streams are ordered before their batch work. */
int ka_batch_create(int capacity, void *hip_stream, ka_batch **out);

/* Add sim s to advance by n_sweeps sweeps, starting at the next step enqueued (or later,
 * under KA_BOPT_CACHE_BUDGET, or for a solo member behind the solo members added before
 * it: see KA_BOPT_SOLO_BYTES).  The sim
 * must be on the batch's device and in no other batch; until it is detached (ka_batch_poll,
 * ka_batch_wait_all) every other call on it returns KA_ESTATE.  *slot receives its slot. */
int ka_batch_add(ka_batch *b, ka_sim *s, int64_t n_sweeps, int *slot);

/* Enqueue n_steps steps (asynchronous).  Each step is one kernel launch per words-per-
 * thread variant present, one workgroup per tile of active work, and the running solo
 * member's own class pass.  The first call tunes the tile (workgroup) size on its first
 * steps unless KA_BOPT_AUTOTUNE is 0. */
int ka_batch_run(ka_batch *b, int64_t n_steps);

/* Steps still to enqueue until every member's work is enqueued. */
int ka_batch_steps_left(const ka_batch *b, int64_t *steps_left);

/* Detach members whose work the device has completed (non-blocking); their slots are
 * written to slots[0..*n_done) (at most max_slots) and their t advanced. */
int ka_batch_poll(ka_batch *b, int *slots, int max_slots, int *n_done);

/* Run every member to completion, wait, and detach all members. */
int ka_batch_wait_all(ka_batch *b);

/* Options: KA_BOPT_AUTOTUNE (1 default / 0), KA_BOPT_BLOCK (tile = workgroup size: 128,
 * 256 or 512; disables autotuning), KA_BOPT_GRAPH_STEPS (steps per captured graph, default
 * 64; 0 = plain launches), KA_BOPT_CACHE_BUDGET (bytes, default 0 = off; set while the batch
 * has no members, else KA_ESTATE): members whose working set (n and f, 2 x 8 x N x n_replicas/64 bytes)
 * is at least 1/8 of the budget are large, and a large member starts only while it fits
 * the budget next to the large members still running (or when none runs); otherwise it
 * waits, in the order added, and starts at the step where enough of them have finished.
 * Sized to the device's last-level cache (256 MiB Infinity Cache on MI355X), this keeps the
 * large members' state cache-resident between steps.  KA_BOPT_SOLO_BYTES (bytes, default
 * 32 MiB; 0 = off; set while the batch has no members, else KA_ESTATE): members whose n and
 * f take at least this many bytes fill the device with their own class passes, so they are
 * solo members: they skip the step kernel, wait in the order added, and run one at a time,
 * each step advancing the running one by one class pass through the pass kernels ka_sweep
 * uses (in its groups of word planes, each group through a run of steps before the next),
 * which keeps its state in the Infinity Cache instead of sharing it with every other
 * member's.  Cache-budget rules apply to the other members only.  A
 * member's result does not depend on when it starts or how it runs; ka_batch_steps_left
 * counts the waiting members' steps too. */
#define KA_BOPT_AUTOTUNE 1
#define KA_BOPT_BLOCK 2
#define KA_BOPT_GRAPH_STEPS 4
#define KA_BOPT_CACHE_BUDGET 5
#define KA_BOPT_SOLO_BYTES 6
int ka_batch_set_option(ka_batch *b, int option, int64_t value);

/* Global step (enqueued), attached members, tile size in use, and tiles per step of the
 * current segment (any may be NULL). */
int ka_batch_info(const ka_batch *b, int64_t *step, int *members, int *block, int *tiles);

/* Finish all members (as ka_batch_wait_all) and release the batch. */
void ka_batch_free(ka_batch *b);

/* ------------------------------------------------------------------------------------ */
/* Serving: a job server with continuous batching.  A worker thread owns one stream and  */
/* one batch; submitted jobs wait in FIFO order until a slot is free and their device    */
/* footprint (ka_footprint) fits the budget, then are initialised on the device and join */
/* the batch, so jobs that arrive while others run share the same step kernels.  A job's */
/* observation times cut it into batch segments; at each one the per-replica counts of   */
/* ka_observe are taken on the device and copied back without stopping the batch.  Each  */
/* job's results are bit-identical to running it alone (same kernels, same counters).    */
/* ------------------------------------------------------------------------------------ */
typedef struct ka_server ka_server;

typedef struct {
  const ka_graph *graph;     /* borrowed: keep it valid until the job is reported done  */
  int m;                     /* activation number                                       */
  double rho;                /* density; K = floor(rho*N + 1/2)                          */
  uint64_t seed;
  int n_replicas;            /* multiple of 64                                          */
  int64_t n_sweeps;          /* total sweeps                                            */
  const int64_t *obs_times;  /* sweep indices in [0, n_sweeps], non-decreasing; copied;  */
  int n_obs;                 /* NULL/0: one observation at n_sweeps                     */
  int keep_sim;              /* 1: keep the final sim for ka_server_take_sim             */
} ka_job_desc;

/* Server with a device-memory budget (bytes) and at most max_active concurrent jobs
 * (1..1024), on hip_stream (NULL: its own stream).  Starts the worker thread. */
int ka_server_create(size_t device_budget, int max_active, void *hip_stream, ka_server **out);

/* Queue a job (thread-safe, non-blocking).  KA_EINVAL if it can never fit the budget. */
int ka_server_submit(ka_server *sv, const ka_job_desc *job, int64_t *job_id);

/* Ids of jobs completed since the last call (at most max_ids; thread-safe). */
int ka_server_poll(ka_server *sv, int64_t *job_ids, int max_ids, int *n);

/* Results of a completed job: counts int64 [n_obs][n_replicas] each (any may be NULL),
 * and seconds from submission to admission and to completion.  KA_ESTATE if not done. */
int ka_server_result(ka_server *sv, int64_t job_id, int64_t *density, int64_t *overlap,
                     int64_t *persistence, double *wait_s, double *latency_s);

/* Hand over the final sim of a completed job submitted with keep_sim; the caller frees it
 * with ka_free.  A kept sim belongs to the caller once its job completes and no longer counts
 * against the budget.  The sim moves to a stream of its own (created by the library), so it may
 * outlive the server and never waits on the server's stream. */
int ka_server_take_sim(ka_server *sv, int64_t job_id, ka_sim **out);

/* Forget a completed job: drop its results and free its kept sim if it was not taken.
 * Completed jobs' results are otherwise kept until ka_server_free.  KA_ESTATE if the job is
 * not complete (or already released). */
int ka_server_release(ka_server *sv, int64_t job_id);

/* Block until every submitted job has completed. */
int ka_server_wait_idle(ka_server *sv);

/* Counters: jobs completed, site-replica attempts completed, peak concurrent jobs, peak
 * device bytes in use (any may be NULL). */
int ka_server_stats(ka_server *sv, int64_t *jobs_done, double *attempts, int *peak_active,
                    size_t *peak_bytes);

/* Stop the worker after the queued jobs complete, and release everything. */
void ka_server_free(ka_server *sv);

/* ------------------------------------------------------------------------------------ */
/* Calibration: integer vector-ALU issue rate of this device, for the rooflines of the    */
/* bit-logic kernels.  kind 0 times chains of 32-bit v_xor_b32, kind 1 chains of           */
/* v_mad_u64_u32 (the 32 x 32 -> 64-bit multiply-add of the Philox rounds), both from      */
/* registers only, `iters` loop iterations per thread over `blocks` workgroups of 256      */
/* threads, on hip_stream (NULL: a stream of its own).  Writes wave-level instructions per */
/* second and lane operations per second (64 per instruction; may be NULL).  Allocates a   */
/* small buffer and synchronises the stream.                                               */
/* ------------------------------------------------------------------------------------ */
int ka_probe_valu(int kind, int iters, int blocks, void *hip_stream, double *instr_per_s,
                  double *lane_ops_per_s);

/* ------------------------------------------------------------------------------------ */
/* Host-side quantities derived from the counts (no device work; callable without a GPU). */
/* ------------------------------------------------------------------------------------ */

/* Particle number of density rho on N sites (Sec. 3.1: the configurations at fixed density
 * rho): K = floor(rho*N + 1/2) in IEEE double, as ka_init uses.  KA_EINVAL if rho is outside
 * [0, 1] or N < 1. */
int ka_particles(int64_t N, double rho, int64_t *K);

/* Replica averages of per-replica counts (Sec. 2.2), one value per row of the int64
 * [n_rows][n_replicas] arrays overlap and persistence (as ka_run returns them), with
 * r = K/N:
 *   q_b  = (overlap_b / N - r^2) / (r (1 - r))          (the overlap normalised so q(0) = 1)
 *   C    = mean_b q_b,   chi4 = N (mean_b q_b^2 - (mean_b q_b)^2)   (population variance)
 *   P    = mean_b persistence_b / K.
 * C and chi4 are NaN when K is 0 or N, P when K is 0.  Outputs double [n_rows] (any may be
 * NULL; persistence may be NULL when P is).  KA_EINVAL on bad sizes. */
int ka_derived(int64_t N, int64_t K, int n_replicas, int n_rows, const int64_t *overlap,
               const int64_t *persistence, double *C, double *chi4, double *P);

/* g4 per shell from the sums of ka_observe_pairs (Sec. 2.2): the replica covariance of the
 * q fields summed over the shell's pairs, normalised by N r^2 (1-r)^2 with r = K/N (the
 * normalisation under which the shells sum to chi4 of ka_derived):
 *   g4[k] = (S2[k] / R - S11[k] / R^2) / (N r^2 (1 - r)^2),   R = n_replicas.
 * NaN when K is 0 or N.  KA_EINVAL on bad sizes. */
int ka_g4(int64_t N, int64_t K, int n_replicas, int n_shells, const int64_t *S2,
          const int64_t *S11, double *g4);

/* Message describing the last error on the calling thread ("" if none). */
const char *ka_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* KA_H */
