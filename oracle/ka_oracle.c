/*
 * ka_oracle.c -- reference ("oracle") implementation of the multispin Kob-Andersen
 * sweep of Boccagna, "A Multispin Algorithm for the Kob-Andersen Stochastic Dynamics on
 * Regular Lattices" (arXiv 1710.05155).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark load.  The
 * product library (libka) shares no source with it and never calls it.
 *
 * Everything here is deliberately plain: one replica at a time, uint8 occupation
 * numbers, explicit neighbour loops, no bit packing, no blocking.  The dynamics is a
 * Markov chain, so there is no closed form to compare against; the oracle executes the
 * same schedule step by step:
 *
 *   for each sweep t, for each edge class c (in increasing c), for each edge e of class c
 *   (in increasing canonical id e), for replica b:
 *       if n_i != n_j and the acceptance bit r(t,c,e,b) is set and
 *          #occupied(N(i)\{j}) <= m and #occupied(N(j)\{i}) <= m
 *       then exchange n_i, n_j and mark both sites as "moved".
 *
 * The exchange rule is the paper's rules (a)-(c) of Sec. 2.1: a particle at i may hop to
 * an empty neighbour j iff i has at most m occupied neighbours (j is empty, so this is
 * the count over N(i)\{j}) and j has at most m+1 occupied neighbours (i is occupied, so
 * this is the count over N(j)\{i} being at most m).  The rule is symmetric in i and j,
 * which is what makes the dynamics reversible (Sec. 2.1, remark after rule (c)).
 *
 * Readings of the paper used here (where it is silent; listed with reasons in the design
 * notes of the repository):
 *   - parallel update of edge classes whose members are at graph distance >= 2, instead
 *     of the paper's random-sequential choice of one pair at a time (Sec. 3.2);
 *   - a per-replica Bernoulli(1/2) acceptance bit from Philox4x32-10 (Salmon et al.,
 *     SC'11), counter (t, c, e, b>>7), key (seed_lo, seed_hi), 64-bit half (b>>6)&1,
 *     bit b&63; the paper lets all N_b replicas share one random pair and has no
 *     acceptance step, which would make the replicas' noise correlated;
 *   - the initial state: the K sites with the smallest keys (u_i, i), u_i drawn from
 *     Philox with counter (0, 0xFFFFFFFF, i, b>>1), half b&1 (a uniform K-subset, i.e.
 *     a uniform sample of the fixed-density configuration space of Sec. 3.1);
 *   - random regular graphs by the configuration model with rejection of the whole
 *     pairing on any self-loop or multi-edge (Sec. 2.1, Bollobas' construction);
 *   - edge classes: on lattices 4*mu + ((x_mu + 2*sum_{nu!=mu} x_nu) mod 4); on general
 *     graphs the greedy distance-2 ("strong") edge colouring in canonical edge order.
 *
 * The paper's own random-sequential algorithm (one random particle and neighbour per
 * attempt) is here too (ko_rs_run), for statistical cross-checks of the class schedule
 * only; no parity test uses it.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11, "Parallel random numbers: as easy  */
/* as 1, 2, 3").  Round: multiply words 0 and 2 by the two Philox multipliers, take the */
/* high halves xor the odd words and the round key, keep the low halves; the key is     */
/* bumped by the two Weyl constants between rounds.                                      */
/* ------------------------------------------------------------------------------------ */
#define KO_PHILOX_M0 0xD2511F53u
#define KO_PHILOX_M1 0xCD9E8D57u
#define KO_WEYL_0 0x9E3779B9u
#define KO_WEYL_1 0xBB67AE85u

void ko_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)KO_PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)KO_PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += KO_WEYL_0;
        k1 += KO_WEYL_1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* n calls; ctr is n*4 words, out is n*4 words. */
void ko_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out)
{
    for (int64_t q = 0; q < n; ++q) ko_philox(ctr + 4 * q, key, out + 4 * q);
}

/* The 64-bit half h (0: out0 | out1<<32, 1: out2 | out3<<32) of Philox(ctr, key). */
static uint64_t ko_philox_half(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                               uint64_t seed, int h)
{
    uint32_t ctr[4] = {c0, c1, c2, c3};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    ko_philox(ctr, key, out);
    if (h == 0) return (uint64_t)out[0] | ((uint64_t)out[1] << 32);
    return (uint64_t)out[2] | ((uint64_t)out[3] << 32);
}

/* ------------------------------------------------------------------------------------ */
/* Hypercubic lattice with periodic boundaries (Sec. 2.1): N = L^d sites, site index     */
/* i = sum_nu x_nu L^nu (x_0 fastest), neighbours x +- e_mu (mod L), z = 2d.             */
/* Edge (x, x+e_mu) has canonical id e = i*d + mu and class                              */
/* 4*mu + ((x_mu + 2*sum_{nu != mu} x_nu) mod 4).                                        */
/* ------------------------------------------------------------------------------------ */
int ko_lattice(int d, int L, int32_t *adj, int32_t *eu, int32_t *ev, int32_t *ecls)
{
    if (d < 1 || d > 3 || L < 4 || L % 4 != 0) return -1;
    int64_t N = 1;
    for (int k = 0; k < d; ++k) N *= L;
    int z = 2 * d;
    for (int64_t i = 0; i < N; ++i) {
        int x[3] = {0, 0, 0};
        int64_t rest = i;
        for (int k = 0; k < d; ++k) { x[k] = (int)(rest % L); rest /= L; }
        for (int mu = 0; mu < d; ++mu) {
            int up[3] = {x[0], x[1], x[2]}, dn[3] = {x[0], x[1], x[2]};
            up[mu] = (x[mu] + 1) % L;
            dn[mu] = (x[mu] + L - 1) % L;
            int64_t iu = 0, id = 0, stride = 1;
            for (int k = 0; k < d; ++k) { iu += up[k] * stride; id += dn[k] * stride; stride *= L; }
            adj[i * z + 2 * mu] = (int32_t)iu;
            adj[i * z + 2 * mu + 1] = (int32_t)id;
            int64_t e = i * d + mu;
            eu[e] = (int32_t)i;
            ev[e] = (int32_t)iu;
            int others = 0;
            for (int nu = 0; nu < d; ++nu) if (nu != mu) others += x[nu];
            ecls[e] = 4 * mu + ((x[mu] + 2 * others) % 4);
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* Random regular graph by the configuration model (Sec. 2.1, Bollobas): N*z stubs,     */
/* stub s belongs to vertex s/z; a uniformly random perfect matching of the stubs is    */
/* drawn by a Fisher-Yates shuffle (k = S-1 down to 1, swap positions k and U[0,k])     */
/* followed by pairing positions (2q, 2q+1).  The whole pairing is rejected if it has a */
/* self-loop or a repeated edge, and a fresh attempt is drawn.                           */
/* Random words of attempt a: word s is output s%4 of Philox with counter               */
/* (a, 0xFFFFFFFE, s/4 low, s/4 high) and key graph_seed.  U[0,k] is Lemire's           */
/* multiply-shift method with rejection (Lemire 2019, "Fast random integer generation  */
/* in an interval").                                                                     */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    uint64_t seed;
    uint32_t attempt;
    uint64_t next;     /* index of the next 32-bit word */
} ko_stream;

static uint32_t ko_stream_word(ko_stream *st)
{
    uint64_t s = st->next++;
    uint32_t ctr[4] = {st->attempt, 0xFFFFFFFEu, (uint32_t)(s / 4), (uint32_t)((s / 4) >> 32)};
    uint32_t key[2] = {(uint32_t)st->seed, (uint32_t)(st->seed >> 32)};
    uint32_t out[4];
    ko_philox(ctr, key, out);
    return out[s % 4];
}

static uint32_t ko_uniform_below(ko_stream *st, uint32_t range)
{
    uint64_t prod = (uint64_t)ko_stream_word(st) * range;
    uint32_t low = (uint32_t)prod;
    if (low < range) {
        uint32_t threshold = (uint32_t)(-range) % range;
        while (low < threshold) {
            prod = (uint64_t)ko_stream_word(st) * range;
            low = (uint32_t)prod;
        }
    }
    return (uint32_t)(prod >> 32);
}

static int ko_cmp_pair(const void *a, const void *b)
{
    const int64_t *p = (const int64_t *)a, *q = (const int64_t *)b;
    if (p[0] != q[0]) return p[0] < q[0] ? -1 : 1;
    if (p[1] != q[1]) return p[1] < q[1] ? -1 : 1;
    return 0;
}

static int ko_cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* adj: N*z, each row sorted ascending.  Returns 0, or -1 on bad arguments, -2 if no
 * simple pairing was found within max_attempts. */
int ko_rrg(int64_t N, int z, uint64_t graph_seed, int64_t max_attempts, int32_t *adj,
           int64_t *attempts_used)
{
    if (N < 2 || z < 1 || z >= N || (N * z) % 2 != 0 || N * z > 0xFFFFFFFFll) return -1;
    int64_t S = N * z;
    int32_t *stub = (int32_t *)malloc(sizeof(int32_t) * S);
    int64_t *pairs = (int64_t *)malloc(sizeof(int64_t) * S);
    int rc = -2;
    for (int64_t a = 0; a < max_attempts; ++a) {
        ko_stream st = {graph_seed, (uint32_t)a, 0};
        for (int64_t s = 0; s < S; ++s) stub[s] = (int32_t)(s / z);
        for (int64_t k = S - 1; k >= 1; --k) {
            int64_t j = ko_uniform_below(&st, (uint32_t)(k + 1));
            int32_t tmp = stub[k]; stub[k] = stub[j]; stub[j] = tmp;
        }
        int ok = 1;
        for (int64_t q = 0; q < S / 2; ++q) {
            int64_t u = stub[2 * q], v = stub[2 * q + 1];
            if (u == v) { ok = 0; break; }
            pairs[2 * q] = u < v ? u : v;
            pairs[2 * q + 1] = u < v ? v : u;
        }
        if (ok) {
            qsort(pairs, (size_t)(S / 2), 2 * sizeof(int64_t), ko_cmp_pair);
            for (int64_t q = 1; q < S / 2; ++q)
                if (pairs[2 * q] == pairs[2 * q - 2] && pairs[2 * q + 1] == pairs[2 * q - 1]) { ok = 0; break; }
        }
        if (!ok) continue;
        int32_t *deg = (int32_t *)calloc((size_t)N, sizeof(int32_t));
        for (int64_t q = 0; q < S / 2; ++q) {
            int64_t u = pairs[2 * q], v = pairs[2 * q + 1];
            adj[u * z + deg[u]++] = (int32_t)v;
            adj[v * z + deg[v]++] = (int32_t)u;
        }
        free(deg);
        for (int64_t i = 0; i < N; ++i) qsort(adj + i * z, (size_t)z, sizeof(int32_t), ko_cmp_i32);
        if (attempts_used) *attempts_used = a + 1;
        rc = 0;
        break;
    }
    free(stub);
    free(pairs);
    return rc;
}

/* ------------------------------------------------------------------------------------ */
/* Canonical edge list of a simple graph: all {u < v}, lexicographic order; e = rank.    */
/* Returns the number of edges (N*z/2), or -1 if adj is not simple (self-loop, repeated  */
/* neighbour, or asymmetric).                                                             */
/* ------------------------------------------------------------------------------------ */
int64_t ko_edges(int64_t N, int z, const int32_t *adj, int32_t *eu, int32_t *ev)
{
    for (int64_t i = 0; i < N; ++i) {
        for (int k = 0; k < z; ++k) {
            int64_t j = adj[i * z + k];
            if (j < 0 || j >= N || j == i) return -1;
            for (int l = 0; l < k; ++l) if (adj[i * z + l] == j) return -1;
            int back = 0;
            for (int l = 0; l < z; ++l) if (adj[j * z + l] == i) back = 1;
            if (!back) return -1;
        }
    }
    int64_t E = 0;
    for (int64_t u = 0; u < N; ++u) {
        int32_t row[64];
        for (int k = 0; k < z; ++k) row[k] = adj[u * z + k];
        qsort(row, (size_t)z, sizeof(int32_t), ko_cmp_i32);
        for (int k = 0; k < z; ++k) {
            if (row[k] > u) { eu[E] = (int32_t)u; ev[E] = row[k]; ++E; }
        }
    }
    return E;
}

/* Greedy distance-2 edge colouring in canonical order: edge e=(u,v) takes the smallest
 * colour not held by an earlier edge that is incident to u, to v, or to a neighbour of
 * u or of v (an edge sharing a vertex with e, or joined to e by an edge).  Two edges of
 * one colour are then at distance >= 2: no endpoint of one is an endpoint of, or adjacent
 * to an endpoint of, the other.  Returns the number of colours. */
int ko_colour(int64_t N, int z, const int32_t *adj, int64_t E, const int32_t *eu,
              const int32_t *ev, int32_t *ecls)
{
    /* incident edge ids per vertex */
    int64_t *inc = (int64_t *)malloc(sizeof(int64_t) * N * z);
    int32_t *deg = (int32_t *)calloc((size_t)N, sizeof(int32_t));
    for (int64_t e = 0; e < E; ++e) {
        inc[(int64_t)eu[e] * z + deg[eu[e]]++] = e;
        inc[(int64_t)ev[e] * z + deg[ev[e]]++] = e;
    }
    int ncol = 0;
    for (int64_t e = 0; e < E; ++e) {
        uint8_t used[1024];
        memset(used, 0, sizeof(used));
        int64_t verts[2 + 2 * 64];
        int nv = 0;
        verts[nv++] = eu[e];
        verts[nv++] = ev[e];
        for (int k = 0; k < z; ++k) verts[nv++] = adj[(int64_t)eu[e] * z + k];
        for (int k = 0; k < z; ++k) verts[nv++] = adj[(int64_t)ev[e] * z + k];
        for (int q = 0; q < nv; ++q) {
            int64_t x = verts[q];
            for (int k = 0; k < deg[x]; ++k) {
                int64_t f = inc[x * z + k];
                if (f < e) used[ecls[f]] = 1;
            }
        }
        int c = 0;
        while (used[c]) ++c;
        ecls[e] = c;
        if (c + 1 > ncol) ncol = c + 1;
    }
    free(inc);
    free(deg);
    return ncol;
}

/* ------------------------------------------------------------------------------------ */
/* Initial state of replica b (Sec. 3.1, "select omega in Omega_{N,rho} at random"):     */
/* the K sites with the smallest keys (u_i, i) are occupied, where u_i is half b&1 of    */
/* Philox(counter (0, 0xFFFFFFFF, i, b>>1), key seed).                                   */
/* ------------------------------------------------------------------------------------ */
void ko_init_replica(int64_t N, int64_t K, uint64_t seed, int64_t b, uint8_t *occ)
{
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * 2 * N);
    for (int64_t i = 0; i < N; ++i) {
        uint64_t u = ko_philox_half(0u, 0xFFFFFFFFu, (uint32_t)i, (uint32_t)(b >> 1), seed, (int)(b & 1));
        /* order by unsigned u: flip the sign bit so that signed comparison agrees */
        keys[2 * i] = (int64_t)(u ^ 0x8000000000000000ull);
        keys[2 * i + 1] = i;
    }
    qsort(keys, (size_t)N, 2 * sizeof(int64_t), ko_cmp_pair);
    memset(occ, 0, (size_t)N);
    for (int64_t k = 0; k < K; ++k) occ[keys[2 * k + 1]] = 1;
    free(keys);
}

/* ------------------------------------------------------------------------------------ */
/* The exchange rule for one edge (i, j) of one replica (Sec. 2.1 rules (a)-(c)).        */
/* ni, nj: occupations of the endpoints; nbr_i: the z-1 occupations of N(i)\{j};          */
/* nbr_j: those of N(j)\{i}; r: acceptance bit.  Writes the new occupations.             */
/* ------------------------------------------------------------------------------------ */
void ko_exchange(int z, int m, int ni, int nj, const uint8_t *nbr_i, const uint8_t *nbr_j,
                 int r, int *ni_out, int *nj_out)
{
    *ni_out = ni;
    *nj_out = nj;
    if (ni == nj || !r) return;
    int count_i = 0, count_j = 0;
    for (int k = 0; k < z - 1; ++k) { count_i += nbr_i[k]; count_j += nbr_j[k]; }
    if (count_i <= m && count_j <= m) {
        *ni_out = nj;
        *nj_out = ni;
    }
}

/* One edge of one replica, in place on occ/moved (length N). */
static void ko_edge(int z, int m, const int32_t *adj, int64_t i, int64_t j, int r,
                    uint8_t *occ, uint8_t *moved)
{
    uint8_t nbr_i[64], nbr_j[64];
    int qi = 0, qj = 0;
    for (int k = 0; k < z; ++k) {
        int64_t a = adj[i * z + k];
        if (a != j) nbr_i[qi++] = occ[a];
        int64_t b = adj[j * z + k];
        if (b != i) nbr_j[qj++] = occ[b];
    }
    int ni, nj;
    ko_exchange(z, m, occ[i], occ[j], nbr_i, nbr_j, r, &ni, &nj);
    if (ni != occ[i]) {
        occ[i] = (uint8_t)ni;
        occ[j] = (uint8_t)nj;
        moved[i] = 1;
        moved[j] = 1;
    }
}

/* One pass over class c for R independent states with explicit acceptance bits
 * accept[r*E + e]; occ and moved are R*N. */
void ko_pass(int64_t N, int z, const int32_t *adj, int64_t E, const int32_t *eu,
             const int32_t *ev, const int32_t *ecls, int c, int m, int64_t R, uint8_t *occ,
             uint8_t *moved, const uint8_t *accept)
{
    for (int64_t r = 0; r < R; ++r)
        for (int64_t e = 0; e < E; ++e)
            if (ecls[e] == c)
                ko_edge(z, m, adj, eu[e], ev[e], accept[r * E + e], occ + r * N, moved + r * N);
}

/* The acceptance bit of replica b for edge e of class c in sweep t. */
int ko_accept_bit(uint64_t seed, int64_t t, int c, int64_t e, int64_t b)
{
    uint64_t half = ko_philox_half((uint32_t)t, (uint32_t)c, (uint32_t)e, (uint32_t)(b >> 7),
                                   seed, (int)((b >> 6) & 1));
    return (int)((half >> (b & 63)) & 1);
}

/* Shared-noise variant (the paper's multispin step applies one random choice to every
 * replica of a word, Sec. 3.2): one acceptance bit per (sweep t, class c, edge e) common to
 * all replicas, bit 0 of output word 0 of Philox(t, c, e, 0xFFFFFFFF). */
int ko_accept_bit_shared(uint64_t seed, int64_t t, int c, int64_t e)
{
    uint64_t half = ko_philox_half((uint32_t)t, (uint32_t)c, (uint32_t)e, 0xFFFFFFFFu, seed, 0);
    return (int)(half & 1);
}

/* n_sweeps sweeps (t = t0 .. t0+n_sweeps-1) of the replicas listed in reps[0..nrep-1];
 * occ and moved are nrep*N, row q belonging to replica reps[q].  Classes are visited in
 * increasing c, edges of a class in increasing canonical id.  shared selects the
 * shared-noise acceptance bits.  Each replica's run reads only its own row and the
 * (deterministic) bits, so replicas are distributed over threads. */
void ko_run(int64_t N, int z, const int32_t *adj, int64_t E, const int32_t *eu,
            const int32_t *ev, const int32_t *ecls, int C, int m, uint64_t seed, int64_t nrep,
            const int64_t *reps, int64_t t0, int64_t n_sweeps, uint8_t *occ, uint8_t *moved,
            int shared)
{
    /* edges bucketed by class, each bucket in increasing e */
    int64_t *start = (int64_t *)calloc((size_t)C + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (E > 0 ? E : 1));
    for (int64_t e = 0; e < E; ++e) start[ecls[e] + 1]++;
    for (int c = 0; c < C; ++c) start[c + 1] += start[c];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * ((size_t)C + 1));
    memcpy(fill, start, sizeof(int64_t) * ((size_t)C + 1));
    for (int64_t e = 0; e < E; ++e) order[fill[ecls[e]]++] = e;
    free(fill);

#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrep; ++q) {
        int64_t b = reps[q];
        uint8_t *o = occ + q * N, *mv = moved + q * N;
        for (int64_t t = t0; t < t0 + n_sweeps; ++t)
            for (int c = 0; c < C; ++c)
                for (int64_t k = start[c]; k < start[c + 1]; ++k) {
                    int64_t e = order[k];
                    int r = shared ? ko_accept_bit_shared(seed, t, c, e)
                                   : ko_accept_bit(seed, t, c, e, b);
                    if (r) ko_edge(z, m, adj, eu[e], ev[e], r, o, mv);
                }
    }
    free(start);
    free(order);
}

/* Number of threads an OpenMP parallel region would use (for reporting). */
int ko_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------------------ */
/* Random-sequential dynamics: the paper's own algorithm (Sec. 2.1), kept for            */
/* statistical cross-checks of the class schedule, never for parity.  One attempt picks  */
/* a particle uniformly among the K, then one of its z neighbours uniformly; the particle */
/* at i moves to j iff (a) j is empty, (b) i has at most m occupied neighbours and (c) j  */
/* has at most m+1 occupied neighbours (i, occupied, counted among them).                */
/* Attempt a of replica b draws Philox with counter (b, 0xFFFFFFFC, a low, a high) and    */
/* key seed: words 0|1<<32 choose the particle, words 2|3<<32 the neighbour slot, each by */
/* the multiply-shift floor(u * range / 2^64) of the 64-bit word (bias below range/2^64). */
/* The particle with index p is the p-th occupied site in increasing site order, so a     */
/* run split into several calls draws the same moves as one call.                         */
/* ------------------------------------------------------------------------------------ */

/* Target site of the attempt "particle at i, neighbour slot k" in occ, or -1 if the move
 * is not allowed (or i is empty). */
int64_t ko_rs_target(int z, int m, const int32_t *adj, const uint8_t *occ, int64_t i, int k)
{
    if (!occ[i]) return -1;
    int64_t j = adj[i * z + k];
    if (occ[j]) return -1;                                   /* (a) */
    int count_i = 0, count_j = 0;
    for (int q = 0; q < z; ++q) {
        count_i += occ[adj[i * z + q]];
        count_j += occ[adj[j * z + q]];
    }
    return (count_i <= m && count_j <= m + 1) ? j : -1;     /* (b), (c) */
}

/* ko_rs_target for every state row (n_states x N), site i and slot k: out is
 * n_states x N x z. */
void ko_rs_targets(int64_t N, int z, const int32_t *adj, int m, int64_t n_states,
                   const uint8_t *occ, int64_t *out)
{
    for (int64_t s = 0; s < n_states; ++s)
        for (int64_t i = 0; i < N; ++i)
            for (int k = 0; k < z; ++k)
                out[(s * N + i) * z + k] = ko_rs_target(z, m, adj, occ + s * N, i, k);
}

static uint64_t ko_rs_pick(uint32_t lo, uint32_t hi, uint64_t range)
{
    unsigned __int128 u = (unsigned __int128)(((uint64_t)hi << 32) | lo);
    return (uint64_t)((u * range) >> 64);
}

/* Attempts a0 .. a0+n_attempts-1 of the replicas reps[0..nrep-1]; occ and moved are
 * nrep*N, row q belonging to replica reps[q].  Every row must hold K >= 1 particles. */
void ko_rs_run(int64_t N, int z, const int32_t *adj, int m, uint64_t seed, int64_t nrep,
               const int64_t *reps, uint64_t a0, uint64_t n_attempts, uint8_t *occ,
               uint8_t *moved)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < nrep; ++q) {
        uint8_t *o = occ + q * N, *mv = moved + q * N;
        /* occupied sites in increasing order */
        int64_t *part = (int64_t *)malloc(sizeof(int64_t) * (N > 0 ? N : 1));
        int64_t K = 0;
        for (int64_t i = 0; i < N; ++i)
            if (o[i]) part[K++] = i;
        uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
        for (uint64_t a = a0; K > 0 && a < a0 + n_attempts; ++a) {
            uint32_t ctr[4] = {(uint32_t)reps[q], 0xFFFFFFFCu, (uint32_t)a, (uint32_t)(a >> 32)};
            uint32_t w[4];
            ko_philox(ctr, key, w);
            int64_t p = (int64_t)ko_rs_pick(w[0], w[1], (uint64_t)K);
            int k = (int)ko_rs_pick(w[2], w[3], (uint64_t)z);
            int64_t i = part[p];
            int64_t j = ko_rs_target(z, m, adj, o, i, k);
            if (j < 0) continue;
            o[i] = 0;
            o[j] = 1;
            mv[i] = 1;
            mv[j] = 1;
            /* keep part sorted: drop i at position p, insert j */
            memmove(part + p, part + p + 1, sizeof(int64_t) * (size_t)(K - 1 - p));
            int64_t pos = 0;
            while (pos < K - 1 && part[pos] < j) ++pos;
            memmove(part + pos + 1, part + pos, sizeof(int64_t) * (size_t)(K - 1 - pos));
            part[pos] = j;
        }
        free(part);
    }
}

/* ------------------------------------------------------------------------------------ */
/* Layered random graph (Sec. 5.2): M copies of the periodic lattice Z_L^d; for every     */
/* bond (x, x+e_mu) of the base lattice the M links (x, a)-(x+e_mu, a) are replaced by    */
/* (x, a)-(x+e_mu, P(a)) with P a uniformly random permutation of the M copies, drawn     */
/* independently for every bond.  Vertex (x, a) has id a*N + i(x).  P for the bond with   */
/* base edge id e = i*d + mu is a Fisher-Yates shuffle (k = M-1 down to 1, swap k and      */
/* U[0,k]) of 0..M-1 driven by the words of Philox with counter (e, 0xFFFFFFFD, s/4, 0),  */
/* word s = output s%4, key graph_seed, with Lemire's method for U[0,k].                  */
/* Rows of adj are sorted ascending.  base_class[v*z + k] receives the lattice class of   */
/* the bond that carries the k-th (sorted) neighbour link of v.                           */
/* ------------------------------------------------------------------------------------ */
static uint32_t ko_bond_word(uint64_t seed, uint32_t e, uint64_t s)
{
    uint32_t ctr[4] = {e, 0xFFFFFFFDu, (uint32_t)(s / 4), 0u};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    ko_philox(ctr, key, out);
    return out[s % 4];
}

static uint32_t ko_bond_below(uint64_t seed, uint32_t e, uint64_t *s, uint32_t range)
{
    uint64_t prod = (uint64_t)ko_bond_word(seed, e, (*s)++) * range;
    uint32_t low = (uint32_t)prod;
    if (low < range) {
        uint32_t threshold = (uint32_t)(-range) % range;
        while (low < threshold) {
            prod = (uint64_t)ko_bond_word(seed, e, (*s)++) * range;
            low = (uint32_t)prod;
        }
    }
    return (uint32_t)(prod >> 32);
}

int ko_layered(int d, int L, int M, uint64_t seed, int32_t *adj)
{
    if (d < 2 || d > 3 || L < 3 || M < 1) return -1;
    int64_t N = 1;
    for (int k = 0; k < d; ++k) N *= L;
    int z = 2 * d;
    int32_t *eu = (int32_t *)malloc(sizeof(int32_t) * N * d);
    int32_t *ev = (int32_t *)malloc(sizeof(int32_t) * N * d);
    /* the bonds of the base lattice (any L >= 3 gives distinct neighbours) */
    for (int64_t i = 0; i < N; ++i) {
        int x[3] = {0, 0, 0};
        int64_t rest = i;
        for (int k = 0; k < d; ++k) { x[k] = (int)(rest % L); rest /= L; }
        for (int mu = 0; mu < d; ++mu) {
            int up[3] = {x[0], x[1], x[2]};
            up[mu] = (x[mu] + 1) % L;
            int64_t iu = 0, stride = 1;
            for (int k = 0; k < d; ++k) { iu += up[k] * stride; stride *= L; }
            eu[i * d + mu] = (int32_t)i;
            ev[i * d + mu] = (int32_t)iu;
        }
    }
    int32_t *fill = (int32_t *)calloc((size_t)(N * M), sizeof(int32_t));
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * M);
    for (int64_t e = 0; e < N * d; ++e) {
        for (int a = 0; a < M; ++a) perm[a] = a;
        uint64_t s = 0;
        for (int k = M - 1; k >= 1; --k) {
            uint32_t j = ko_bond_below(seed, (uint32_t)e, &s, (uint32_t)(k + 1));
            int32_t t = perm[k]; perm[k] = perm[j]; perm[j] = t;
        }
        for (int a = 0; a < M; ++a) {
            int64_t u = (int64_t)a * N + eu[e];
            int64_t v = (int64_t)perm[a] * N + ev[e];
            adj[u * z + fill[u]++] = (int32_t)v;
            adj[v * z + fill[v]++] = (int32_t)u;
        }
    }
    for (int64_t v = 0; v < N * M; ++v) qsort(adj + v * z, (size_t)z, sizeof(int32_t), ko_cmp_i32);
    free(eu); free(ev); free(fill); free(perm);
    return 0;
}

/* Class of each canonical edge of a layered graph by projection to the base lattice:
 * the class of the base bond joining the two endpoints' sites (valid when L % 4 == 0). */
void ko_layered_classes(int d, int L, int64_t N, int64_t E, const int32_t *eu, const int32_t *ev,
                        int32_t *ecls)
{
    for (int64_t q = 0; q < E; ++q) {
        int64_t iu = eu[q] % N, iv = ev[q] % N;
        int xu[3] = {0, 0, 0}, xv[3] = {0, 0, 0};
        int64_t ru = iu, rv = iv;
        for (int k = 0; k < d; ++k) { xu[k] = (int)(ru % L); ru /= L; xv[k] = (int)(rv % L); rv /= L; }
        int mu = 0;
        for (int k = 0; k < d; ++k) if (xu[k] != xv[k]) mu = k;
        /* the lower endpoint of the bond is the one whose +e_mu neighbour is the other */
        const int *lo = ((xu[mu] + 1) % L == xv[mu]) ? xu : xv;
        int others = 0;
        for (int nu = 0; nu < d; ++nu) if (nu != mu) others += lo[nu];
        ecls[q] = 4 * mu + ((lo[mu] + 2 * others) % 4);
    }
}
