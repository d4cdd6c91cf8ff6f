// ka_host.cpp -- host side of libka: graphs, edge classes, device state, kernel dispatch.
//
// Method: Boccagna, arXiv 1710.05155 (Sec. 2.1 model and graphs, Sec. 3 multispin
// algorithm).  The C ABI is declared and documented in include/ka.h.
#include "ka.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "ka_internal.h"
#include "ka_objects.h"

using ka::u64;

namespace {

thread_local std::string g_err;

}  // namespace

void ka_set_error(const char *msg) { g_err = msg; }

namespace {

int fail(int code, const char *fmt, ...)
{
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char *what)
{
  return fail(KA_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

// ------------------------------------------------------------------------------------
// Philox4x32-10 on the host (Salmon et al., SC'11), for the random regular graph builder.
// ------------------------------------------------------------------------------------
void philox_host(const uint32_t in[4], uint64_t seed, uint32_t out[4])
{
  uint32_t c0 = in[0], c1 = in[1], c2 = in[2], c3 = in[3];
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    c1 = (uint32_t)p1;
    c3 = (uint32_t)p0;
    c0 = n0;
    c2 = n2;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

// 32-bit words of one configuration-model attempt, buffered four at a time.
class WordStream {
 public:
  WordStream(uint64_t seed, uint32_t attempt) : seed_(seed), attempt_(attempt) {}
  uint32_t next()
  {
    if (have_ == 0) {
      const uint32_t ctr[4] = {attempt_, 0xFFFFFFFEu, (uint32_t)block_, (uint32_t)(block_ >> 32)};
      philox_host(ctr, seed_, buf_);
      ++block_;
      have_ = 4;
    }
    return buf_[4 - have_--];
  }
  // Uniform integer in [0, range) by Lemire's multiply-shift method with rejection.
  uint32_t below(uint32_t range)
  {
    uint64_t prod = (uint64_t)next() * range;
    uint32_t low = (uint32_t)prod;
    if (low < range) {
      const uint32_t thresh = (uint32_t)(0u - range) % range;
      while (low < thresh) {
        prod = (uint64_t)next() * range;
        low = (uint32_t)prod;
      }
    }
    return (uint32_t)(prod >> 32);
  }

 private:
  uint64_t seed_;
  uint32_t attempt_;
  uint64_t block_ = 0;
  uint32_t buf_[4];
  int have_ = 0;
};

}  // namespace

// ----------------------------------------------------------------------------------------
// Graph
// ----------------------------------------------------------------------------------------

namespace {

// Greedy distance-2 edge colouring in canonical edge order: each edge takes the smallest
// colour not held by an earlier edge incident to an endpoint or to a neighbour of an
// endpoint.  Same-colour edges are then at distance >= 2, so they can be updated at once.
int colour_edges(ka_graph &g)
{
  const int64_t E = (int64_t)g.eu.size();
  std::vector<int64_t> inc((size_t)g.N * g.z, -1);
  std::vector<int> fill((size_t)g.N, 0);
  for (int64_t e = 0; e < E; ++e) {
    inc[(size_t)g.eu[e] * g.z + fill[g.eu[e]]++] = e;
    inc[(size_t)g.ev[e] * g.z + fill[g.ev[e]]++] = e;
  }
  g.ecls.assign((size_t)E, 0);
  int ncol = 0;
  std::vector<int32_t> verts;
  for (int64_t e = 0; e < E; ++e) {
    uint64_t used[4] = {0, 0, 0, 0};
    verts.clear();
    verts.push_back(g.eu[e]);
    verts.push_back(g.ev[e]);
    for (int k = 0; k < g.z; ++k) verts.push_back(g.adj[(size_t)g.eu[e] * g.z + k]);
    for (int k = 0; k < g.z; ++k) verts.push_back(g.adj[(size_t)g.ev[e] * g.z + k]);
    for (int32_t x : verts)
      for (int k = 0; k < g.z; ++k) {
        const int64_t f = inc[(size_t)x * g.z + k];
        if (f >= 0 && f < e) used[g.ecls[f] >> 6] |= 1ull << (g.ecls[f] & 63);
      }
    int c = 0;
    while (c < 256 && ((used[c >> 6] >> (c & 63)) & 1ull)) ++c;
    if (c >= 256) return -1;
    g.ecls[e] = c;
    ncol = std::max(ncol, c + 1);
  }
  g.C = ncol;
  return 0;
}

// Validate a z-regular simple adjacency, then build canonical edges and classes.
int finish_general_graph(ka_graph &g)
{
  for (int64_t i = 0; i < g.N; ++i) {
    const int32_t *row = &g.adj[(size_t)i * g.z];
    for (int k = 0; k < g.z; ++k) {
      const int64_t j = row[k];
      if (j < 0 || j >= g.N) return fail(KA_EINVAL, "adjacency entry out of range at vertex %lld", (long long)i);
      if (j == i) return fail(KA_EINVAL, "self-loop at vertex %lld", (long long)i);
      for (int l = 0; l < k; ++l)
        if (row[l] == j) return fail(KA_EINVAL, "repeated neighbour at vertex %lld", (long long)i);
      const int32_t *back = &g.adj[(size_t)j * g.z];
      if (std::find(back, back + g.z, (int32_t)i) == back + g.z)
        return fail(KA_EINVAL, "adjacency not symmetric at edge (%lld, %lld)", (long long)i, (long long)j);
    }
  }
  g.eu.clear();
  g.ev.clear();
  g.eu.reserve((size_t)(g.N * g.z / 2));
  g.ev.reserve((size_t)(g.N * g.z / 2));
  std::vector<int32_t> row((size_t)g.z);
  for (int64_t u = 0; u < g.N; ++u) {
    std::copy(&g.adj[(size_t)u * g.z], &g.adj[(size_t)u * g.z] + g.z, row.begin());
    std::sort(row.begin(), row.end());
    for (int32_t v : row)
      if (v > u) {
        g.eu.push_back((int32_t)u);
        g.ev.push_back(v);
      }
  }
  if (colour_edges(g) != 0) return fail(KA_EINVAL, "edge colouring needs more than 256 classes");
  return KA_OK;
}

}  // namespace

extern "C" int ka_graph_lattice(int d, int L, ka_graph **out)
{
  return ka_guard([&]() -> int {
    if (!out) return fail(KA_EINVAL, "out is NULL");
    *out = nullptr;
    if (d != 2 && d != 3) return fail(KA_EINVAL, "lattice dimension must be 2 or 3 (got %d)", d);
    if (L < 4 || L % 4 != 0) return fail(KA_EINVAL, "lattice side must be a multiple of 4, >= 4 (got %d)", L);
    int64_t N = 1;
    for (int k = 0; k < d; ++k) N *= L;
    if (N > (1ll << 30)) return fail(KA_EINVAL, "lattice too large (N = %lld > 2^30)", (long long)N);
    ka_graph *g = new (std::nothrow) ka_graph;
    if (!g) return fail(KA_ENOMEM, "host allocation failed");
    g->lattice = 1;
    g->d = d;
    g->L = L;
    g->N = N;
    g->z = 2 * d;
    g->C = 4 * d;
    // The explicit adjacency and edge lists of a lattice are written on export only: the
    // kernels compute neighbours and classes from coordinates.
    *out = g;
    return KA_OK;
  });
}

namespace {

// Adjacency [N][2d] (x+e_mu, x-e_mu per direction), canonical edges e = i*d + mu of
// (x, x+e_mu) and their classes 4 mu + ((x_mu + 2 sum_{nu != mu} x_nu) mod 4); any output may
// be NULL.
void lattice_export(const ka_graph *g, int32_t *adj, int32_t *eu, int32_t *ev, int32_t *ecls)
{
  const int d = g->d, L = g->L, z = g->z;
  const int64_t N = g->N;
  const int64_t stride[3] = {1, L, (int64_t)L * L};
  for (int64_t i = 0; i < N; ++i) {
    int x[3] = {0, 0, 0};
    for (int k = 0; k < d; ++k) x[k] = (int)((i / stride[k]) % L);
    const int others_all = x[0] + x[1] + x[2];
    for (int mu = 0; mu < d; ++mu) {
      const int64_t up = i + (x[mu] + 1 < L ? stride[mu] : -(int64_t)(L - 1) * stride[mu]);
      const int64_t dn = i + (x[mu] > 0 ? -stride[mu] : (int64_t)(L - 1) * stride[mu]);
      if (adj) {
        adj[(size_t)i * z + 2 * mu] = (int32_t)up;
        adj[(size_t)i * z + 2 * mu + 1] = (int32_t)dn;
      }
      const int64_t e = i * d + mu;
      if (eu) eu[e] = (int32_t)i;
      if (ev) ev[e] = (int32_t)up;
      if (ecls) ecls[e] = 4 * mu + ((x[mu] + 2 * (others_all - x[mu])) & 3);
    }
  }
}

}  // namespace

extern "C" int ka_graph_rrg(int64_t N, int z, uint64_t graph_seed, ka_graph **out)
{
  return ka_guard([&]() -> int {
    if (!out) return fail(KA_EINVAL, "out is NULL");
    *out = nullptr;
    if (z < 3 || z > 6) return fail(KA_EINVAL, "degree z must be in [3, 6] (got %d)", z);
    if (N <= z || N > (1ll << 28) || (N * z) % 2 != 0)
      return fail(KA_EINVAL, "need z < N <= 2^28 and N*z even (N = %lld, z = %d)", (long long)N, z);
    ka_graph *g = new (std::nothrow) ka_graph;
    if (!g) return fail(KA_ENOMEM, "host allocation failed");
    g->N = N;
    g->z = z;
    const int64_t S = N * z;
    std::vector<int32_t> stub, deg;
    try {
      stub.resize((size_t)S);
      deg.resize((size_t)N);
      g->adj.resize((size_t)S);
    } catch (...) {
      delete g;
      return fail(KA_ENOMEM, "host allocation failed");
    }
    int32_t *adj = g->adj.data();
    // Adds the edge (u, v) unless it is a self-loop or already present.
    auto add_pair = [&](int32_t u, int32_t v) -> bool {
      if (u == v) return false;
      const int32_t *ru = adj + (size_t)u * z;
      for (int k = 0; k < deg[u]; ++k)
        if (ru[k] == v) return false;
      adj[(size_t)u * z + deg[u]++] = v;
      adj[(size_t)v * z + deg[v]++] = u;
      return true;
    };
    bool found = false;
    const int64_t max_attempts = 1000000;
    for (int64_t a = 0; a < max_attempts && !found; ++a) {
      WordStream ws(graph_seed, (uint32_t)a);
      for (int64_t s = 0; s < S; ++s) stub[(size_t)s] = (int32_t)(s / z);
      std::fill(deg.begin(), deg.end(), 0);
      bool ok = true;
      // Fisher-Yates from the top: after step k, positions k..S-1 are final, so the pair
      // (2q, 2q+1) is known after step 2q and a bad pair ends the attempt early.  The
      // attempt's random words do not depend on earlier attempts, so the accepted pairing
      // is the same as with a complete shuffle followed by a check.
      for (int64_t k = S - 1; k >= 1; --k) {
        const int64_t j = ws.below((uint32_t)(k + 1));
        std::swap(stub[(size_t)k], stub[(size_t)j]);
        if ((k & 1) == 0 && !add_pair(stub[(size_t)k], stub[(size_t)k + 1])) {
          ok = false;
          break;
        }
      }
      if (ok && !add_pair(stub[0], stub[1])) ok = false;
      found = ok;
    }
    if (!found) {
      delete g;
      return fail(KA_ESTATE, "no simple pairing within %lld attempts", (long long)max_attempts);
    }
    for (int64_t i = 0; i < N; ++i) std::sort(adj + (size_t)i * z, adj + (size_t)i * z + z);
    int rc = finish_general_graph(*g);
    if (rc != KA_OK) {
      delete g;
      return rc;
    }
    *out = g;
    return KA_OK;
  });
}

extern "C" int ka_graph_layered(int d, int L, int M, uint64_t graph_seed, ka_graph **out)
{
  return ka_guard([&]() -> int {
    if (!out) return fail(KA_EINVAL, "out is NULL");
    *out = nullptr;
    if (d != 2 && d != 3) return fail(KA_EINVAL, "lattice dimension must be 2 or 3 (got %d)", d);
    if (L < 3) return fail(KA_EINVAL, "lattice side must be >= 3 (got %d)", L);
    if (M < 1) return fail(KA_EINVAL, "number of copies must be >= 1 (got %d)", M);
    int64_t Nb = 1;
    for (int k = 0; k < d; ++k) Nb *= L;
    if (Nb * M > (1ll << 28)) return fail(KA_EINVAL, "layered graph too large (%lld sites)", (long long)(Nb * M));
    ka_graph *g = new (std::nothrow) ka_graph;
    if (!g) return fail(KA_ENOMEM, "host allocation failed");
    const int z = 2 * d;
    g->N = Nb * M;
    g->z = z;
    try {
      g->adj.resize((size_t)g->N * z);
    } catch (...) {
      delete g;
      return fail(KA_ENOMEM, "host allocation failed");
    }
    const int64_t stride[3] = {1, L, (int64_t)L * L};
    std::vector<int> fill((size_t)g->N, 0);
    std::vector<int32_t> perm((size_t)M);
    for (int64_t i = 0; i < Nb; ++i) {
      for (int mu = 0; mu < d; ++mu) {
        const int x_mu = (int)((i / stride[mu]) % L);
        const int64_t j = i + (x_mu + 1 < L ? stride[mu] : -(int64_t)(L - 1) * stride[mu]);
        // permutation of the M copies for this bond (base edge id i*d + mu)
        const uint64_t e = (uint64_t)(i * d + mu);
        uint32_t words[4];
        uint64_t next = 0, block = UINT64_MAX;
        auto word = [&]() -> uint32_t {
          const uint64_t q = next / 4;
          if (q != block) {
            const uint32_t ctr[4] = {(uint32_t)e, 0xFFFFFFFDu, (uint32_t)q, 0u};
            philox_host(ctr, graph_seed, words);
            block = q;
          }
          return words[next++ % 4];
        };
        auto below = [&](uint32_t range) -> uint32_t {  // Lemire's multiply-shift with rejection
          uint64_t prod = (uint64_t)word() * range;
          uint32_t low = (uint32_t)prod;
          if (low < range) {
            const uint32_t thresh = (uint32_t)(0u - range) % range;
            while (low < thresh) {
              prod = (uint64_t)word() * range;
              low = (uint32_t)prod;
            }
          }
          return (uint32_t)(prod >> 32);
        };
        for (int a = 0; a < M; ++a) perm[(size_t)a] = a;
        for (int k = M - 1; k >= 1; --k) std::swap(perm[(size_t)k], perm[below((uint32_t)(k + 1))]);
        for (int a = 0; a < M; ++a) {
          const int64_t u = (int64_t)a * Nb + i, v = (int64_t)perm[(size_t)a] * Nb + j;
          g->adj[(size_t)u * z + fill[(size_t)u]++] = (int32_t)v;
          g->adj[(size_t)v * z + fill[(size_t)v]++] = (int32_t)u;
        }
      }
    }
    for (int64_t v = 0; v < g->N; ++v) std::sort(&g->adj[(size_t)v * z], &g->adj[(size_t)v * z] + z);
    int rc = finish_general_graph(*g);
    if (rc != KA_OK) {
      delete g;
      return rc;
    }
    if (L % 4 == 0) {
      // Classes by projection to the lattice: an edge takes the class of the bond it lifts.
      // Projection maps edges to edges, so distances can only shrink under it; two lifts of
      // one bond share no site and no link.  The lattice classes therefore stay valid.
      for (size_t q = 0; q < g->eu.size(); ++q) {
        const int64_t iu = g->eu[q] % Nb, iv = g->ev[q] % Nb;
        int mu = 0;
        for (int k = 0; k < d; ++k)
          if ((iu / stride[k]) % L != (iv / stride[k]) % L) mu = k;
        const int64_t xu = (iu / stride[mu]) % L;
        const int64_t lo = ((xu + 1) % L == (iv / stride[mu]) % L) ? iu : iv;
        int others = 0;
        for (int k = 0; k < d; ++k)
          if (k != mu) others += (int)((lo / stride[k]) % L);
        g->ecls[q] = 4 * mu + (int)((((lo / stride[mu]) % L) + 2 * others) & 3);
      }
      g->C = 4 * d;
    }
    *out = g;
    return KA_OK;
  });
}

extern "C" int ka_graph_from_adjacency(int64_t N, int z, const int32_t *adj, ka_graph **out)
{
  return ka_guard([&]() -> int {
    if (!out || !adj) return fail(KA_EINVAL, "NULL argument");
    *out = nullptr;
    if (z < 3 || z > 6) return fail(KA_EINVAL, "degree z must be in [3, 6] (got %d)", z);
    if (N <= z || N > (1ll << 28)) return fail(KA_EINVAL, "need z < N <= 2^28 (N = %lld)", (long long)N);
    ka_graph *g = new (std::nothrow) ka_graph;
    if (!g) return fail(KA_ENOMEM, "host allocation failed");
    g->N = N;
    g->z = z;
    try {
      g->adj.assign(adj, adj + (size_t)N * z);
    } catch (...) {
      delete g;
      return fail(KA_ENOMEM, "host allocation failed");
    }
    int rc = finish_general_graph(*g);
    if (rc != KA_OK) {
      delete g;
      return rc;
    }
    *out = g;
    return KA_OK;
  });
}

extern "C" int ka_graph_info(const ka_graph *g, int64_t *N, int *z, int64_t *n_edges, int *n_classes)
{
  return ka_guard([&]() -> int {
    if (!g) return fail(KA_EINVAL, "graph is NULL");
    if (N) *N = g->N;
    if (z) *z = g->z;
    if (n_edges) *n_edges = g->lattice ? g->N * g->d : (int64_t)g->eu.size();
    if (n_classes) *n_classes = g->C;
    return KA_OK;
  });
}

extern "C" int ka_graph_export(const ka_graph *g, int32_t *adj, int32_t *edge_u, int32_t *edge_v,
                               int32_t *edge_class)
{
  return ka_guard([&]() -> int {
    if (!g) return fail(KA_EINVAL, "graph is NULL");
    if (g->lattice) {
      lattice_export(g, adj, edge_u, edge_v, edge_class);
      return KA_OK;
    }
    if (adj) std::memcpy(adj, g->adj.data(), g->adj.size() * sizeof(int32_t));
    if (edge_u) std::memcpy(edge_u, g->eu.data(), g->eu.size() * sizeof(int32_t));
    if (edge_v) std::memcpy(edge_v, g->ev.data(), g->ev.size() * sizeof(int32_t));
    if (edge_class) std::memcpy(edge_class, g->ecls.data(), g->ecls.size() * sizeof(int32_t));
    return KA_OK;
  });
}

extern "C" void ka_graph_free(ka_graph *g) { delete g; }

// ----------------------------------------------------------------------------------------
// Simulation
// ----------------------------------------------------------------------------------------

namespace {

size_t state_bytes(int64_t N, int R) { return (size_t)3 * (size_t)N * (size_t)(R / 64) * 8u; }

// Summary of full moved-ever elements of a general-graph sim (one bit per element and plane,
// in 32-bit words); 0 when the bit index would not fit 32 bits (the summary is then off).
size_t fsat_bytes(int64_t N, int R)
{
  const int W = R / 64, wpt = (W % 2 == 0) ? 2 : 1;
  const uint64_t bits = (uint64_t)N * (uint64_t)(W / wpt);
  if (bits >= (1ull << 32)) return 0;
  return (size_t)((bits + 31) / 32) * 4u;
}

size_t graph_device_bytes(const ka_graph *g)
{
  if (g->lattice) return 0;
  // edge records, slot-major neighbour lists, class offsets, vertex numbering
  return g->eu.size() * (sizeof(int4) + (size_t)2 * (size_t)(g->z - 1) * 4u) +
         (size_t)(g->C + 1) * sizeof(int) + (size_t)g->N * 4u;
}

void free_device(ka_sim *s)
{
  (void)hipFree(s->n);
  (void)hipFree(s->n0);
  (void)hipFree(s->f);
  (void)hipFree(s->nbr);
  (void)hipFree(s->edges);
  (void)hipFree(s->class_start_d);
  (void)hipFree(s->site_of);
  (void)hipFree(s->fsat);
  s->fsat = nullptr;
  (void)hipFree(s->thr_u);
  (void)hipFree(s->thr_i);
  (void)hipFree(s->err);
  (void)hipFree(s->counts);
  (void)hipFree(s->obs_d);
  (void)hipFree(s->lds_acc);
  s->lds_acc = nullptr;
  s->lds_acc_sweeps = 0;
  (void)hipFree(s->lds_snap);
  s->lds_snap = nullptr;
  s->lds_snap_rows = 0;
  s->n = s->n0 = s->f = nullptr;
}

template <typename T>
hipError_t dalloc(T **p, size_t bytes)
{
  return hipMalloc(reinterpret_cast<void **>(p), bytes ? bytes : 16);
}

// Element index of canonical site i in the lattice device layout.
inline int64_t lattice_element(const ka::LatticeGeom &g, int64_t i)
{
  int64_t sub = 0, pos = 0, sm = 1, pm = 1;
  for (int k = 0; k < g.d; ++k) {
    const int x = (int)(i % g.L);
    i /= g.L;
    sub += (x & 3) * sm;
    pos += (x >> 2) * pm;
    sm *= 4;
    pm *= g.Q;
  }
  return sub * g.P + pos;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev)
  {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard()
  {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool use_lds(const ka_sim *s)
{
  if (s->path_opt == 1) return false;
  if (s->path_opt == 2) return s->lds_fits;
  return s->lds_fits;
}

hipEvent_t pooled_event(ka_sim *s)
{
  if (!s->event_pool.empty()) {
    hipEvent_t e = s->event_pool.back();
    s->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Collect the durations of completed timed launches (call after a stream sync).
void harvest_timing(ka_sim *s)
{
  for (auto &pr : s->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, pr.first, pr.second) == hipSuccess) {
      s->timed_ms += ms;
      s->timed += 1;
    }
    s->event_pool.push_back(pr.first);
    s->event_pool.push_back(pr.second);
  }
  s->pending.clear();
}

// Release the sim's plane streams and their events (after the sim's stream has been
// synchronised, which waits for their work through the join events).
void release_plane_streams(ka_sim *s)
{
  for (int k = 0; k < 2; ++k) {
    if (s->plane_stream[k]) {
      (void)hipStreamSynchronize(s->plane_stream[k]);
      (void)hipStreamDestroy(s->plane_stream[k]);
    }
    if (s->join_ev[k]) (void)hipEventDestroy(s->join_ev[k]);
    s->plane_stream[k] = nullptr;
    s->join_ev[k] = nullptr;
  }
  if (s->fork_ev) (void)hipEventDestroy(s->fork_ev);
  s->fork_ev = nullptr;
}

// Whether the sweeps about to be enqueued run the word planes on the sim's two plane
// streams (KA_OPT_PLANE_STREAMS); creates them on first use and falls back to the sim's
// stream alone if that fails.
bool plane_split(ka_sim *s)
{
  if (!s->lattice || s->planes < 2 || !s->plane_streams || s->timing_every > 0) return false;
  if (s->plane_stream[0]) return true;
  hipError_t e = hipSuccess;
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipStreamCreateWithFlags(&s->plane_stream[k], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork_ev, hipEventDisableTiming);
  for (int k = 0; k < 2 && e == hipSuccess; ++k)
    e = hipEventCreateWithFlags(&s->join_ev[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    release_plane_streams(s);
    (void)hipGetLastError();
    s->plane_streams = 0;
    return false;
  }
  return true;
}

// One class pass over global memory: one launch over all planes on the sim's stream, or
// with `split` one launch per plane on the plane streams.
// Words per site of n and f that fit the Infinity Cache (256 MiB) together: a lattice whose
// 64-replica words do not all fit runs them in groups of this many (at least one), each group
// through a block of sweeps before the next, so that consecutive class passes of a group find
// its n and f in the cache instead of HBM.  Measured per class pass (3D, 256 replicas):
// L = 192 (108 MiB per word) 105.8 -> 83.2 us in groups of two words; L = 224 (172 MiB)
// 190.0 -> 131.1 us and L = 256 (256 MiB) 232 -> 162 us one word at a time; L = 160 (62.5 MiB,
// all four words fit) is fastest as one group.
constexpr int64_t kPlaneCacheBytes = (int64_t)256 << 20;

int plane_cache_words(int64_t N, int W)
{
  const int64_t per_word = N * 16;   // n and f, 8 bytes each
  const int64_t fit = kPlaneCacheBytes / per_word;
  return (int)std::max<int64_t>(1, std::min<int64_t>(fit, W));
}

// Rows per tile (log2) of the large-3D-lattice chunk order in the class pass.
#ifndef KA_ROW_TILE_LOG2
#define KA_ROW_TILE_LOG2 5
#endif
constexpr int kRowTileLog2 = KA_ROW_TILE_LOG2;

// One class pass (classes c .. c_end - 1 of a general graph's merged tail in one launch) on
// the sim's stream, or on `on` when given (then without per-launch timing events).
hipError_t launch_class(ka_sim *s, int c, uint32_t t, bool split, int c_end, int plane0 = 0, int nplanes = 0,
                        hipStream_t on = nullptr)
{
  const uint32_t k0 = (uint32_t)s->seed, k1 = (uint32_t)(s->seed >> 32);
  hipStream_t st = on ? on : s->stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool timed = !on && s->timing_every > 0 && (s->launches % s->timing_every) == 0;
  if (timed) {
    e0 = pooled_event(s);
    e1 = pooled_event(s);
    (void)hipEventRecord(e0, s->stream);
  }
  hipError_t err;
  if (s->lattice) {
    ka::PassLattice a{};
    a.n = s->n;
    a.f = s->f;
    a.g = s->geom;
    a.mu = c >> 2;
    a.planes = s->planes;
    const int nsub = s->geom.d == 2 ? 4 : 16;   // lower-endpoint sublattices per class
    const int per_plane = nsub * 64 * ((s->geom.P + 63) / 64);  // whole 64-position chunks
    a.blocks_per_plane = (per_plane + 255) / 256;
    a.t = t;
    a.c = (uint32_t)c;
    a.key0 = k0;
    a.key1 = k1;
    a.noise = s->noise;
    // Large 3D lattices (Q = L/4 a power of two >= 64): rows visited in tiles of 32 along
    // p1, so that the +-e_2 neighbour rows of a chunk are read within one L2's reach
    a.row_tile_log2 = 0;
    a.q_log2 = 0;
    if (s->geom.d == 3 && s->geom.Q >= 64 && (s->geom.Q & (s->geom.Q - 1)) == 0) {
      int lq = 0;
      while ((1 << lq) < s->geom.Q) ++lq;
      a.q_log2 = lq;
      a.row_tile_log2 = kRowTileLog2;
    }
    if (split) {
      err = hipSuccess;
      for (int p = 0; p < s->planes && err == hipSuccess; ++p) {
        a.plane0 = p;
        a.planes = 1;
        err = ka::launch_pass_lattice(a, s->m, s->wpt, s->plane_stream[p & 1]);
        s->launches += 1;
      }
      return err;
    }
    a.plane0 = plane0;
    if (nplanes > 0) a.planes = nplanes;   // one group of planes
    err = ka::launch_pass_lattice(a, s->m, s->wpt, st);
  } else {
    ka::PassGraph a{};
    a.n = s->n;
    a.f = s->f;
    a.edges = s->edges;
    a.nbr = s->nbr;
    a.stride = s->edges_total;
    a.first = s->plan->class_start[c];
    a.count = s->plan->class_start[c + 1] - s->plan->class_start[c];
    a.N = (int)s->N;
    a.plane0 = plane0;
    a.planes = nplanes > 0 ? nplanes : s->planes;   // the launcher picks the workgroup size and blocks per plane
    a.t = t;
    a.c = (uint32_t)c;
    a.key0 = k0;
    a.key1 = k1;
    a.noise = s->noise;
    a.fsat = s->fsat;
    if (c_end > c + 1) {
      a.class_start = s->class_start_d;
      a.c_end = (uint32_t)c_end;
      err = ka::launch_tail_graph(a, s->z, s->m, s->wpt, st);
    } else {
      err = a.count > 0 ? ka::launch_pass_graph(a, s->z, s->m, s->wpt, st) : hipSuccess;
    }
  }
  if (timed) {
    (void)hipEventRecord(e1, s->stream);
    s->pending.emplace_back(e0, e1);
  }
  s->launches += 1;
  return err;
}

// First class of the trailing run of classes with at most kTailEdges edges each, which the
// global path runs in one launch (one workgroup per plane); the class count if that run has
// fewer than two classes.  Greedy distance-2 colourings end in a few such tiny classes, each
// of which would otherwise cost a whole launch for a few hundred edges.  The merge is used
// only for graphs whose words of one plane take at most kTailPlaneBytes: on larger graphs
// the one CU's gathers for a few hundred edges miss its caches and take longer than the
// launches they replace (per sweep, 2^14 to 2^16 vertices: 4-7 us less; 2^18 and 2^20:
// 1 and 4.5 us more).
constexpr size_t kTailPlaneBytes = (size_t)1 << 20;

int tail_first(const std::vector<int> &class_start)
{
  const int C = (int)class_start.size() - 1;
  int c = C;
  while (c > 0 && class_start[(size_t)c] - class_start[(size_t)c - 1] <= ka::kTailEdges) --c;
  return C - c >= 2 ? c : C;
}

constexpr int64_t kLdsChunk = 20000;            // sweeps per LDS-resident launch
constexpr size_t kLdsAccBudget = (size_t)8 << 20;  // bytes of pre-generated acceptance words
// Observations of an LDS-resident launch are copied out as snapshots of n and f and counted
// on the whole device after the launch, when its snapshots fit this many bytes; otherwise the
// launch's one workgroup counts them in place.
constexpr size_t kLdsSnapBudget = (size_t)4 << 20;

// Sweeps per launch and buffer bytes of the pre-generated acceptance words of an LDS lattice
// sweep (d, L, R); 0 sweeps if that layout draws its words in the loop.
int64_t lds_acc_plan(int d, int L, int R, size_t *bytes)
{
  const int wpt = ((R / 64) % 2 == 0) ? 2 : 1;
  const int planes = (R / 64) / wpt;
  if (bytes) *bytes = 0;
  const int Q = L / 4;
  const int P = d == 2 ? Q * Q : Q * Q * Q;
  if (!ka::lds_accept_supported(d, wpt, ka::lds_lattice_slots(d, P))) return 0;
  const size_t per_sweep = (size_t)planes * (size_t)(4 * d) * (size_t)ka::lds_lattice_slots(d, P) * 1024u *
                           (size_t)wpt * 8u;
  if (per_sweep > kLdsAccBudget) return 0;   // drawn in the loop: the buffer stays within budget
  const int64_t sweeps = std::max<int64_t>(1, std::min<int64_t>(kLdsChunk, (int64_t)(kLdsAccBudget / per_sweep)));
  if (bytes) *bytes = (size_t)sweeps * per_sweep;
  return sweeps;
}

// The same for the LDS graph sweep over E class-sorted edges of degree z whose largest class
// has max_class edges; 0 sweeps if a class has more edges per thread than the sweep prefetches
// or the layout draws its words in the loop.
int64_t lds_acc_plan_graph(int64_t E, int max_class, int z, int R, size_t *bytes)
{
  if (bytes) *bytes = 0;
  const int wpt = ((R / 64) % 2 == 0) ? 2 : 1;
  if (E < 1 || ka::lds_graph_slots(max_class) > ka::kLdsGraphAcceptSlots || !ka::lds_graph_accept_supported(z, wpt))
    return 0;
  const size_t per_sweep = (size_t)E * (size_t)(R / 64) * 8u;   // every plane's words
  if (per_sweep > kLdsAccBudget) return 0;
  const int64_t sweeps = std::max<int64_t>(1, std::min<int64_t>(kLdsChunk, (int64_t)(kLdsAccBudget / per_sweep)));
  if (bytes) *bytes = (size_t)sweeps * per_sweep;
  return sweeps;
}

int max_class_edges(const std::vector<int> &class_start)
{
  int most = 0;
  for (size_t c = 0; c + 1 < class_start.size(); ++c) most = std::max(most, class_start[c + 1] - class_start[c]);
  return most;
}

// Sweeps per LDS-resident launch of this sim; when its layout takes pre-generated acceptance
// words, allocates their buffer on first use (if that fails, the words are drawn in the loop
// and launches cover up to kLdsChunk sweeps).
int64_t lds_chunk(ka_sim *s)
{
  if (!s->lds_acc_tried) {
    s->lds_acc_tried = true;
    size_t bytes = 0;
    const int64_t sweeps = s->lattice ? lds_acc_plan(s->geom.d, s->geom.L, s->R, &bytes)
                                      : lds_acc_plan_graph((int64_t)s->edges_total,
                                                           max_class_edges(s->plan->class_start), s->z, s->R, &bytes);
    if (sweeps > 0 && dalloc(&s->lds_acc, bytes) == hipSuccess) {
      s->lds_acc_sweeps = sweeps;
    } else {
      (void)hipGetLastError();
      s->lds_acc = nullptr;
      s->lds_acc_sweeps = 0;
    }
  }
  return s->lds_acc ? s->lds_acc_sweeps : kLdsChunk;
}

hipError_t ensure_obs_buffers(ka_sim *s, size_t n_obs)
{
  const size_t need = n_obs * 3u * (size_t)s->R;
  if (need > s->counts_cap) {
    (void)hipFree(s->counts);
    s->counts = nullptr;
    s->counts_cap = 0;
    hipError_t e = dalloc(&s->counts, need * sizeof(unsigned long long));
    if (e != hipSuccess) return e;
    s->counts_cap = need;
  }
  if (n_obs > s->obs_cap) {
    (void)hipFree(s->obs_d);
    s->obs_d = nullptr;
    s->obs_cap = 0;
    hipError_t e = dalloc(&s->obs_d, n_obs * sizeof(int64_t));
    if (e != hipSuccess) return e;
    s->obs_cap = n_obs;
  }
  return hipSuccess;
}

// Bytes of one snapshot row of the LDS-resident path: n and f of every plane.
size_t lds_snap_row_bytes(int64_t N, int R) { return 2u * (size_t)N * (size_t)(R / 64) * 8u; }

// Room for `rows` snapshot rows within kLdsSnapBudget; false if they do not fit it or the
// allocation fails (the observations are then counted in the loop).  Called at the start of
// ka_run, when no queued work uses the old buffer.
bool ensure_lds_snap(ka_sim *s, size_t rows)
{
  const size_t row = lds_snap_row_bytes(s->N, s->R);
  if (rows == 0 || rows * row > kLdsSnapBudget) return false;
  if (rows <= s->lds_snap_rows) return true;
  (void)hipFree(s->lds_snap);
  s->lds_snap = nullptr;
  s->lds_snap_rows = 0;
  const size_t want = std::min(kLdsSnapBudget / row, std::max<size_t>(rows, 32));
  if (dalloc(&s->lds_snap, want * row) != hipSuccess) {
    (void)hipGetLastError();
    s->lds_snap = nullptr;
    return false;
  }
  s->lds_snap_rows = want;
  return true;
}

// Count `rows` states into counts rows q0.. on the whole device: n and f of row r start at
// n + r * stride and f + r * stride (stride 0: the same state for every row).
hipError_t observe_rows(ka_sim *s, const ka::u64 *n, const ka::u64 *f, size_t stride, int q0, int rows)
{
  ka::ObserveArgs a{};
  a.n0 = s->n0;
  a.N = (int)s->N;
  a.planes = s->planes;
  a.R = s->R;
  a.row_stride = stride;
  hipError_t e = hipSuccess;
  for (int r0 = 0; r0 < rows && e == hipSuccess; r0 += 65535) {   // grid z limit
    a.n = n + (size_t)r0 * stride;
    a.f = f + (size_t)r0 * stride;
    a.out = s->counts + (size_t)(q0 + r0) * 3u * (size_t)s->R;
    a.rows = std::min(rows - r0, 65535);
    e = ka::launch_observe(a, s->wpt, s->stream);
  }
  return e;
}

// LDS-resident launch covering sweeps [t_from, t_to) that also records observations
// obs[q0..q1) (absolute times) into counts rows q0..q1 (which start at zero): with `snap` as
// snapshots counted by the observation kernel after the launch (lds_snap holds q1 - q0 rows),
// otherwise counted in the loop.
hipError_t launch_lds(ka_sim *s, int64_t t_from, int64_t t_to, int q0, int q1, bool snap)
{
  if (q1 > q0 && t_to == t_from)   // no sweep: every observation is of the current state
    return observe_rows(s, s->n, s->f, 0, q0, q1 - q0);
  ka::SweepLds a{};
  a.n = s->n;
  a.f = s->f;
  a.n0 = s->n0;
  a.g = s->geom;
  a.edges = s->edges;
  a.nbr = s->nbr;
  a.stride = s->edges_total;
  a.class_start = s->class_start_d;
  a.N = (int)s->N;
  a.C = s->C;
  a.t0 = (uint32_t)t_from;
  a.n_sweeps = (int)(t_to - t_from);
  a.obs_times = s->obs_d + q0;
  a.n_obs = q1 - q0;
  a.obs_out = s->counts + (size_t)q0 * 3u * (size_t)s->R;
  a.R = s->R;
  a.key0 = (uint32_t)s->seed;
  a.key1 = (uint32_t)(s->seed >> 32);
  a.noise = s->noise;
  if (s->lds_acc && a.n_sweeps > 0) {
    if (a.n_sweeps > s->lds_acc_sweeps) return hipErrorInvalidValue;
    a.acc = s->lds_acc;
    a.acc_slots = s->lattice ? ka::lds_lattice_slots(s->geom.d, s->geom.P)
                             : ka::lds_graph_slots(max_class_edges(s->plan->class_start));
    hipError_t e = ka::launch_lds_accept(a, s->lattice != 0, s->wpt, s->stream);
    if (e != hipSuccess) return e;
  }
  const bool snapshots = snap && q1 > q0;
  if (snapshots) {
    if (!s->lds_snap || (size_t)(q1 - q0) > s->lds_snap_rows) return hipErrorInvalidValue;
    a.snap = s->lds_snap;
  }
  hipError_t e = ka::launch_sweep_lds(a, s->lattice != 0, s->z, s->m, s->wpt, s->lds_bytes, s->stream);
  if (e == hipSuccess && snapshots) {
    const size_t row_words = (size_t)s->N * (size_t)s->W;
    e = observe_rows(s, s->lds_snap, s->lds_snap + row_words, 2u * row_words, q0, q1 - q0);
  }
  return e;
}

hipError_t sweep_global(ka_sim *s, int64_t n)
{
  if (n <= 0) return hipSuccess;
  const bool split = plane_split(s);
  hipError_t e = hipSuccess;
  if (split) {
    e = hipEventRecord(s->fork_ev, s->stream);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipStreamWaitEvent(s->plane_stream[k], s->fork_ev, 0);
    if (e != hipSuccess) return e;
  }
  // word planes in groups, each group through all n sweeps before the next (the planes are
  // independent chains); np = 0: every plane in each launch
  const int group = split ? 0 : (s->plane_group_opt >= 0 ? s->plane_group_opt : s->plane_group);
  const bool grouped = group > 0 && group < s->planes;
  // general graphs: the trailing run of tiny classes in one launch
  const int tail = (!s->lattice && s->tail_opt) ? s->tail_first : s->C;
  for (int p0 = 0; p0 < (grouped ? s->planes : 1) && e == hipSuccess; p0 += (grouped ? group : 1)) {
    const int np = grouped ? std::min(group, s->planes - p0) : 0;
    for (int64_t q = 0; q < n && e == hipSuccess; ++q) {
      const uint32_t t = (uint32_t)(s->t + q);
      for (int c = 0; c < tail && e == hipSuccess; ++c) e = launch_class(s, c, t, split, c + 1, p0, np);
      if (tail < s->C && e == hipSuccess) e = launch_class(s, tail, t, split, s->C, p0, np);
    }
  }
  if (split) {
    // joined even after a failed launch, so that later work on the sim's stream stays
    // ordered after everything the plane streams received
    for (int k = 0; k < 2; ++k) {
      hipError_t j = hipEventRecord(s->join_ev[k], s->plane_stream[k]);
      if (j == hipSuccess) j = hipStreamWaitEvent(s->stream, s->join_ev[k], 0);
      if (e == hipSuccess) e = j;
    }
  }
  return e;
}

hipError_t observe_global(ka_sim *s, int row) { return observe_rows(s, s->n, s->f, 0, row, 1); }

// After a stream synchronisation: report a failure flagged by the initial-state kernels.
int check_init_flag(ka_sim *s)
{
  if (s->init_checked) return KA_OK;
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, s->err, sizeof(int), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return hip_fail(e, "reading the init status");
  s->init_checked = true;
  if (flag) return fail(KA_EDEVICE, "initial-state selection failed (flag %d)", flag);
  return KA_OK;
}

int check_sim(const ka_sim *s)
{
  if (!s) return fail(KA_EINVAL, "sim is NULL");
  if (!s->n) return fail(KA_ESTATE, "sim has no device state");
  if (s->batch) return fail(KA_ESTATE, "sim is a batch member until its batch work is detached");
  return KA_OK;
}

}  // namespace

extern "C" int ka_footprint(const ka_graph *g, int n_replicas, size_t *device_bytes)
{
  return ka_guard([&]() -> int {
    if (!g || !device_bytes) return fail(KA_EINVAL, "NULL argument");
    if (n_replicas <= 0 || n_replicas % 64 != 0) return fail(KA_EINVAL, "n_replicas must be a positive multiple of 64");
    *device_bytes = state_bytes(g->N, n_replicas) + graph_device_bytes(g) +
                    (size_t)n_replicas * 16u + (size_t)3 * n_replicas * 8u + 64u +
                    (g->lattice ? 0 : fsat_bytes(g->N, n_replicas));
    const int wpt = ((n_replicas / 64) % 2 == 0) ? 2 : 1;
    if (ka::sweep_lds_bytes((int)g->N, wpt) + 4096 <= (size_t)ka::max_lds_bytes()) {
      // an instance on the LDS-resident path adds its pre-generated acceptance words and its
      // observation snapshots
      size_t acc = 0;
      if (g->lattice) {
        (void)lds_acc_plan(g->d, g->L, n_replicas, &acc);
      } else {
        std::vector<int> cs((size_t)g->C + 1, 0);
        for (int32_t c : g->ecls) cs[(size_t)c + 1] += 1;
        for (size_t c = 1; c < cs.size(); ++c) cs[c] += cs[c - 1];
        (void)lds_acc_plan_graph((int64_t)g->ecls.size(), max_class_edges(cs), g->z, n_replicas, &acc);
      }
      const size_t row = lds_snap_row_bytes(g->N, n_replicas);
      *device_bytes += acc + (kLdsSnapBudget / row) * row;
    }
    return KA_OK;
  });
}

extern "C" int ka_init_k(const ka_graph *g, int m, int64_t K, uint64_t seed, int n_replicas,
                         void *hip_stream, ka_sim **out)
{
  return ka_guard([&]() -> int {
    if (!out) return fail(KA_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(KA_EINVAL, "graph is NULL");
    if (m < 0 || m > g->z - 1) return fail(KA_EINVAL, "activation number m must be in [0, z-1] = [0, %d] (got %d)", g->z - 1, m);
    if (n_replicas <= 0 || n_replicas % 64 != 0)
      return fail(KA_EINVAL, "n_replicas must be a positive multiple of 64 (got %d)", n_replicas);
    if (K < 0 || K > g->N) return fail(KA_EINVAL, "particle number K must be in [0, N] (got %lld)", (long long)K);
    ka_sim *s = new (std::nothrow) ka_sim;
    if (!s) return fail(KA_ENOMEM, "host allocation failed");
    s->lattice = g->lattice;
    s->z = g->z;
    s->C = g->C;
    s->N = g->N;
    s->m = m;
    s->K = K;
    s->seed = seed;
    s->R = n_replicas;
    s->W = n_replicas / 64;
    s->wpt = (s->W % 2 == 0) ? 2 : 1;
    if (g->lattice) {
      // A lattice whose n and f exceed the Infinity Cache runs its word planes group by group
      // (each group through a whole block of sweeps), each group small enough for its n and f
      // to stay in the cache across the block's class passes.  (General graphs gain nothing
      // from it: on a 2^23-vertex z=4 graph with 256 replicas, 6.27 ms per sweep in groups
      // against 6.16 ms with all planes per launch; their passes are bound by gathers.)
      const int per_group = plane_cache_words(g->N, s->W);
      if (per_group < s->W) {
        s->wpt = (per_group >= 2 && s->W % 2 == 0) ? 2 : 1;
        s->plane_group = std::max(1, per_group / s->wpt);
      }
    }
    s->planes = s->W / s->wpt;
    (void)hipGetDevice(&s->device);
    {
      const hipError_t se = ka::observe_scratch_setup(s->device);
      if (se != hipSuccess) {
        delete s;
        return hip_fail(se, "observation scratch");
      }
    }
    if (hip_stream) {
      s->stream = (hipStream_t)hip_stream;
    } else {
      hipError_t e = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking);
      if (e != hipSuccess) {
        delete s;
        return hip_fail(e, "hipStreamCreate");
      }
      s->own_stream = true;
    }
    const size_t words = (size_t)s->N * s->W;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = dalloc(&s->n, words * 8);
    if (e == hipSuccess) e = dalloc(&s->n0, words * 8);
    if (e == hipSuccess) e = dalloc(&s->f, words * 8);
    if (e == hipSuccess) e = dalloc(&s->thr_u, (size_t)s->R * 8);
    if (e == hipSuccess) e = dalloc(&s->thr_i, (size_t)s->R * 8);
    if (e == hipSuccess) e = dalloc(&s->err, sizeof(int));
    if (e != hipSuccess) {
      free_device(s);
      if (s->own_stream) (void)hipStreamDestroy(s->stream);
      delete s;
      return fail(KA_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    if (s->lattice) {
      s->geom.d = g->d;
      s->geom.L = g->L;
      s->geom.Q = g->L / 4;
      s->geom.P = g->d == 2 ? s->geom.Q * s->geom.Q : s->geom.Q * s->geom.Q * s->geom.Q;
      s->geom.N = (int)g->N;
      s->geom.qinv = ka::lattice_qinv(s->geom.Q);
    } else {
      const std::shared_ptr<const GraphPlan> plan = graph_plan(g);
      if (!plan) {
        free_device(s);
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(KA_ENOMEM, "host allocation failed for the graph schedule");
      }
      // The sim keeps the plan alive, so the copies below may run after the graph is freed.
      s->plan = plan;
      // merged only while one plane's words are small enough to stay near the one CU
      s->tail_first = (size_t)s->N * 8u * (size_t)s->wpt <= kTailPlaneBytes ? tail_first(plan->class_start) : s->C;
      const std::vector<int32_t> &site_of = plan->site_of;
      const std::vector<int4> &rec = plan->rec;
      const std::vector<int32_t> &nbr = plan->nbr;
      const std::vector<int> &cs = plan->class_start;
      s->edges_total = rec.size();
      e = dalloc(&s->nbr, nbr.size() * 4);
      if (e == hipSuccess) e = dalloc(&s->site_of, site_of.size() * sizeof(int32_t));
      if (e == hipSuccess) e = dalloc(&s->edges, rec.size() * sizeof(int4));
      if (e == hipSuccess) e = dalloc(&s->class_start_d, cs.size() * sizeof(int));
      if (e == hipSuccess) e = hipMemcpyAsync(s->nbr, nbr.data(), nbr.size() * 4, hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->site_of, site_of.data(), site_of.size() * sizeof(int32_t), hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->edges, rec.data(), rec.size() * sizeof(int4), hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(s->class_start_d, cs.data(), cs.size() * sizeof(int), hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess && fsat_bytes(s->N, s->R) > 0) {
        e = dalloc(&s->fsat, fsat_bytes(s->N, s->R));
        if (e == hipSuccess) e = hipMemsetAsync(s->fsat, 0, fsat_bytes(s->N, s->R), s->stream);
      }
      if (e != hipSuccess) {
        free_device(s);
        if (s->own_stream) (void)hipStreamDestroy(s->stream);
        delete s;
        return fail(KA_ENOMEM, "device allocation/copy failed: %s", hipGetErrorString(e));
      }
    }
    s->lds_bytes = ka::sweep_lds_bytes((int)s->N, s->wpt);
    s->lds_fits = s->lds_bytes + 4096 <= (size_t)ka::max_lds_bytes();
    // initial state
    ka::InitArgs a{};
    a.N = (int)s->N;
    a.K = K;
    a.key0 = (uint32_t)seed;
    a.key1 = (uint32_t)(seed >> 32);
    a.thr_u = s->thr_u;
    a.thr_i = s->thr_i;
    a.err = s->err;
    a.n = s->n;
    a.n0 = s->n0;
    a.f = s->f;
    a.planes = s->planes;
    a.is_lattice = s->lattice;
    a.g = s->geom;
    a.site_of = s->site_of;
    e = hipMemsetAsync(s->err, 0, sizeof(int), s->stream);
    if (e == hipSuccess) e = ka::launch_init(a, s->R, s->wpt, s->stream);
    if (e != hipSuccess) {
      free_device(s);
      if (s->own_stream) (void)hipStreamDestroy(s->stream);
      delete s;
      return hip_fail(e, "init kernels");
    }
    *out = s;
    return KA_OK;
  });
}

extern "C" int ka_init(const ka_graph *g, int m, double rho, uint64_t seed, int n_replicas,
                       void *hip_stream, ka_sim **out)
{
  return ka_guard([&]() -> int {
    if (!g) return fail(KA_EINVAL, "graph is NULL");
    if (!(rho >= 0.0 && rho <= 1.0)) return fail(KA_EINVAL, "density rho must be in [0, 1]");
    const int64_t K = (int64_t)std::floor(rho * (double)g->N + 0.5);
    return ka_init_k(g, m, K, seed, n_replicas, hip_stream, out);
  });
}

extern "C" int ka_sweep(ka_sim *s, int64_t n_sweeps)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    if (n_sweeps < 0) return fail(KA_EINVAL, "n_sweeps < 0");
    if (s->t + n_sweeps >= (1ll << 32)) return fail(KA_ESTATE, "sweep index would reach 2^32");
    DeviceGuard dg(s->device);
    hipError_t e = hipSuccess;
    if (use_lds(s)) {
      int64_t done = 0;
      while (done < n_sweeps && e == hipSuccess) {
        const int64_t chunk = std::min(lds_chunk(s), n_sweeps - done);
        e = ensure_obs_buffers(s, 1);
        if (e == hipSuccess) e = launch_lds(s, s->t + done, s->t + done + chunk, 0, 0, false);
        done += chunk;
      }
    } else {
      e = sweep_global(s, n_sweeps);
    }
    if (e != hipSuccess) return hip_fail(e, "ka_sweep");
    s->t += n_sweeps;
    return KA_OK;
  });
}

extern "C" int ka_run(ka_sim *s, const int64_t *obs_times, int n_obs, int64_t *density,
                      int64_t *overlap, int64_t *persistence)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    if (n_obs < 0 || (n_obs > 0 && !obs_times)) return fail(KA_EINVAL, "bad observation list");
    int64_t prev = s->t;
    for (int q = 0; q < n_obs; ++q) {
      if (obs_times[q] < prev) return fail(KA_EINVAL, "observation times must be non-decreasing and >= t");
      prev = obs_times[q];
    }
    if (prev >= (1ll << 32)) return fail(KA_ESTATE, "sweep index would reach 2^32");
    if (n_obs == 0) return KA_OK;
    DeviceGuard dg(s->device);
    hipError_t e = ensure_obs_buffers(s, (size_t)n_obs);
    if (e != hipSuccess) return fail(KA_ENOMEM, "observation buffers: %s", hipGetErrorString(e));
    const size_t cbytes = (size_t)n_obs * 3u * (size_t)s->R * sizeof(unsigned long long);
    e = hipMemsetAsync(s->counts, 0, cbytes, s->stream);
    if (e == hipSuccess && use_lds(s)) {
      e = hipMemcpyAsync(s->obs_d, obs_times, (size_t)n_obs * sizeof(int64_t), hipMemcpyHostToDevice, s->stream);
      // chunks [a, b) of at most lds_chunk sweeps; observation q goes to the first chunk
      // that can record it (times in [a, b] for the first chunk, (a, b] afterwards)
      struct Chunk {
        int64_t a, b;
        int q0, q1;
      };
      std::vector<Chunk> plan;
      int q = 0;
      int64_t a = s->t;
      const int64_t chunk = lds_chunk(s);
      size_t most = 0;   // observations of the fullest chunk that sweeps
      while (q < n_obs) {
        const int64_t b = std::min(a + chunk, obs_times[n_obs - 1]);
        int q1 = q;
        while (q1 < n_obs && obs_times[q1] <= b && (plan.empty() || obs_times[q1] > a)) ++q1;
        plan.push_back({a, b, q, q1});
        if (b > a) most = std::max(most, (size_t)(q1 - q));
        q = q1;
        a = b;
      }
      const bool snap = most > 0 && ensure_lds_snap(s, most);
      for (size_t k = 0; k < plan.size() && e == hipSuccess; ++k)
        e = launch_lds(s, plan[k].a, plan[k].b, plan[k].q0, plan[k].q1, snap);
    } else {
      for (int q = 0; q < n_obs && e == hipSuccess; ++q) {
        const int64_t n = obs_times[q] - s->t;
        e = sweep_global(s, n);
        s->t = obs_times[q];
        if (e == hipSuccess) e = observe_global(s, q);
      }
    }
    s->t = obs_times[n_obs - 1];
    std::vector<unsigned long long> host((size_t)n_obs * 3u * (size_t)s->R);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), s->counts, cbytes, hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "ka_run");
    rc = check_init_flag(s);
    if (rc) return rc;
    harvest_timing(s);
    for (int q = 0; q < n_obs; ++q)
      for (int b = 0; b < s->R; ++b) {
        const size_t base = (size_t)q * 3u * s->R;
        if (density) density[(size_t)q * s->R + b] = (int64_t)host[base + b];
        if (overlap) overlap[(size_t)q * s->R + b] = (int64_t)host[base + s->R + b];
        if (persistence) persistence[(size_t)q * s->R + b] = (int64_t)host[base + 2u * s->R + b];
      }
    return KA_OK;
  });
}

extern "C" int ka_observe(ka_sim *s, int64_t *t, int64_t *density, int64_t *overlap,
                          int64_t *persistence)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    const int64_t now = s->t;
    rc = ka_run(s, &now, 1, density, overlap, persistence);
    if (rc) return rc;
    if (t) *t = s->t;
    return KA_OK;
  });
}

extern "C" int ka_observe_noalloc(ka_sim *s, int64_t *t, int64_t *density, int64_t *overlap,
                                  int64_t *persistence)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    if (s->R > ka::kObserveScratchReplicas)
      return fail(KA_EINVAL, "ka_observe_noalloc supports at most %d replicas (got %d)",
                  ka::kObserveScratchReplicas, s->R);
    DeviceGuard dg(s->device);
    unsigned long long *scr = ka::observe_scratch(s->device);
    if (!scr) return fail(KA_ESTATE, "observation scratch not set up on device %d", s->device);
    const int words = 3 * s->R;
    hipError_t e = ka::launch_fill_u64(scr, words, 0ull, s->stream);
    if (e == hipSuccess) {
      ka::ObserveArgs a{};
      a.n = s->n;
      a.n0 = s->n0;
      a.f = s->f;
      a.N = (int)s->N;
      a.planes = s->planes;
      a.R = s->R;
      a.out = scr;
      a.rows = 1;
      a.row_stride = 0;
      e = ka::launch_observe(a, s->wpt, s->stream);
    }
    // the counts (below 2^63) go straight into the caller's arrays: no host buffer either
    int64_t *dst[3] = {density, overlap, persistence};
    for (int o = 0; o < 3 && e == hipSuccess; ++o)
      if (dst[o])
        e = hipMemcpyAsync(dst[o], scr + (size_t)o * s->R, (size_t)s->R * sizeof(int64_t), hipMemcpyDeviceToHost,
                           s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "ka_observe_noalloc");
    if (t) *t = s->t;
    return KA_OK;
  });
}

int ka_sim_steps_per_sweep(const ka_sim *s)
{
  return (!s->lattice && s->tail_opt && s->tail_first < s->C) ? s->tail_first + 1 : s->C;
}

hipError_t ka_sim_passes(ka_sim *s, int64_t p0, int64_t count, hipStream_t stream)
{
  const int per = ka_sim_steps_per_sweep(s);
  // word planes in the groups ka_sweep uses, each group through all `count` launches before
  // the next (the planes are independent chains)
  const int group = s->plane_group_opt >= 0 ? s->plane_group_opt : s->plane_group;
  const bool grouped = group > 0 && group < s->planes;
  hipError_t e = hipSuccess;
  for (int q0 = 0; q0 < (grouped ? s->planes : 1) && e == hipSuccess; q0 += (grouped ? group : 1)) {
    const int np = grouped ? std::min(group, s->planes - q0) : 0;
    for (int64_t p = p0; p < p0 + count && e == hipSuccess; ++p) {
      const uint32_t t = (uint32_t)(s->t + p / per);
      const int c = (int)(p % per);
      const int c_end = (per < s->C && c == per - 1) ? s->C : c + 1;   // the merged tail
      e = launch_class(s, c, t, false, c_end, q0, np, stream);
    }
  }
  return e;
}

// Enqueue the counts of ka_observe at the current t on the sim's stream, copied into
// host_out (pinned, 3 * R values: density, overlap, persistence), without synchronising.
int ka_sim_observe_async(ka_sim *s, unsigned long long *host_out)
{
  int rc = check_sim(s);
  if (rc) return rc;
  DeviceGuard dg(s->device);
  hipError_t e = ensure_obs_buffers(s, 1);
  const size_t bytes = 3u * (size_t)s->R * sizeof(unsigned long long);
  if (e == hipSuccess) e = hipMemsetAsync(s->counts, 0, bytes, s->stream);
  if (e == hipSuccess) e = observe_global(s, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(host_out, s->counts, bytes, hipMemcpyDeviceToHost, s->stream);
  if (e != hipSuccess) return hip_fail(e, "observe");
  return KA_OK;
}

void ka_sim_rebind_stream(ka_sim *s, hipStream_t stream)
{
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  s->stream = stream;
  s->own_stream = false;
}

// Bind the sim to a new stream that it owns (after waiting for its old one if asked to).
int ka_sim_take_own_stream(ka_sim *s, bool wait)
{
  if (!s) return fail(KA_EINVAL, "sim is NULL");
  DeviceGuard dg(s->device);
  hipError_t e = wait ? hipStreamSynchronize(s->stream) : hipSuccess;
  hipStream_t fresh = nullptr;
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&fresh, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "stream");
  if (s->own_stream) (void)hipStreamDestroy(s->stream);
  s->stream = fresh;
  s->own_stream = true;
  return KA_OK;
}

namespace {

// Four-point sums on a graph without a geometry (Sec. 3.3: distance 0 for i = j and 1 for
// i != j).  With Q_i = sum_b q_i^b and O_b = sum_i q_i^b (the overlap count of replica b):
//   shell 0: S2 = sum_i sum_b q_i^b = sum_b O_b,   S11 = sum_i Q_i^2,          count 1;
//   shell 1: S2 = sum_b (O_b^2 - O_b),            S11 = (sum_i Q_i)^2 - sum_i Q_i^2, count N-1.
int pair_sums_graph(ka_sim *s, int r2_max, int64_t *S2, int64_t *S11, int64_t *count)
{
  std::vector<int64_t> ov((size_t)s->R);
  int rc = ka_observe(s, nullptr, nullptr, ov.data(), nullptr);
  if (rc) return rc;
  DeviceGuard dg(s->device);
  unsigned long long *d_out = nullptr;
  unsigned long long host[2] = {0, 0};
  hipError_t e = dalloc(&d_out, 2 * sizeof(unsigned long long));
  if (e == hipSuccess) e = hipMemsetAsync(d_out, 0, 2 * sizeof(unsigned long long), s->stream);
  if (e == hipSuccess) {
    ka::PairGraphArgs a{};
    a.n = s->n;
    a.n0 = s->n0;
    a.N = (int)s->N;
    a.planes = s->planes;
    a.out = d_out;
    e = ka::launch_pairs_graph(a, s->wpt, s->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(host, d_out, sizeof(host), hipMemcpyDeviceToHost, s->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  (void)hipFree(d_out);
  if (e != hipSuccess) return hip_fail(e, "ka_observe_pairs");
  __int128 sum_o = 0, sum_o2 = 0;
  for (int64_t o : ov) {
    sum_o += o;
    sum_o2 += (__int128)o * o;
  }
  const __int128 sq = (__int128)host[0];
  const __int128 sq2 = (__int128)host[1];
  if (sq != sum_o) return fail(KA_EDEVICE, "pair sums: per-site and per-replica overlap totals differ");
  const __int128 lim = (__int128)INT64_MAX;
  const __int128 s2_1 = sum_o2 - sum_o, s11_1 = sq * sq - sq2;
  if (s2_1 > lim || s11_1 > lim) return fail(KA_EINVAL, "pair sums exceed int64 (N x n_replicas too large)");
  for (int q = 0; q <= r2_max; ++q) {
    const int64_t v2 = q == 0 ? (int64_t)sum_o : q == 1 ? (int64_t)s2_1 : 0;
    const int64_t v11 = q == 0 ? (int64_t)sq2 : q == 1 ? (int64_t)s11_1 : 0;
    if (S2) S2[q] = v2;
    if (S11) S11[q] = v11;
    if (count) count[q] = q == 0 ? 1 : q == 1 ? s->N - 1 : 0;
  }
  return KA_OK;
}

}  // namespace

extern "C" int ka_observe_pairs(ka_sim *s, int r2_max, int64_t *S2, int64_t *S11, int64_t *count)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    if (r2_max < 0 || r2_max > ka::kMaxPairShells - 1)
      return fail(KA_EINVAL, "r2_max must be in [0, %d]", ka::kMaxPairShells - 1);
    if (s->W > 16) return fail(KA_EINVAL, "spatial pair sums support up to 1024 replicas");
    if (!s->lattice) return pair_sums_graph(s, r2_max, S2, S11, count);
    const int d = s->geom.d, L = s->geom.L;
    // every displacement of the torus once, components in the minimum image (|c| <= L/2)
    std::vector<int4> disp;
    std::vector<int64_t> cnt((size_t)r2_max + 1, 0);
    const int n_total = d == 2 ? L * L : L * L * L;
    for (int q = 0; q < n_total; ++q) {
      int c[3] = {q % L, (q / L) % L, d == 3 ? q / (L * L) : 0};
      int r2 = 0;
      for (int k = 0; k < d; ++k) {
        if (c[k] > L / 2) c[k] -= L;
        r2 += c[k] * c[k];
      }
      if (r2 > r2_max) continue;
      disp.push_back(make_int4(c[0], c[1], c[2], r2));
      cnt[(size_t)r2] += 1;
    }
    DeviceGuard dg(s->device);
    int4 *d_disp = nullptr;
    unsigned long long *d_out = nullptr;
    const size_t shells = (size_t)r2_max + 1;
    hipError_t e = dalloc(&d_disp, disp.size() * sizeof(int4));
    if (e == hipSuccess) e = dalloc(&d_out, 2 * shells * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMemcpyAsync(d_disp, disp.data(), disp.size() * sizeof(int4), hipMemcpyHostToDevice, s->stream);
    if (e == hipSuccess) e = hipMemsetAsync(d_out, 0, 2 * shells * sizeof(unsigned long long), s->stream);
    if (e == hipSuccess) {
      ka::PairArgs a{};
      a.n = s->n;
      a.n0 = s->n0;
      a.g = s->geom;
      a.planes = s->planes;
      a.disp = d_disp;
      a.n_disp = (int)disp.size();
      a.r2_max = r2_max;
      a.S2 = d_out;
      a.S11 = d_out + shells;
      e = ka::launch_pairs(a, s->wpt, s->stream);
    }
    std::vector<unsigned long long> host(2 * shells);
    if (e == hipSuccess) e = hipMemcpyAsync(host.data(), d_out, 2 * shells * sizeof(unsigned long long), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    (void)hipFree(d_disp);
    (void)hipFree(d_out);
    if (e != hipSuccess) return hip_fail(e, "ka_observe_pairs");
    for (size_t q = 0; q < shells; ++q) {
      if (S2) S2[q] = (int64_t)host[q];
      if (S11) S11[q] = (int64_t)host[shells + q];
      if (count) count[q] = cnt[q];
    }
    return KA_OK;
  });
}

extern "C" int ka_get_state(ka_sim *s, uint64_t *n, uint64_t *n0, uint64_t *f, int64_t *t)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    DeviceGuard dg(s->device);
    const size_t words = (size_t)s->N * s->W;
    std::vector<u64> buf(words);
    uint64_t *outs[3] = {n, n0, f};
    u64 *srcs[3] = {s->n, s->n0, s->f};
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "ka_get_state");
    rc = check_init_flag(s);
    if (rc) return rc;
    for (int k = 0; k < 3; ++k) {
      if (!outs[k]) continue;
      e = hipMemcpyAsync(buf.data(), srcs[k], words * 8, hipMemcpyDeviceToHost, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return hip_fail(e, "ka_get_state copy");
      for (int64_t i = 0; i < s->N; ++i) {
        const int64_t el = s->lattice ? lattice_element(s->geom, i) : s->plan->label[(size_t)i];
        for (int p = 0; p < s->planes; ++p)
          for (int w = 0; w < s->wpt; ++w)
            outs[k][(size_t)(p * s->wpt + w) * s->N + i] = buf[((size_t)p * s->N + el) * s->wpt + w];
      }
    }
    if (t) *t = s->t;
    return KA_OK;
  });
}

extern "C" int ka_set_state(ka_sim *s, const uint64_t *n, const uint64_t *n0, const uint64_t *f,
                            int64_t t)
{
  return ka_guard([&]() -> int {
    int rc = check_sim(s);
    if (rc) return rc;
    if (!n || !n0 || !f) return fail(KA_EINVAL, "ka_set_state needs n, n0 and f");
    if (t < 0 || t >= (1ll << 32)) return fail(KA_EINVAL, "t out of range");
    DeviceGuard dg(s->device);
    const size_t words = (size_t)s->N * s->W;
    std::vector<u64> buf(words);
    const uint64_t *ins[3] = {n, n0, f};
    u64 *dsts[3] = {s->n, s->n0, s->f};
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "ka_set_state");
    for (int k = 0; k < 3; ++k) {
      for (int64_t i = 0; i < s->N; ++i) {
        const int64_t el = s->lattice ? lattice_element(s->geom, i) : s->plan->label[(size_t)i];
        for (int p = 0; p < s->planes; ++p)
          for (int w = 0; w < s->wpt; ++w)
            buf[((size_t)p * s->N + el) * s->wpt + w] = ins[k][(size_t)(p * s->wpt + w) * s->N + i];
      }
      e = hipMemcpyAsync(dsts[k], buf.data(), words * 8, hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return hip_fail(e, "ka_set_state copy");
    }
    // the new f may have fewer bits: forget which elements were known to be full
    if (s->fsat) {
      e = hipMemsetAsync(s->fsat, 0, fsat_bytes(s->N, s->R), s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return hip_fail(e, "ka_set_state summary");
    }
    s->t = t;
    return KA_OK;
  });
}

extern "C" int ka_sim_info(const ka_sim *s, int64_t *N, int *n_replicas, int64_t *K, int *m,
                           int64_t *t, int *n_classes)
{
  return ka_guard([&]() -> int {
    if (!s) return fail(KA_EINVAL, "sim is NULL");
    if (N) *N = s->N;
    if (n_replicas) *n_replicas = s->R;
    if (K) *K = s->K;
    if (m) *m = s->m;
    if (t) *t = s->t;
    if (n_classes) *n_classes = s->C;
    return KA_OK;
  });
}

extern "C" int ka_set_option(ka_sim *s, int option, int64_t value)
{
  return ka_guard([&]() -> int {
    if (!s) return fail(KA_EINVAL, "sim is NULL");
    if (s->batch) return fail(KA_ESTATE, "sim is a batch member");
    if (option == KA_OPT_PATH) {
      if (value < 0 || value > 2) return fail(KA_EINVAL, "path must be 0, 1 or 2");
      if (value == 2 && !s->lds_fits) return fail(KA_EINVAL, "instance does not fit in LDS");
      s->path_opt = (int)value;
      return KA_OK;
    }
    if (option == KA_OPT_TIMING) {
      if (value < 0) return fail(KA_EINVAL, "timing interval must be >= 0");
      s->timing_every = value;
      return KA_OK;
    }
    if (option == KA_OPT_NOISE) {
      if (value != 0 && value != 1) return fail(KA_EINVAL, "noise must be 0 or 1");
      s->noise = (int)value;
      return KA_OK;
    }
    if (option == KA_OPT_PLANE_STREAMS) {
      if (value != 0 && value != 1) return fail(KA_EINVAL, "plane streams must be 0 or 1");
      s->plane_streams = (int)value;
      return KA_OK;
    }
    if (option == KA_OPT_PLANE_GROUPS) {
      if (value < -1 || value > s->planes) return fail(KA_EINVAL, "plane group must be -1, 0 or 1..%d", s->planes);
      s->plane_group_opt = (int)value;
      return KA_OK;
    }
    if (option == KA_OPT_TAIL) {
      if (value != 0 && value != 1) return fail(KA_EINVAL, "tail merging must be 0 or 1");
      s->tail_opt = (int)value;
      return KA_OK;
    }
    return fail(KA_EINVAL, "unknown option %d", option);
  });
}

extern "C" int ka_timing(ka_sim *s, int64_t *launches, int64_t *timed, double *timed_ms)
{
  return ka_guard([&]() -> int {
    if (!s) return fail(KA_EINVAL, "sim is NULL");
    DeviceGuard dg(s->device);
    hipError_t e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return hip_fail(e, "ka_timing");
    harvest_timing(s);
    if (launches) *launches = s->launches;
    if (timed) *timed = s->timed;
    if (timed_ms) *timed_ms = s->timed_ms;
    return KA_OK;
  });
}

extern "C" int ka_sim_path(const ka_sim *s, int *path)
{
  return ka_guard([&]() -> int {
    if (!s || !path) return fail(KA_EINVAL, "NULL argument");
    *path = use_lds(s) ? 2 : 1;
    return KA_OK;
  });
}

extern "C" void ka_free(ka_sim *s)
{
  try {
    if (!s) return;
    if (s->batch) (void)ka_batch_release_member(s->batch, s);
    DeviceGuard dg(s->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    release_plane_streams(s);
    harvest_timing(s);
    for (hipEvent_t ev : s->event_pool) (void)hipEventDestroy(ev);
    free_device(s);
    if (s->own_stream) (void)hipStreamDestroy(s->stream);
    delete s;
  } catch (...) {
  }
}

// ------------------------------------------------------------------------------------
// Host-side quantities derived from the counts (Sec. 2.2, Sec. 3.1).
// ------------------------------------------------------------------------------------
extern "C" int ka_particles(int64_t N, double rho, int64_t *K)
{
  return ka_guard([&]() -> int {
    if (!K) return fail(KA_EINVAL, "K is NULL");
    if (N < 1) return fail(KA_EINVAL, "N must be positive");
    if (!(rho >= 0.0 && rho <= 1.0)) return fail(KA_EINVAL, "density rho must be in [0, 1]");
    *K = (int64_t)std::floor(rho * (double)N + 0.5);
    return KA_OK;
  });
}

extern "C" int ka_derived(int64_t N, int64_t K, int n_replicas, int n_rows, const int64_t *overlap,
                          const int64_t *persistence, double *C, double *chi4, double *P)
{
  return ka_guard([&]() -> int {
    if (N < 1 || K < 0 || K > N || n_replicas < 1 || n_rows < 0) return fail(KA_EINVAL, "bad sizes");
    if ((C || chi4) && !overlap) return fail(KA_EINVAL, "overlap is NULL");
    if (P && !persistence) return fail(KA_EINVAL, "persistence is NULL");
    const double nan = std::nan("");
    const double r = (double)K / (double)N;
    for (int q = 0; q < n_rows; ++q) {
      if (C || chi4) {
        double sum = 0.0, sum2 = 0.0;
        if (K > 0 && K < N) {
          for (int b = 0; b < n_replicas; ++b) {
            const double qb = ((double)overlap[(size_t)q * n_replicas + b] / (double)N - r * r) / (r * (1.0 - r));
            sum += qb;
            sum2 += qb * qb;
          }
        }
        const double mean = sum / n_replicas;
        if (C) C[q] = (K > 0 && K < N) ? mean : nan;
        if (chi4) chi4[q] = (K > 0 && K < N) ? (double)N * (sum2 / n_replicas - mean * mean) : nan;
      }
      if (P) {
        double sum = 0.0;
        for (int b = 0; b < n_replicas; ++b) sum += (double)persistence[(size_t)q * n_replicas + b];
        P[q] = K > 0 ? sum / n_replicas / (double)K : nan;
      }
    }
    return KA_OK;
  });
}

extern "C" int ka_g4(int64_t N, int64_t K, int n_replicas, int n_shells, const int64_t *S2,
                     const int64_t *S11, double *g4)
{
  return ka_guard([&]() -> int {
    if (N < 1 || K < 0 || K > N || n_replicas < 1 || n_shells < 0) return fail(KA_EINVAL, "bad sizes");
    if (n_shells > 0 && (!S2 || !S11 || !g4)) return fail(KA_EINVAL, "NULL argument");
    const double r = (double)K / (double)N;
    const double R = (double)n_replicas;
    const double norm = (double)N * r * r * (1.0 - r) * (1.0 - r);
    for (int k = 0; k < n_shells; ++k)
      g4[k] = (K > 0 && K < N) ? ((double)S2[k] / R - (double)S11[k] / (R * R)) / norm : std::nan("");
    return KA_OK;
  });
}

extern "C" const char *ka_last_error(void) { return g_err.c_str(); }
