// ka_plan.cpp -- device schedule of a general graph: vertex numbering, class-sorted edge
// records and neighbour lists (host side of libka).
//
// Method: Boccagna, arXiv 1710.05155 (Sec. 2.1 graphs).  The dynamics does not depend on the
// numbering: the canonical vertex and edge ids keep every result the same, and the numbering
// only places the state words so that a class pass's gathers share cache lines.
#include <algorithm>
#include <memory>
#include <mutex>
#include <new>
#include <utility>
#include <vector>

#include "ka_internal.h"
#include "ka_objects.h"

namespace {

// Vertex parts for XCD-local gathers.  The 8 XCDs each have their own L2 and take
// contiguous ranges of a pass's workgroups, so a class pass whose edges are ordered by part
// gathers mostly from the XCD's own part.  P parts of at most ceil(N/P) vertices are grown
// breadth-first from P seed vertices in turn (a part whose frontier runs dry restarts at the
// next unassigned vertex), then refined: a vertex moves to the part holding most of its
// neighbours if that part stays within 2% of N/P.  Deterministic.
std::vector<int> partition_vertices(const ka_graph *g, int P)
{
  const int64_t N = g->N;
  const int z = g->z;
  std::vector<int> part((size_t)N, -1);
  if (P <= 1) {
    std::fill(part.begin(), part.end(), 0);
    return part;
  }
  const int64_t cap = (N + P - 1) / P;
  std::vector<int64_t> size((size_t)P, 0);
  std::vector<std::vector<int32_t>> front((size_t)P);
  std::vector<size_t> head((size_t)P, 0);
  int64_t scan = 0;
  auto claim = [&](int q, int32_t v) {
    part[(size_t)v] = q;
    ++size[(size_t)q];
    front[(size_t)q].push_back(v);
  };
  for (int q = 0; q < P; ++q) claim(q, (int32_t)((int64_t)q * N / P));
  for (bool grew = true; grew;) {
    grew = false;
    for (int q = 0; q < P; ++q) {
      for (int step = 0; step < 64 && size[(size_t)q] < cap; ++step) {
        if (head[(size_t)q] == front[(size_t)q].size()) {
          while (scan < N && part[(size_t)scan] >= 0) ++scan;
          if (scan == N) break;
          claim(q, (int32_t)scan);
        }
        const int32_t v = front[(size_t)q][head[(size_t)q]++];
        for (int k = 0; k < z && size[(size_t)q] < cap; ++k) {
          const int32_t w = g->adj[(size_t)v * z + k];
          if (part[(size_t)w] < 0) claim(q, w);
        }
        grew = true;
      }
    }
  }
  for (int64_t v = 0; v < N; ++v)
    if (part[(size_t)v] < 0) {
      const int q = (int)(std::min_element(size.begin(), size.end()) - size.begin());
      part[(size_t)v] = q;
      ++size[(size_t)q];
    }
  const int64_t hi = cap + cap / 50, lo = cap - cap / 50;
  std::vector<int> cnt((size_t)P);
  for (int it = 0; it < 8; ++it) {
    int64_t moved = 0;
    for (int64_t v = 0; v < N; ++v) {
      std::fill(cnt.begin(), cnt.end(), 0);
      for (int k = 0; k < z; ++k) ++cnt[(size_t)part[(size_t)g->adj[(size_t)v * z + k]]];
      const int cur = part[(size_t)v];
      int best = cur;
      for (int q = 0; q < P; ++q)
        if (cnt[(size_t)q] > cnt[(size_t)best]) best = q;
      if (best != cur && size[(size_t)best] < hi && size[(size_t)cur] > lo) {
        part[(size_t)v] = best;
        ++size[(size_t)best];
        --size[(size_t)cur];
        ++moved;
      }
    }
    if (moved == 0) break;
  }
  return part;
}

// Part of the XCD that updates canonical edge q with endpoints in parts pu, pv: their common
// part, else alternately one endpoint's part (by the parity of q), which balances the parts.
int edge_owner_part(int pu, int pv, int64_t q) { return pu == pv || (q & 1) == 0 ? pu : pv; }

constexpr int kGraphParts = 8;              // one per XCD
constexpr int64_t kGraphPartMinN = 1 << 19; // below this a word plane fits one 4 MB L2

}  // namespace

// The device schedule of a general graph (see GraphPlan), built on first use and kept in the
// graph: later ka_init calls on the same graph only copy it to the device.  Returns null if
// host memory runs out.
std::shared_ptr<const GraphPlan> graph_plan(const ka_graph *g)
{
  std::lock_guard<std::mutex> lock(g->plan_mu);
  if (g->plan) return g->plan;
  try {
    auto p = std::make_shared<GraphPlan>();
    // Device numbering of the vertices: part by part (see partition_vertices), then by the
    // set of parts whose XCDs read the vertex, breadth-first inside each group.
    const int64_t Nv = g->N;
    const int z = g->z;
    const std::vector<int> part = partition_vertices(g, Nv >= kGraphPartMinN ? kGraphParts : 1);
    std::vector<int32_t> &label = p->label;
    std::vector<int32_t> &site_of = p->site_of;
    std::vector<int32_t> bfs;
    bfs.reserve((size_t)Nv);
    label.assign((size_t)Nv, -1);
    site_of.resize((size_t)Nv);
    for (int64_t root = 0; root < Nv; ++root) {
      if (label[(size_t)root] >= 0) continue;
      size_t h = bfs.size();
      label[(size_t)root] = 0;
      bfs.push_back((int32_t)root);
      while (h < bfs.size()) {
        const int32_t v = bfs[h++];
        for (int k = 0; k < z; ++k) {
          const int32_t w = g->adj[(size_t)v * z + k];
          if (label[(size_t)w] < 0) {
            label[(size_t)w] = 0;
            bfs.push_back(w);
          }
        }
      }
    }
    {
      // Inside a part, vertices are grouped by the set of parts whose XCDs read them in some
      // class pass (breadth-first order inside a group).  The XCD of part x reads the closed
      // neighbourhoods of both endpoints of the edges x owns (owner rule below), so it
      // gathers from another part only that part's vertices within two steps of x's edges;
      // grouped, those share cache lines (on a 2^20-vertex z=4 graph a vertex is read by
      // about 4 of the 8 XCDs, and the grouping leaves about a third fewer lines per pass).
      std::vector<uint32_t> readers((size_t)Nv, 0);
      const int64_t Ecount = (int64_t)g->eu.size();
      for (int64_t q = 0; q < Ecount; ++q) {
        const int32_t a = g->eu[(size_t)q], b = g->ev[(size_t)q];
        const uint32_t bit = 1u << edge_owner_part(part[(size_t)a], part[(size_t)b], q);
        for (const int32_t x : {a, b}) {
          readers[(size_t)x] |= bit;
          for (int k = 0; k < z; ++k) readers[(size_t)g->adj[(size_t)x * z + k]] |= bit;
        }
      }
      const int groups = kGraphParts << kGraphParts;   // (part, reader set)
      auto group = [&](int32_t v) { return ((size_t)part[(size_t)v] << kGraphParts) | readers[(size_t)v]; };
      std::vector<int64_t> start((size_t)groups + 1, 0);
      for (int64_t v = 0; v < Nv; ++v) ++start[group((int32_t)v) + 1];
      for (int q = 0; q < groups; ++q) start[(size_t)q + 1] += start[(size_t)q];
      for (const int32_t v : bfs) {
        const int64_t id = start[group(v)]++;
        label[(size_t)v] = (int32_t)id;
        site_of[(size_t)id] = v;
      }
    }
    // class-sorted edge records (u, v, e, 0) in device numbering, canonical edge id e;
    // inside a class ordered by the smaller endpoint (any order gives the same result)
    const int64_t E = (int64_t)g->eu.size();
    std::vector<int> &cs = p->class_start;
    cs.assign((size_t)g->C + 1, 0);
    for (int64_t q = 0; q < E; ++q) cs[(size_t)g->ecls[q] + 1]++;
    for (int c = 0; c < g->C; ++c) cs[(size_t)c + 1] += cs[(size_t)c];
    std::vector<int> fill(cs.begin(), cs.end() - 1);
    std::vector<int4> &rec = p->rec;
    rec.resize((size_t)E);
    for (int64_t q = 0; q < E; ++q)
      rec[(size_t)fill[(size_t)g->ecls[q]]++] =
          make_int4(label[(size_t)g->eu[q]], label[(size_t)g->ev[q]], (int)q, (int)g->ecls[q]);
    // Owner of an edge: its endpoints' part when they share one (key: the smaller endpoint
    // number); else, alternating with the canonical id, one endpoint's part (key: that
    // endpoint's number).  Inside a class, edges go by owner part, then by key.
    auto owner = [&](const int4 &r) {
      const int pu = part[(size_t)site_of[(size_t)r.x]], pv = part[(size_t)site_of[(size_t)r.y]];
      const int po = edge_owner_part(pu, pv, r.z);
      if (pu == pv) return std::make_pair(po, std::min(r.x, r.y));
      return po == pu ? std::make_pair(po, r.x) : std::make_pair(po, r.y);
    };
    for (int c = 0; c < g->C; ++c)
      std::sort(rec.begin() + cs[(size_t)c], rec.begin() + cs[(size_t)c + 1],
                [&](const int4 &x, const int4 &y) {
                  const auto ox = owner(x), oy = owner(y);
                  return ox != oy ? ox < oy : x.z < y.z;
                });
    // Neighbour lists of every record, slot-major: slot q < z-1 is the q-th neighbour of u
    // other than v, slot z-1+q the q-th neighbour of v other than u (device numbering).
    const int K = z - 1;
    std::vector<int32_t> &nbr = p->nbr;
    nbr.resize((size_t)2 * K * (size_t)E);
    for (int64_t k = 0; k < E; ++k) {
      const int32_t ends[2] = {rec[(size_t)k].x, rec[(size_t)k].y};
      for (int side = 0; side < 2; ++side) {
        const int32_t a_end = site_of[(size_t)ends[side]], b_end = site_of[(size_t)ends[1 - side]];
        int q = 0;
        for (int j = 0; j < z; ++j) {
          const int32_t w = g->adj[(size_t)a_end * z + j];
          if (w == b_end) continue;
          nbr[(size_t)(side * K + q++) * (size_t)E + (size_t)k] = label[(size_t)w];
        }
      }
    }
    g->plan = std::move(p);
  } catch (const std::bad_alloc &) {
    return nullptr;
  }
  return g->plan;
}
