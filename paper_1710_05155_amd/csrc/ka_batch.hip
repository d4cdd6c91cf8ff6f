// ka_batch.hip -- one kernel launch applies one class pass to every active instance of a
// batch (gfx950).  Method: Boccagna, arXiv 1710.05155; the per-edge bit logic is the same
// device code as the single-instance passes (ka_device.h), so a member's result does not
// depend on what else is in the batch.
//
// Work list: between membership changes ("segments") every member owns a fixed number of
// tiles of BLOCK threads per step: planes x tiles per plane, where a lattice class always
// has the same size and a graph member is padded to its largest class (workgroups past the
// current class exit at once).  The prepare kernel writes the tile -> (member, local tile)
// table of a segment; each step kernel then runs one workgroup per tile, mapped so that
// each XCD holds a contiguous range of tiles (stencil halos meet in its L2).  The step
// index is a device base plus the launch's offset, so a captured graph of G step kernels
// followed by one "base += G" kernel replays any number of steps.
#include "ka_device.h"

namespace ka {
namespace {

using namespace dev;

template <int BLOCK, int WPT>
__device__ __forceinline__ void run_lattice_tile(const BatchMember &mb, int local, int c, uint32_t t)
{
  const int nsub = mb.d == 2 ? 4 : 16;
  const int bpp = mb.tiles_per_plane;
  const int plane = local / bpp;
  const int blk = local - plane * bpp;
  const int gid = blk * BLOCK + (int)threadIdx.x;
  const int span = nsub * 64;
  const int chunk = gid / span;
  const int rem = gid - chunk * span;
  const int q = rem >> 6;
  const int pos = chunk * 64 + (rem & 63);
  if (pos >= mb.P) return;
  const int mu = c >> 2, r = c & 3;
  const int sub = class_sublattice(mb.d, mu, r, q);
  LatticeGeom g;
  g.d = mb.d;
  g.L = mb.L;
  g.Q = mb.Q;
  g.P = mb.P;
  g.N = mb.N;
  g.qinv = mb.qinv;
  const size_t off = (size_t)plane * (size_t)mb.N * WPT;
  u64 *n = mb.n + off, *f = mb.f + off;
  if (mb.d == 2) {
    if (mu == 0) lattice_edge<2, 0, WPT>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise);
    else lattice_edge<2, 1, WPT>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise);
  } else {
    if (mu == 0) lattice_edge<3, 0, WPT>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise);
    else if (mu == 1) lattice_edge<3, 1, WPT>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise);
    else lattice_edge<3, 2, WPT>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise);
  }
}

// One edge of a graph member (entry k of its class-sorted list, class c).
template <int WPT>
__device__ __forceinline__ void member_graph_edge(const BatchMember &mb, u64 *n, u64 *f, int plane, int k,
                                                  int c, uint32_t t)
{
  const size_t st = (size_t)mb.stride;
  if (mb.fsat) {
    const FSat sat{mb.fsat, plane * mb.N};
    switch (mb.z) {
      case 3: graph_edge<3, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise, sat); break;
      case 4: graph_edge<4, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise, sat); break;
      case 5: graph_edge<5, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise, sat); break;
      case 6: graph_edge<6, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise, sat); break;
      default: break;
    }
    return;
  }
  switch (mb.z) {
    case 3: graph_edge<3, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise); break;
    case 4: graph_edge<4, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise); break;
    case 5: graph_edge<5, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise); break;
    case 6: graph_edge<6, WPT>(n, f, mb.edges, mb.nbr, st, k, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1, mb.noise); break;
    default: break;
  }
}

template <int BLOCK, int WPT>
__device__ __forceinline__ void run_graph_tile(const BatchMember &mb, int local, int c, uint32_t t)
{
  const int bpp = mb.tiles_per_plane;
  const int plane = local / bpp;
  const int blk = local - plane * bpp;
  const size_t off = (size_t)plane * (size_t)mb.N * WPT;
  u64 *n = mb.n + off, *f = mb.f + off;
  if (c == mb.C - 1 && mb.classes > mb.C) {
    // the merged run of tiny trailing classes: the plane's first tile takes them in order,
    // with a workgroup barrier between classes (as in the single-instance tail launch; the
    // condition is the same for every thread of the workgroup)
    if (blk != 0) return;
    for (int cc = c; cc < mb.classes; ++cc) {
      const int b0 = mb.class_start[cc], b1 = mb.class_start[cc + 1];
      for (int k = b0 + (int)threadIdx.x; k < b1; k += BLOCK) member_graph_edge<WPT>(mb, n, f, plane, k, cc, t);
      __syncthreads();
    }
    return;
  }
  const int b0 = mb.class_start[c];
  const int count = mb.class_start[c + 1] - b0;
  const int k = blk * BLOCK + (int)threadIdx.x;
  if (k >= count) return;
  member_graph_edge<WPT>(mb, n, f, plane, b0 + k, c, t);
}

// Tile table of the segment that starts at `step`: members with `wpt` words per thread
// that are active at `step` own planes x tiles_per_plane consecutive tiles, in member
// order.  One workgroup; the total is written to *total.
__global__ __launch_bounds__(1024) void k_batch_prepare(const BatchMember *mem, int n, long long step, int wpt,
                                                        BatchTiles tiles, int *total)
{
  __shared__ int start[kBatchMaxMembers + 1];
  const int tid = (int)threadIdx.x;
  if (tid == 0) {
    int acc = 0;
    for (int k = 0; k < n; ++k) {
      start[k] = acc;
      const BatchMember &mb = mem[k];
      if (mb.wpt == wpt && step >= mb.s_begin && step < mb.s_end) acc += mb.planes * mb.tiles_per_plane;
    }
    start[n] = acc;
    *total = acc;
  }
  __syncthreads();
  for (int k = 0; k < n; ++k) {
    const int a = start[k], b = min(start[k + 1], tiles.cap);
    for (int q = a + tid; q < b; q += (int)blockDim.x) {
      tiles.member[q] = k;
      tiles.local[q] = q - a;
    }
  }
  // The host computes the same total from the same table; should they ever differ, tiles
  // past the total run nothing instead of reading stale entries.
  for (int q = start[n] + tid; q < tiles.cap; q += (int)blockDim.x) {
    tiles.member[q] = -1;
    tiles.local[q] = 0;
  }
}

template <int BLOCK, int WPT>
__global__ __launch_bounds__(BLOCK) void k_batch_step(const BatchMember *mem, BatchTiles tiles,
                                                           const long long *base, int offset)
{
  const int tile = xcd_remap((int)blockIdx.x, (int)gridDim.x);
  const long long s = *base + offset;
  const int k = tiles.member[tile];
  if (k < 0) return;
  const int local = tiles.local[tile];
  const BatchMember mb = mem[k];
  if (s < mb.s_begin || s >= mb.s_end) return;
  const long long rel = s - mb.s_begin;
  const int c = (int)(rel % mb.C);
  const uint32_t t = mb.t0 + (uint32_t)(rel / mb.C);
  if (mb.kind == 0) run_lattice_tile<BLOCK, WPT>(mb, local, c, t);
  else run_graph_tile<BLOCK, WPT>(mb, local, c, t);
}

__global__ void k_batch_advance(long long *base, int by)
{
  if (threadIdx.x == 0 && blockIdx.x == 0) *base += by;
}

}  // namespace

hipError_t launch_batch_prepare(const BatchMember *mem, int n_members, long long step, int wpt,
                                BatchTiles tiles, int *total, hipStream_t s)
{
  hipLaunchKernelGGL(k_batch_prepare, dim3(1), dim3(1024), 0, s, mem, n_members, step, wpt, tiles, total);
  return hipGetLastError();
}

hipError_t launch_batch_step(const BatchMember *mem, BatchTiles tiles, int n_tiles, const long long *base,
                             int offset, int block, int wpt, hipStream_t s)
{
  if (n_tiles <= 0) return hipErrorInvalidValue;
#define KA_BS(B, W) \
  hipLaunchKernelGGL((k_batch_step<B, W>), dim3(n_tiles), dim3(B), 0, s, mem, tiles, base, offset)
  switch (block * 4 + wpt) {
    case 128 * 4 + 1: KA_BS(128, 1); break;
    case 128 * 4 + 2: KA_BS(128, 2); break;
    case 256 * 4 + 1: KA_BS(256, 1); break;
    case 256 * 4 + 2: KA_BS(256, 2); break;
    case 512 * 4 + 1: KA_BS(512, 1); break;
    case 512 * 4 + 2: KA_BS(512, 2); break;
    default: return hipErrorInvalidValue;
  }
#undef KA_BS
  return hipGetLastError();
}

hipError_t launch_batch_advance(long long *base, int by, hipStream_t s)
{
  hipLaunchKernelGGL(k_batch_advance, dim3(1), dim3(64), 0, s, base, by);
  return hipGetLastError();
}

}  // namespace ka
