// ka_batch.hip -- one kernel launch applies one class pass to every active instance of a
// batch (gfx950).  Method: Boccagna, arXiv 1710.05155; the per-edge bit logic is the same
// device code as the single-instance passes (ka_device.h), so a member's result does not
// depend on what else is in the batch.
//
// Work list: every member contributes planes x ceil(threads of its current class / BLOCK)
// tiles of BLOCK threads.  The tile prefix over members for the current step lives in
// BatchCtl; each workgroup copies it to LDS and takes one contiguous range of tiles
// (ranges ordered so that each XCD holds a contiguous part of the work).  The last
// workgroup to finish advances the global step and builds the next step's prefix, so a
// captured graph of identical launches replays any number of steps without host work.
#include "ka_device.h"

namespace ka {
namespace {

using namespace dev;

// Lower-endpoint sublattice number q of lattice class (mu, r): the residues of the other
// directions are the base-4 digits of q, and a_mu = (r - 2 * their sum) mod 4.  Any
// enumeration of the class's sublattices gives the same result (its edges commute).
__device__ __forceinline__ int class_sublattice(int D, int mu, int r, int q)
{
  int a[3] = {0, 0, 0};
  int rest = q, others = 0;
  for (int nu = 0; nu < D; ++nu) {
    if (nu == mu) continue;
    a[nu] = rest & 3;
    rest >>= 2;
    others += a[nu];
  }
  a[mu] = (r - 2 * others) & 3;
  return a[0] + 4 * a[1] + 16 * a[2];
}

template <int BLOCK>
__device__ __forceinline__ int tiles_per_plane(const BatchMember &mb, int c)
{
  if (mb.kind == 0) {
    const int nsub = mb.d == 2 ? 4 : 16;
    const int threads = nsub * 64 * ((mb.P + 63) / 64);
    return (threads + BLOCK - 1) / BLOCK;
  }
  const int count = mb.class_start[c + 1] - mb.class_start[c];
  return (count + BLOCK - 1) / BLOCK;
}

template <int BLOCK>
__device__ __forceinline__ int member_tiles(const BatchMember &mb, long long s)
{
  if (s < mb.s_begin || s >= mb.s_end) return 0;
  const int c = (int)((s - mb.s_begin) % mb.C);
  return mb.planes * tiles_per_plane<BLOCK>(mb, c);
}

// Block-wide exclusive prefix of member tiles at step s into out[0..n] (out[n] = total).
template <int BLOCK>
__device__ void build_prefix(const BatchMember *mem, int n, long long s, int *out, int *scratch)
{
  const int tid = (int)threadIdx.x;
  // each thread sums a contiguous run of members, then a scan over thread totals
  const int per = (n + BLOCK - 1) / BLOCK;
  const int b0 = tid * per, b1 = min(n, b0 + per);
  int local = 0;
  for (int k = b0; k < b1; ++k) local += member_tiles<BLOCK>(mem[k], s);
  scratch[tid] = local;
  __syncthreads();
  if (tid == 0) {
    int acc = 0;
    for (int q = 0; q < BLOCK; ++q) {
      const int v = scratch[q];
      scratch[q] = acc;
      acc += v;
    }
    out[n] = acc;
  }
  __syncthreads();
  int acc = scratch[tid];
  for (int k = b0; k < b1; ++k) {
    out[k] = acc;
    acc += member_tiles<BLOCK>(mem[k], s);
  }
  __syncthreads();
}

template <int BLOCK>
__device__ __forceinline__ void run_lattice_tile(const BatchMember &mb, int local, int c, uint32_t t)
{
  const int nsub = mb.d == 2 ? 4 : 16;
  const int bpp = tiles_per_plane<BLOCK>(mb, c);
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
  const size_t off = (size_t)plane * (size_t)mb.N * (size_t)mb.wpt;
  u64 *n = mb.n + off, *f = mb.f + off;
  if (mb.d == 2) {
    if (mb.wpt == 2) {
      if (mu == 0) lattice_edge<2, 0, 2>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
      else lattice_edge<2, 1, 2>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
    } else {
      if (mu == 0) lattice_edge<2, 0, 1>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
      else lattice_edge<2, 1, 1>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
    }
  } else {
    if (mb.wpt == 2) {
      if (mu == 0) lattice_edge<3, 0, 2>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
      else if (mu == 1) lattice_edge<3, 1, 2>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
      else lattice_edge<3, 2, 2>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
    } else {
      if (mu == 0) lattice_edge<3, 0, 1>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
      else if (mu == 1) lattice_edge<3, 1, 1>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
      else lattice_edge<3, 2, 1>(n, f, g, sub, pos, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1);
    }
  }
}

template <int BLOCK>
__device__ __forceinline__ void run_graph_tile(const BatchMember &mb, int local, int c, uint32_t t)
{
  const int b0 = mb.class_start[c];
  const int count = mb.class_start[c + 1] - b0;
  const int bpp = (count + BLOCK - 1) / BLOCK;
  const int plane = local / bpp;
  const int blk = local - plane * bpp;
  const int k = blk * BLOCK + (int)threadIdx.x;
  if (k >= count) return;
  const size_t off = (size_t)plane * (size_t)mb.N * (size_t)mb.wpt;
  u64 *n = mb.n + off, *f = mb.f + off;
  const int4 E = mb.edges[b0 + k];
  switch (mb.z * 4 + mb.wpt) {
    case 3 * 4 + 1: graph_edge<3, 1>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 3 * 4 + 2: graph_edge<3, 2>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 4 * 4 + 1: graph_edge<4, 1>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 4 * 4 + 2: graph_edge<4, 2>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 5 * 4 + 1: graph_edge<5, 1>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 5 * 4 + 2: graph_edge<5, 2>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 6 * 4 + 1: graph_edge<6, 1>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    case 6 * 4 + 2: graph_edge<6, 2>(n, f, mb.adj, E, plane, mb.m, t, (uint32_t)c, mb.key0, mb.key1); break;
    default: break;
  }
}

// After the member table changed: set the member count and rebuild the work list of the
// step the next step kernel executes.  The tile size is BLOCK of the step kernels that
// follow, so this kernel is launched with the same BLOCK.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_prepare(BatchCtl *ctl, const BatchMember *mem, int n)
{
  __shared__ int scratch[BLOCK];
  const long long s = ctl->step;
  build_prefix<BLOCK>(mem, n, s, ctl->prefix, scratch);
  if (threadIdx.x == 0) {
    ctl->n_members = n;
    ctl->done = 0;
  }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_batch_step(BatchCtl *ctl, const BatchMember *mem)
{
  __shared__ int sp[kBatchMaxMembers + 1];
  __shared__ int scratch[BLOCK];
  __shared__ long long s_step;
  __shared__ int s_n;
  __shared__ int s_last;
  const int tid = (int)threadIdx.x;
  if (tid == 0) {
    s_step = ctl->step;
    s_n = ctl->n_members;
  }
  __syncthreads();
  const long long s = s_step;
  const int n = s_n;
  for (int k = tid; k <= n; k += BLOCK) sp[k] = ctl->prefix[k];
  __syncthreads();
  const int total = sp[n];
  const int G = (int)gridDim.x;
  const int lb = xcd_remap((int)blockIdx.x, G);
  const int per = (total + G - 1) / G;
  const int t_begin = lb * per;
  const int t_end = min(total, t_begin + per);
  for (int tile = t_begin; tile < t_end; ++tile) {
    // member holding this tile: the last k with sp[k] <= tile (members with no tiles have
    // sp[k] == sp[k+1] and are skipped by taking the last such k)
    int lo = 0, hi = n - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (sp[mid] <= tile) lo = mid;
      else hi = mid - 1;
    }
    const BatchMember mb = mem[lo];
    const int local = tile - sp[lo];
    const long long rel = s - mb.s_begin;
    const int c = (int)(rel % mb.C);
    const uint32_t t = mb.t0 + (uint32_t)(rel / mb.C);
    if (mb.kind == 0) run_lattice_tile<BLOCK>(mb, local, c, t);
    else run_graph_tile<BLOCK>(mb, local, c, t);
  }
  // the last workgroup to finish advances the step and prepares the next work list
  __syncthreads();
  if (tid == 0) {
    __threadfence();
    const unsigned old = atomicAdd(&ctl->done, 1u);
    s_last = (old == (unsigned)(G - 1));
  }
  __syncthreads();
  if (s_last) {
    __threadfence();
    build_prefix<BLOCK>(mem, n, s + 1, ctl->prefix, scratch);
    if (tid == 0) {
      ctl->step = s + 1;
      ctl->done = 0;
    }
  }
}

}  // namespace

hipError_t launch_batch_prepare(BatchCtl *ctl, const BatchMember *mem, int n_members, int block,
                                hipStream_t s)
{
  switch (block) {
    case 128: hipLaunchKernelGGL((k_batch_prepare<128>), dim3(1), dim3(128), 0, s, ctl, mem, n_members); break;
    case 256: hipLaunchKernelGGL((k_batch_prepare<256>), dim3(1), dim3(256), 0, s, ctl, mem, n_members); break;
    case 512: hipLaunchKernelGGL((k_batch_prepare<512>), dim3(1), dim3(512), 0, s, ctl, mem, n_members); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_batch_step(BatchCtl *ctl, const BatchMember *mem, int block, int grid, hipStream_t s)
{
  switch (block) {
    case 128: hipLaunchKernelGGL((k_batch_step<128>), dim3(grid), dim3(128), 0, s, ctl, mem); break;
    case 256: hipLaunchKernelGGL((k_batch_step<256>), dim3(grid), dim3(256), 0, s, ctl, mem); break;
    case 512: hipLaunchKernelGGL((k_batch_step<512>), dim3(grid), dim3(512), 0, s, ctl, mem); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ka
