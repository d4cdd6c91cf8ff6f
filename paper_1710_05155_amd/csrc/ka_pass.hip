// ka_pass.hip -- global-memory class passes, observables and initial state (gfx950).
//
// Method: Boccagna, arXiv 1710.05155; the per-edge bit logic lives in ka_device.h.
#include <mutex>

#include "ka_device.h"

// Fixed device scratch of the observation entry point that allocates nothing (see
// observe_scratch_setup below): one copy per device, held until the process ends.
static __device__ __align__(256) unsigned long long scratch[ka::kObserveScratchWords];

namespace ka {
namespace {

using namespace dev;

constexpr int kPassBlock = 256;
constexpr int kObsBlock = 256;
// Graph classes are uneven (greedy colouring): a class with fewer edges than this (over all
// planes) runs in 64-thread workgroups, which spread it over more CUs; larger ones in
// kPassBlock-thread workgroups.
constexpr int kGraphSmallBlock = 64;
constexpr long long kGraphSmallEdges = 65536;

// ------------------------------------------------------------------------------------
// Global-memory class pass kernels: one launch per (class, sweep) over a range of planes.
// ------------------------------------------------------------------------------------
// Thread order: a wave covers 64 consecutive positions of one lower-endpoint sublattice
// (coalesced 64 x 16 B loads); consecutive waves cover the class's other lower-endpoint
// sublattices at the same positions, so the neighbour sublattices they share are fetched
// once and then served from L2 (together with the XCD-contiguous block order).
template <int D, int MU, int WPT>
__global__ __launch_bounds__(kPassBlock) void k_pass_lattice(PassLattice a, int m)
{
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int pl = lin / a.blocks_per_plane;
  const int blk = lin - pl * a.blocks_per_plane;
  const int plane = a.plane0 + pl;
  const int gid = blk * kPassBlock + (int)threadIdx.x;
  constexpr int nsub = D == 2 ? 4 : 16;   // lower-endpoint sublattices per class
  const int span = nsub * 64;              // threads per 64-position chunk
  const int chunk = gid / span;
  const int rem = gid - chunk * span;
  // Waves are 64-thread aligned and span is a multiple of 64, so q is the same on every lane
  // of the wave: take it (and the sublattice) in scalar registers.
  const int q = __builtin_amdgcn_readfirstlane(rem >> 6);
  int chk = chunk;
  if (D == 3 && a.row_tile_log2 > 0) {
    // Rows (p1, p2) of whole chunks visited in tiles of T = 2^row_tile_log2 rows along p1,
    // p2 next: the +-e_2 neighbour rows are then T rows apart instead of Q (inside one L2),
    // at the cost of the +-e_1 neighbours at tile edges.  A permutation of the chunks.
    const int lt = a.row_tile_log2, lq = a.q_log2, lr = lq - 6;
    const int row = chk >> lr, xc = chk & ((1 << lr) - 1);
    const int tb = row >> (lt + lq);
    const int in = row & ((1 << (lt + lq)) - 1);
    const int p2 = in >> lt, p1 = (tb << lt) | (in & ((1 << lt) - 1));
    chk = ((p1 | (p2 << lq)) << lr) | xc;
  }
  const int pos = chk * 64 + (rem & 63);
  if (pos >= a.g.P) return;
  const int sub = class_sublattice(D, MU, (int)(a.c & 3u), q);
  const size_t off = (size_t)plane * (size_t)a.g.N * WPT;
  lattice_edge<D, MU, WPT>(a.n + off, a.f + off, a.g, sub, pos, plane, m, a.t, a.c,
                           a.key0, a.key1, a.noise);
}

template <int Z, int WPT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_pass_graph(PassGraph a, int m)
{
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int pl = lin / a.blocks_per_plane;
  const int blk = lin - pl * a.blocks_per_plane;
  const int plane = a.plane0 + pl;
  const int k = blk * BLOCK + (int)threadIdx.x;
  if (k >= a.count) return;
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  if (a.fsat)
    graph_edge<Z, WPT>(a.n + off, a.f + off, a.edges, a.nbr, a.stride, a.first + k, plane, m, a.t,
                       a.c, a.key0, a.key1, a.noise, FSat{a.fsat, plane * a.N});
  else
    graph_edge<Z, WPT>(a.n + off, a.f + off, a.edges, a.nbr, a.stride, a.first + k, plane, m, a.t,
                       a.c, a.key0, a.key1, a.noise);
}

// One launch counts a.rows states (blockIdx.z): the sim's own state, or snapshots taken by the
// LDS-resident sweep loop.
template <int WPT>
__global__ __launch_bounds__(kObsBlock) void k_observe(ObserveArgs a)
{
  const int plane = blockIdx.y;
  const int row = blockIdx.z;
  const int lane = (int)__lane_id();
  const int wave = (int)(blockIdx.x * (kObsBlock / 64) + threadIdx.x / 64);
  const int nwaves = (int)(gridDim.x * (kObsBlock / 64));
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  const size_t soff = off + (size_t)row * a.row_stride;
  unsigned acc[3][WPT];
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int w = 0; w < WPT; ++w) acc[o][w] = 0;
  for (int base = wave * 64; base < a.N; base += nwaves * 64) {  // wave-uniform loop
    const int idx = base + lane;
    Elem<WPT> x, x0, xf;
    if (idx < a.N) {
      x = ld<WPT>(a.n + soff, idx);
      x0 = ld<WPT>(a.n0 + off, idx);
      xf = ld<WPT>(a.f + soff, idx);
    } else {
#pragma unroll
      for (int w = 0; w < WPT; ++w) x.w[w] = x0.w[w] = xf.w[w] = 0;
    }
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      vertical_count(x.w[w], acc[0][w]);
      vertical_count(x.w[w] & x0.w[w], acc[1][w]);
      vertical_count(x0.w[w] & ~xf.w[w], acc[2][w]);
    }
  }
  unsigned long long *out = a.out + (size_t)row * 3u * (size_t)a.R;
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int w = 0; w < WPT; ++w)
      if (acc[o][w])
        atomicAdd(&out[(size_t)o * a.R + (size_t)(plane * WPT + w) * 64 + lane],
                  (unsigned long long)acc[o][w]);
}

// ------------------------------------------------------------------------------------
// LDS-resident sweep loop: one workgroup owns one plane of a small instance, keeps n and f
// in LDS across all class passes of all requested sweeps (a barrier between passes) and
// records observations in place; only the first load and the final store touch HBM.
// ------------------------------------------------------------------------------------
// ------------------------------------------------------------------------------------
// Initial state (uniform K-subset per replica by smallest Philox keys).
// k_init_select: one workgroup per replica pair (2h, 2h+1), which share Philox calls.
// Radix selection of the K-th smallest key (u, i): 12-bit digits of u, most significant
// first, histogrammed in LDS among keys that match the digits fixed so far, until the
// bin that holds the K-th key has at most kCap keys; those are collected and ranked
// exactly by (u, i).  Output: threshold (u*, i*) per replica; site i is occupied iff
// (u_i, i) <= (u*, i*).
// ------------------------------------------------------------------------------------
constexpr int kSelBlock = 1024;
constexpr int kDig = 12;
constexpr int kBins = 1 << kDig;
constexpr int kCap = 2048;

constexpr int kBinsPerThread = kBins / kSelBlock;

__device__ __forceinline__ bool key_matches(u64 u, u64 prefix, int pbits)
{
  return pbits == 0 || (u >> (64 - pbits)) == prefix;
}

// Exclusive prefix sum of v over the kSelBlock threads of the block (every thread calls it;
// tmp holds one value per wave).  Counts stay below 2^32: at most N <= 2^31 keys.
__device__ __forceinline__ unsigned block_exclusive_scan(unsigned v, unsigned *tmp)
{
  const int lane = (int)__lane_id();
  const int wave = (int)threadIdx.x / 64;
  unsigned x = v;   // inclusive scan within the wave
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const unsigned y = __shfl_up(x, d);
    if (lane >= d) x += y;
  }
  if (lane == 63) tmp[wave] = x;
  __syncthreads();
  unsigned off = 0;
  for (int w = 0; w < wave; ++w) off += tmp[w];
  return off + x - v;
}

__global__ __launch_bounds__(kSelBlock) void k_init_select(InitArgs a)
{
  __shared__ unsigned hist[2][kBins];
  __shared__ u64 cand_u[2][kCap];
  __shared__ int cand_i[2][kCap];
  __shared__ u64 prefix[2];
  __shared__ int pbits[2];
  __shared__ long long need[2];
  __shared__ int done[2];
  __shared__ int ncand[2];
  __shared__ int sel_beta[2];
  __shared__ unsigned sel_cum[2];
  __shared__ unsigned scan_tmp[kSelBlock / 64];
  const int hp = blockIdx.x;
  const int tid = (int)threadIdx.x;
  if (a.K == 0) {
    if (tid < 2) {
      a.thr_u[2 * hp + tid] = 0;
      a.thr_i[2 * hp + tid] = -1;
    }
    return;
  }
  if (tid < 2) {
    prefix[tid] = 0;
    pbits[tid] = 0;
    need[tid] = a.K;
    done[tid] = a.N <= kCap;
    ncand[tid] = 0;
  }
  __syncthreads();
  while (!(done[0] && done[1])) {
    for (int q = tid; q < 2 * kBins; q += kSelBlock) (&hist[0][0])[q] = 0;
    __syncthreads();
    for (int i = tid; i < a.N; i += kSelBlock) {
      const uint4 o = philox10(make_uint4(0u, 0xFFFFFFFFu, (uint32_t)i, (uint32_t)hp), a.key0, a.key1);
      const u64 uk[2] = {lo_half(o), hi_half(o)};
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (done[h]) continue;
        const int pb = pbits[h];
        if (!key_matches(uk[h], prefix[h], pb)) continue;
        const int dig = (64 - pb) < kDig ? (64 - pb) : kDig;
        const unsigned digit = (unsigned)((uk[h] >> (64 - pb - dig)) & ((1ull << dig) - 1ull));
        atomicAdd(&hist[h][digit], 1u);
      }
    }
    // The bin holding the need-th key: the one bin b with E[b] < need <= E[b] + hist[b],
    // E the exclusive prefix sum of the histogram, found by a block-wide scan (thread t owns
    // bins kBinsPerThread * t ...).  The scan's own barrier orders these initial values
    // before the one thread that finds the bin writes it.
    if (tid < 2) {
      sel_beta[tid] = -1;
      sel_cum[tid] = 0;
    }
    __syncthreads();   // the histogram is complete
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (done[h]) continue;   // block-uniform
      unsigned c[kBinsPerThread];
      unsigned sum = 0;
#pragma unroll
      for (int q = 0; q < kBinsPerThread; ++q) {
        c[q] = hist[h][kBinsPerThread * tid + q];
        sum += c[q];
      }
      const unsigned before = block_exclusive_scan(sum, scan_tmp);
      unsigned e = before;
#pragma unroll
      for (int q = 0; q < kBinsPerThread; ++q) {
        if ((long long)e < need[h] && need[h] <= (long long)e + (long long)c[q]) {
          sel_beta[h] = kBinsPerThread * tid + q;
          sel_cum[h] = e;
        }
        e += c[q];
      }
      __syncthreads();   // scan_tmp is reused by the next h
    }
    __syncthreads();
    if (tid < 2 && !done[tid]) {
      const int h = tid;
      const int pb = pbits[h];
      const int dig = (64 - pb) < kDig ? (64 - pb) : kDig;
      int beta = sel_beta[h];
      long long cum = sel_cum[h];
      if (beta < 0 || beta >= (1 << dig)) {  // unreachable: need <= keys under the prefix
        beta = (1 << dig) - 1;
        cum = 0;
        atomicOr(a.err, 2);
      }
      need[h] -= cum;
      prefix[h] = (prefix[h] << dig) | (u64)beta;
      pbits[h] = pb + dig;
      done[h] = (hist[h][beta] <= (unsigned)kCap) || pbits[h] == 64;
    }
    __syncthreads();
  }
  for (int i = tid; i < a.N; i += kSelBlock) {
    const uint4 o = philox10(make_uint4(0u, 0xFFFFFFFFu, (uint32_t)i, (uint32_t)hp), a.key0, a.key1);
    const u64 uk[2] = {lo_half(o), hi_half(o)};
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      if (!key_matches(uk[h], prefix[h], pbits[h])) continue;
      const int slot = atomicAdd(&ncand[h], 1);
      if (slot < kCap) {
        cand_u[h][slot] = uk[h];
        cand_i[h][slot] = i;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int nc = ncand[h] < kCap ? ncand[h] : kCap;
    if (ncand[h] > kCap) {
      if (tid == 0) atomicOr(a.err, 1);
      continue;
    }
    for (int s = tid; s < nc; s += kSelBlock) {
      const u64 us = cand_u[h][s];
      const int is = cand_i[h][s];
      int rank = 0;
      for (int q = 0; q < nc; ++q) {
        const u64 uq = cand_u[h][q];
        rank += (uq < us) || (uq == us && cand_i[h][q] < is);
      }
      if (rank == need[h] - 1) {
        a.thr_u[2 * hp + h] = us;
        a.thr_i[2 * hp + h] = is;
      }
    }
  }
}

// Element index -> canonical site id.
__device__ __forceinline__ int element_site(const InitArgs &a, int idx)
{
  if (!a.is_lattice) return a.site_of[idx];
  const int sub = idx / a.g.P;
  const int pos = idx - sub * a.g.P;
  const Site s = decode(a.g, a.g.d, sub, pos);
  return canonical(a.g, a.g.d, s);
}

template <int WPT>
__global__ __launch_bounds__(256) void k_init_fill(InitArgs a)
{
  const int plane = blockIdx.y;
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  for (int idx = blockIdx.x * 256 + (int)threadIdx.x; idx < a.N; idx += gridDim.x * 256) {
    const int i = element_site(a, idx);
    Elem<WPT> x, z;
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      const int word = plane * WPT + w;
      u64 bits = 0;
      for (int l = 0; l < 64; l += 2) {
        const int b = word * 64 + l;
        const uint4 o = philox10(make_uint4(0u, 0xFFFFFFFFu, (uint32_t)i, (uint32_t)(b >> 1)),
                                 a.key0, a.key1);
        const u64 u0 = lo_half(o), u1 = hi_half(o);
        const u64 t0 = a.thr_u[b], t1 = a.thr_u[b + 1];
        const long long i0 = a.thr_i[b], i1 = a.thr_i[b + 1];
        const bool in0 = (u0 < t0) || (u0 == t0 && (long long)i <= i0);
        const bool in1 = (u1 < t1) || (u1 == t1 && (long long)i <= i1);
        bits |= ((u64)in0 << l) | ((u64)in1 << (l + 1));
      }
      x.w[w] = bits;
      z.w[w] = 0;
    }
    st<WPT>(a.n + off, idx, x);
    st<WPT>(a.n0 + off, idx, x);
    st<WPT>(a.f + off, idx, z);
  }
}

}  // namespace

// ------------------------------------------------------------------------------------
// Launchers
// ------------------------------------------------------------------------------------
hipError_t launch_pass_lattice(const PassLattice &a, int m, int wpt, hipStream_t s)
{
  const dim3 grid((unsigned)(a.blocks_per_plane * a.planes));
  const dim3 block(kPassBlock);
#define KA_LAT(D, MU, W) \
  hipLaunchKernelGGL((k_pass_lattice<D, MU, W>), grid, block, 0, s, a, m)
  if (a.g.d == 2) {
    if (wpt == 2) {
      if (a.mu == 0) KA_LAT(2, 0, 2); else KA_LAT(2, 1, 2);
    } else {
      if (a.mu == 0) KA_LAT(2, 0, 1); else KA_LAT(2, 1, 1);
    }
  } else {
    if (wpt == 2) {
      if (a.mu == 0) KA_LAT(3, 0, 2); else if (a.mu == 1) KA_LAT(3, 1, 2); else KA_LAT(3, 2, 2);
    } else {
      if (a.mu == 0) KA_LAT(3, 0, 1); else if (a.mu == 1) KA_LAT(3, 1, 1); else KA_LAT(3, 2, 1);
    }
  }
#undef KA_LAT
  return hipGetLastError();
}

hipError_t launch_pass_graph(const PassGraph &args, int z, int m, int wpt, hipStream_t s)
{
  PassGraph a = args;
  const bool small = (long long)a.count * a.planes < kGraphSmallEdges;
  const int bs = small ? kGraphSmallBlock : kPassBlock;
  a.blocks_per_plane = (a.count + bs - 1) / bs;
  const dim3 grid((unsigned)(a.blocks_per_plane * a.planes));
  const dim3 block((unsigned)bs);
#define KA_GR(Z, W)                                                                        \
  do {                                                                                     \
    if (small)                                                                             \
      hipLaunchKernelGGL((k_pass_graph<Z, W, kGraphSmallBlock>), grid, block, 0, s, a, m); \
    else                                                                                   \
      hipLaunchKernelGGL((k_pass_graph<Z, W, kPassBlock>), grid, block, 0, s, a, m);       \
  } while (0)
  switch (z * 4 + wpt) {
    case 3 * 4 + 1: KA_GR(3, 1); break;
    case 3 * 4 + 2: KA_GR(3, 2); break;
    case 4 * 4 + 1: KA_GR(4, 1); break;
    case 4 * 4 + 2: KA_GR(4, 2); break;
    case 5 * 4 + 1: KA_GR(5, 1); break;
    case 5 * 4 + 2: KA_GR(5, 2); break;
    case 6 * 4 + 1: KA_GR(6, 1); break;
    case 6 * 4 + 2: KA_GR(6, 2); break;
    default: return hipErrorInvalidValue;
  }
#undef KA_GR
  return hipGetLastError();
}

hipError_t launch_init(const InitArgs &a, int R, int wpt, hipStream_t s)
{
  hipLaunchKernelGGL(k_init_select, dim3((unsigned)(R / 2)), dim3(kSelBlock), 0, s, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int planes = (R / 64) / wpt;
  int bx = (a.N + 255) / 256;
  if (bx > 4096) bx = 4096;
  if (wpt == 2)
    hipLaunchKernelGGL((k_init_fill<2>), dim3((unsigned)bx, (unsigned)planes), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL((k_init_fill<1>), dim3((unsigned)bx, (unsigned)planes), dim3(256), 0, s, a);
  return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Fixed scratch for the observation entry point that allocates nothing (ka_observe_noalloc):
// the per-replica counts accumulate here instead of in a sim's own buffer.  One copy per
// device, held until the process ends; every call on a device shares it.
// ------------------------------------------------------------------------------------
namespace {

__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v)
{
  const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
  if (i < n) p[i] = v;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t observe_scratch_setup(int device)
{
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  // the array's name is only a host-side stand-in: the device address comes from the runtime,
  // taken with this device current
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(::scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = static_cast<unsigned long long *>(ptr);
  return hipSuccess;
}

unsigned long long *observe_scratch(int device)
{
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch_ptr[device];
}

hipError_t launch_fill_u64(unsigned long long *p, int n, unsigned long long v, hipStream_t s)
{
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_observe(const ObserveArgs &a, int wpt, hipStream_t s)
{
  if (a.rows < 1 || a.rows > 65535) return hipErrorInvalidValue;
  int bx = (a.N + kObsBlock - 1) / kObsBlock;
  if (bx > 512) bx = 512;
  const dim3 grid((unsigned)bx, (unsigned)a.planes, (unsigned)a.rows);
  if (wpt == 2)
    hipLaunchKernelGGL((k_observe<2>), grid, dim3(kObsBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_observe<1>), grid, dim3(kObsBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace ka
