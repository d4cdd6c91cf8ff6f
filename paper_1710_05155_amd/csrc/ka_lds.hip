// ka_lds.hip -- LDS-resident sweep loop for instances whose word plane fits in LDS (gfx950).
//
// Method: Boccagna, arXiv 1710.05155; the per-edge bit logic lives in ka_device.h.
#include "ka_device.h"

namespace ka {
namespace {

using namespace dev;

constexpr int kLdsBlock = 1024;
// Edges per thread and class on a lattice in LDS: a plane that fits (N * wpt <= 9984 words
// per array) has at most 2496 edges per class.
constexpr int kLdsSlots = 3;

template <int WPT>
__device__ void lds_observe(const SweepLds &a, const u64 *sn, const u64 *sf, int plane,
                            int row, unsigned *cnt)
{
  const int tid = (int)threadIdx.x;
  const int lane = (int)__lane_id();
  const int wave = tid / 64, nw = (int)blockDim.x / 64;
  for (int q = tid; q < 3 * 64 * WPT; q += (int)blockDim.x) cnt[q] = 0;
  __syncthreads();
  unsigned acc[3][WPT];
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int w = 0; w < WPT; ++w) acc[o][w] = 0;
  const u64 *n0 = a.n0 + (size_t)plane * (size_t)a.N * WPT;
  for (int base = wave * 64; base < a.N; base += nw * 64) {
    const int idx = base + lane;
    Elem<WPT> x, x0, xf;
    if (idx < a.N) {
      x = ld<WPT>(sn, idx);
      xf = ld<WPT>(sf, idx);
      x0 = ld<WPT>(n0, idx);
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
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int w = 0; w < WPT; ++w)
      if (acc[o][w]) atomicAdd(&cnt[o * 64 * WPT + w * 64 + lane], acc[o][w]);
  __syncthreads();
  for (int q = tid; q < 3 * 64 * WPT; q += (int)blockDim.x) {
    const int o = q / (64 * WPT), rr = q - o * 64 * WPT;
    a.obs_out[((size_t)row * 3 + o) * a.R + (size_t)plane * 64 * WPT + rr] = cnt[q];
  }
  __syncthreads();
}

template <int WPT>
__device__ void lds_load(const SweepLds &a, u64 *sn, u64 *sf, int plane)
{
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  for (int q = (int)threadIdx.x; q < a.N * WPT; q += (int)blockDim.x) {
    sn[q] = a.n[off + q];
    sf[q] = a.f[off + q];
  }
  __syncthreads();
}

template <int WPT>
__device__ void lds_store(const SweepLds &a, const u64 *sn, const u64 *sf, int plane)
{
  __syncthreads();
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  for (int q = (int)threadIdx.x; q < a.N * WPT; q += (int)blockDim.x) {
    a.n[off + q] = sn[q];
    a.f[off + q] = sf[q];
  }
}

// Copy of the plane's n and f into snapshot row `row` (layout in SweepLds::snap), for the
// observation kernel to count after this launch on the whole device.
template <int WPT>
__device__ void lds_snapshot(const SweepLds &a, const u64 *sn, const u64 *sf, int plane, int row)
{
  const int words = a.N * WPT;                                // one plane
  const size_t row_words = (size_t)(a.R / 64) * (size_t)a.N;  // every plane, n or f
  u64 *dn = a.snap + (size_t)row * 2u * row_words + (size_t)plane * (size_t)words;
  u64 *df = dn + row_words;
  for (int q = (int)threadIdx.x; q < words; q += (int)blockDim.x) {
    dn[q] = sn[q];
    df[q] = sf[q];
  }
  __syncthreads();   // the next pass rewrites sn and sf
}

template <int WPT>
__device__ void lds_observe_due(const SweepLds &a, const u64 *sn, const u64 *sf, int plane,
                                int &qo, int64_t t_now, unsigned *cnt)
{
  while (qo < a.n_obs && a.obs_times[qo] == t_now) {
    if (a.snap) lds_snapshot<WPT>(a, sn, sf, plane, qo);
    else lds_observe<WPT>(a, sn, sf, plane, qo, cnt);
    ++qo;
  }
}

// Element of the pre-generated acceptance words of sweep s (relative to t0), class c, slot j
// for this thread.
__device__ __forceinline__ int acc_element(const SweepLds &a, int plane, int s, int c, int j)
{
  return (((plane * a.n_sweeps + s) * a.C + c) * a.acc_slots + j) * kLdsBlock + (int)threadIdx.x;
}

// Acceptance words of sweeps t0 .. t0 + n_sweeps - 1 for k_sweep_lds_lattice: one workgroup per
// (sweep, class) and plane, each thread drawing the words of its edge slots exactly as the sweep
// loop maps them (the same sublattice, position and canonical edge id).  The words do not
// depend on the state, so the whole device draws them ahead of the single-workgroup loop.
template <int D, int WPT>
__global__ __launch_bounds__(kLdsBlock) void k_lds_accept_lattice(SweepLds a)
{
  const int sc = (int)blockIdx.x;
  const int s = sc / a.C, c = sc - s * a.C;
  const int plane = (int)blockIdx.y;
  const int mu = c >> 2;
  constexpr int nsub = D == 2 ? 4 : 16;
  const int per_class = nsub * a.g.P;
  for (int j = 0; j < a.acc_slots; ++j) {
    const int k = (int)threadIdx.x + j * kLdsBlock;
    if (k >= per_class) break;
    const int q = k / a.g.P;
    const int sub = class_sublattice(D, mu, c & 3, q);
    const Site si = decode(a.g, D, sub, k - q * a.g.P);
    const uint32_t e = (uint32_t)canonical(a.g, D, si) * (uint32_t)D + (uint32_t)mu;
    u64 r[WPT];
    accept_words<WPT>(a.t0 + (uint32_t)s, (uint32_t)c, e, plane, a.key0, a.key1, a.noise, r);
    Elem<WPT> v;
#pragma unroll
    for (int w = 0; w < WPT; ++w) v.w[w] = r[w];
    st<WPT>(a.acc, acc_element(a, plane, s, c, j), v);
  }
}

// One lattice edge of the LDS sweep with its acceptance words given.
template <int D, int MU, int WPT>
__device__ __forceinline__ void lattice_edge_given(u64 *nb, u64 *fb, const LatticeGeom &g,
                                                   const Site &si, const Elem<WPT> &rw, int m)
{
  constexpr int K = 2 * D - 1;
  int i, j, ii[K], jj[K];
  uint32_t e;
  lattice_edge_indices<D, MU>(g, si, i, j, ii, jj, e);
  edge_update_with<K, WPT>(nb, fb, i, j, ii, jj, m, [&](u64 (&r)[WPT]) {
#pragma unroll
    for (int w = 0; w < WPT; ++w) r[w] = rw.w[w];
  });
}

// Acceptance words of sweeps t0 .. t0 + n_sweeps - 1 for k_sweep_lds_graph: blockIdx.x runs
// over (sweep, block of 1024 class-sorted edges), blockIdx.y over planes; each thread draws
// the words of one edge from its record (canonical id e, class c), as the sweep loop would.
template <int WPT>
__global__ __launch_bounds__(kLdsBlock) void k_lds_accept_graph(SweepLds a)
{
  const int E = (int)a.stride;
  const int nblk = (E + kLdsBlock - 1) / kLdsBlock;
  const int s = (int)blockIdx.x / nblk;
  const int k = ((int)blockIdx.x - s * nblk) * kLdsBlock + (int)threadIdx.x;
  const int plane = (int)blockIdx.y;
  if (k >= E) return;
  const int4 rec = a.edges[k];
  u64 r[WPT];
  accept_words<WPT>(a.t0 + (uint32_t)s, (uint32_t)rec.w, (uint32_t)rec.z, plane, a.key0, a.key1, a.noise, r);
  Elem<WPT> rw;
#pragma unroll
  for (int w = 0; w < WPT; ++w) rw.w[w] = r[w];
  st<WPT>(a.acc, (plane * a.n_sweeps + s) * E + k, rw);
}

// SLOTS: edge slots per thread the kernel is compiled for (the class size over 1024, rounded
// up, must not exceed it).
template <int D, int WPT, bool GIVEN, int SLOTS = kLdsSlots>
__global__ __launch_bounds__(kLdsBlock) void k_sweep_lds_lattice(SweepLds a, int m)
{
  extern __shared__ u64 lds[];
  __shared__ unsigned cnt[3 * 64 * WPT];
  u64 *sn = lds;
  u64 *sf = lds + (size_t)a.N * WPT;
  const int plane = blockIdx.x;
  lds_load<WPT>(a, sn, sf, plane);
  int qo = 0;
  lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)a.t0, cnt);
  constexpr int nsub = D == 2 ? 4 : 16;   // lower-endpoint sublattices per class
  const int per_class = nsub * a.g.P;
  // This thread's edges are the same in every class: slot j is edge k = tid + j * blockDim of
  // the class, the q-th lower-endpoint sublattice at position pos.  The divisions and the
  // block coordinates of pos are done once, here; per class only the residues change.
  const int tid = (int)threadIdx.x;
  int slot_q[SLOTS];
  Site slot_site[SLOTS];
#pragma unroll
  for (int j = 0; j < SLOTS; ++j) {
    const int k = tid + j * kLdsBlock;
    const int q = k / a.g.P;
    slot_q[j] = q;
    slot_site[j] = decode(a.g, D, 0, k - q * a.g.P);   // idx = pos, residues 0
  }
  // With pre-generated acceptance words, those of the next class are loaded while this
  // class is processed (the loads stay in flight across the barrier).
  Elem<WPT> rnext[SLOTS];
  if constexpr (GIVEN) {
#pragma unroll
    for (int j = 0; j < SLOTS; ++j)
      if (tid + j * kLdsBlock < per_class) rnext[j] = ld<WPT>(a.acc, acc_element(a, plane, 0, 0, j));
  }
  for (int s = 0; s < a.n_sweeps; ++s) {
    const uint32_t t = a.t0 + (uint32_t)s;
    for (int c = 0; c < a.C; ++c) {
      const int mu = c >> 2;
      Elem<WPT> rcur[SLOTS];
      if constexpr (GIVEN) {
        const int s2 = c + 1 < a.C ? s : s + 1;
        const int c2 = c + 1 < a.C ? c + 1 : 0;
#pragma unroll
        for (int j = 0; j < SLOTS; ++j) {
          rcur[j] = rnext[j];
          if (s2 < a.n_sweeps && tid + j * kLdsBlock < per_class)
            rnext[j] = ld<WPT>(a.acc, acc_element(a, plane, s2, c2, j));
        }
      }
#pragma unroll
      for (int j = 0; j < SLOTS; ++j) {
        if (tid + j * kLdsBlock >= per_class) break;
        const int sub = class_sublattice(D, mu, c & 3, slot_q[j]);
        Site si = slot_site[j];
        si.a[0] = sub & 3;
        si.a[1] = (sub >> 2) & 3;
        si.a[2] = (sub >> 4) & 3;
        si.idx += sub * a.g.P;
        if constexpr (GIVEN) {
          if (mu == 0)
            lattice_edge_given<D, 0, WPT>(sn, sf, a.g, si, rcur[j], m);
          else if (mu == 1)
            lattice_edge_given<D, 1, WPT>(sn, sf, a.g, si, rcur[j], m);
          else if constexpr (D == 3)
            lattice_edge_given<D, 2, WPT>(sn, sf, a.g, si, rcur[j], m);
          continue;
        }
        if (mu == 0)
          lattice_edge_at<D, 0, WPT>(sn, sf, a.g, si, plane, m, t, (uint32_t)c, a.key0, a.key1,
                                     a.noise);
        else if (mu == 1)
          lattice_edge_at<D, 1, WPT>(sn, sf, a.g, si, plane, m, t, (uint32_t)c, a.key0, a.key1,
                                     a.noise);
        else if constexpr (D == 3)
          lattice_edge_at<D, 2, WPT>(sn, sf, a.g, si, plane, m, t, (uint32_t)c, a.key0, a.key1,
                                     a.noise);
      }
      __syncthreads();
    }
    lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)t + 1, cnt);
  }
  lds_store<WPT>(a, sn, sf, plane);
}

// GIVEN: the acceptance words come from a.acc (every class has at most kLdsGraphAcceptSlots
// edges per thread), those of the next class loaded while this class is processed.
template <int Z, int WPT, bool GIVEN>
__global__ __launch_bounds__(kLdsBlock) void k_sweep_lds_graph(SweepLds a, int m)
{
  extern __shared__ u64 lds[];
  __shared__ unsigned cnt[3 * 64 * WPT];
  u64 *sn = lds;
  u64 *sf = lds + (size_t)a.N * WPT;
  const int plane = blockIdx.x;
  const int tid = (int)threadIdx.x;
  const int E = (int)a.stride;
  lds_load<WPT>(a, sn, sf, plane);
  int qo = 0;
  lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)a.t0, cnt);
  constexpr int S = kLdsGraphAcceptSlots;
  Elem<WPT> rnext[S];
  if constexpr (GIVEN) {
    const int b0 = a.class_start[0], b1 = a.class_start[1];
#pragma unroll
    for (int j = 0; j < S; ++j)
      if (b0 + tid + j * kLdsBlock < b1) rnext[j] = ld<WPT>(a.acc, plane * a.n_sweeps * E + b0 + tid + j * kLdsBlock);
  }
  for (int s = 0; s < a.n_sweeps; ++s) {
    const uint32_t t = a.t0 + (uint32_t)s;
    for (int c = 0; c < a.C; ++c) {
      const int b0 = a.class_start[c], b1 = a.class_start[c + 1];
      if constexpr (GIVEN) {
        // This class's records and neighbour lists are loaded before the next class's words:
        // vector loads complete in order, so waiting for the records leaves the words in
        // flight while this class is processed.
        constexpr int K = Z - 1;
        int4 rec[S];
        int iu[S][K], iv[S][K];
#pragma unroll
        for (int j = 0; j < S; ++j) {
          const int k = b0 + tid + j * kLdsBlock;
          if (k < b1) {
            rec[j] = a.edges[k];
#pragma unroll
            for (int q = 0; q < K; ++q) {
              iu[j][q] = a.nbr[(size_t)q * a.stride + (size_t)k];
              iv[j][q] = a.nbr[(size_t)(K + q) * a.stride + (size_t)k];
            }
          }
        }
        Elem<WPT> rcur[S];
        const int s2 = c + 1 < a.C ? s : s + 1;
        const int c2 = c + 1 < a.C ? c + 1 : 0;
        const int n0 = a.class_start[c2], n1 = a.class_start[c2 + 1];
#pragma unroll
        for (int j = 0; j < S; ++j) {
          rcur[j] = rnext[j];
          const int k2 = n0 + tid + j * kLdsBlock;
          if (s2 < a.n_sweeps && k2 < n1) rnext[j] = ld<WPT>(a.acc, (plane * a.n_sweeps + s2) * E + k2);
        }
#pragma unroll
        for (int j = 0; j < S; ++j) {
          if (b0 + tid + j * kLdsBlock >= b1) break;
          edge_update_with<K, WPT>(sn, sf, rec[j].x, rec[j].y, iu[j], iv[j], m, [&](u64 (&r)[WPT]) {
#pragma unroll
            for (int w = 0; w < WPT; ++w) r[w] = rcur[j].w[w];
          });
        }
      } else {
        for (int k = b0 + tid; k < b1; k += (int)blockDim.x)
          graph_edge<Z, WPT>(sn, sf, a.edges, a.nbr, a.stride, k, plane, m, t, (uint32_t)c, a.key0,
                             a.key1, a.noise);
      }
      __syncthreads();
    }
    lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)t + 1, cnt);
  }
  lds_store<WPT>(a, sn, sf, plane);
}

template <typename Kern>
hipError_t set_lds(Kern k, size_t bytes)
{
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

}  // namespace

size_t sweep_lds_bytes(int N, int wpt) { return (size_t)2 * (size_t)N * (size_t)wpt * 8u; }

int lds_lattice_slots(int d, int P) { return ((d == 2 ? 4 : 16) * P + kLdsBlock - 1) / kLdsBlock; }

// The sweep loop with given acceptance words keeps the next class's words in registers.  For
// 3D word pairs it is compiled for one edge slot per thread, the most a 3D plane of word pairs
// that fits in LDS needs (L = 16: 1024 edges per class); three slots would not fit the 128
// registers a 1024-thread workgroup allows.
bool lds_accept_supported(int d, int wpt, int slots) { return !(d == 3 && wpt == 2 && slots > 1); }

int lds_graph_slots(int max_class_edges) { return (max_class_edges + kLdsBlock - 1) / kLdsBlock; }

// With given words the graph sweep holds each slot's record, neighbour ids and words in
// registers; for z = 6 with word pairs that exceeds the 128 a 1024-thread workgroup allows, so
// that layout draws its words in the loop.
bool lds_graph_accept_supported(int z, int wpt) { return !(z == 6 && wpt == 2); }

hipError_t launch_lds_accept(const SweepLds &a, bool lattice, int wpt, hipStream_t s)
{
  const int planes = (a.R / 64) / wpt;
  if (!lattice) {
    const int E = (int)a.stride;
    const int nblk = (E + kLdsBlock - 1) / kLdsBlock;
    if (!a.acc || a.n_sweeps < 1 || E < 1 || a.acc_slots < 1 || a.acc_slots > kLdsGraphAcceptSlots ||
        (long long)a.n_sweeps * nblk > 0x7FFFFFFFLL)
      return hipErrorInvalidValue;
    const dim3 grid((unsigned)(a.n_sweeps * nblk), (unsigned)planes);
    if (wpt == 2) hipLaunchKernelGGL((k_lds_accept_graph<2>), grid, dim3(kLdsBlock), 0, s, a);
    else hipLaunchKernelGGL((k_lds_accept_graph<1>), grid, dim3(kLdsBlock), 0, s, a);
    return hipGetLastError();
  }
  if (!a.acc || a.n_sweeps < 1 || a.acc_slots < 1 || a.acc_slots > kLdsSlots ||
      a.acc_slots != lds_lattice_slots(a.g.d, a.g.P) || !lds_accept_supported(a.g.d, wpt, a.acc_slots))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(a.n_sweeps * a.C), (unsigned)planes);
  const dim3 block(kLdsBlock);
  if (a.g.d == 2) {
    if (wpt == 2) hipLaunchKernelGGL((k_lds_accept_lattice<2, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_lds_accept_lattice<2, 1>), grid, block, 0, s, a);
  } else {
    if (wpt == 2) hipLaunchKernelGGL((k_lds_accept_lattice<3, 2>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_lds_accept_lattice<3, 1>), grid, block, 0, s, a);
  }
  return hipGetLastError();
}

int max_lds_bytes()
{
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return 0;
  return v;
}

hipError_t launch_sweep_lds(const SweepLds &a, bool lattice, int zdeg, int m, int wpt,
                            size_t lds_bytes, hipStream_t s)
{
  const int planes = (a.R / 64) / wpt;
  const dim3 grid((unsigned)planes);
  const dim3 block(kLdsBlock);
  hipError_t e = hipSuccess;
#define KA_LDS_L(D, W, G)                                                         \
  do {                                                                            \
    e = set_lds(k_sweep_lds_lattice<D, W, G>, lds_bytes);                         \
    if (e == hipSuccess)                                                          \
      hipLaunchKernelGGL((k_sweep_lds_lattice<D, W, G>), grid, block, lds_bytes, s, a, m); \
  } while (0)
#define KA_LDS_G1(Z, W, G)                                                        \
  do {                                                                            \
    e = set_lds(k_sweep_lds_graph<Z, W, G>, lds_bytes);                           \
    if (e == hipSuccess)                                                          \
      hipLaunchKernelGGL((k_sweep_lds_graph<Z, W, G>), grid, block, lds_bytes, s, a, m); \
  } while (0)
#define KA_LDS_G(Z, W)                                                            \
  do {                                                                            \
    if (a.acc) KA_LDS_G1(Z, W, true); else KA_LDS_G1(Z, W, false);                 \
  } while (0)
  if (lattice && (a.g.d == 2 ? 4 : 16) * a.g.P > kLdsSlots * kLdsBlock) return hipErrorInvalidValue;
  if (lattice) {
    if (a.acc && !lds_accept_supported(a.g.d, wpt, lds_lattice_slots(a.g.d, a.g.P))) return hipErrorInvalidValue;
    const bool g = a.acc != nullptr;
    if (a.g.d == 2) {
      if (wpt == 2) {
        if (g) KA_LDS_L(2, 2, true); else KA_LDS_L(2, 2, false);
      } else {
        if (g) KA_LDS_L(2, 1, true); else KA_LDS_L(2, 1, false);
      }
    } else {
      if (wpt == 2) {
        if (g) {
          e = set_lds(k_sweep_lds_lattice<3, 2, true, 1>, lds_bytes);
          if (e == hipSuccess)
            hipLaunchKernelGGL((k_sweep_lds_lattice<3, 2, true, 1>), grid, block, lds_bytes, s, a, m);
        } else {
          KA_LDS_L(3, 2, false);
        }
      } else if (g) KA_LDS_L(3, 1, true);
      else KA_LDS_L(3, 1, false);
    }
  } else {
    if (a.acc && (a.acc_slots < 1 || a.acc_slots > kLdsGraphAcceptSlots || !lds_graph_accept_supported(zdeg, wpt)))
      return hipErrorInvalidValue;
    switch (zdeg * 4 + wpt) {
      case 3 * 4 + 1: KA_LDS_G(3, 1); break;
      case 3 * 4 + 2: KA_LDS_G(3, 2); break;
      case 4 * 4 + 1: KA_LDS_G(4, 1); break;
      case 4 * 4 + 2: KA_LDS_G(4, 2); break;
      case 5 * 4 + 1: KA_LDS_G(5, 1); break;
      case 5 * 4 + 2: KA_LDS_G(5, 2); break;
      case 6 * 4 + 1: KA_LDS_G(6, 1); break;
      case 6 * 4 + 2: KA_LDS_G1(6, 2, false); break;   // see lds_graph_accept_supported
      default: return hipErrorInvalidValue;
    }
  }
#undef KA_LDS_L
#undef KA_LDS_G
#undef KA_LDS_G1
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace ka
