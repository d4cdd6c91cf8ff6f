// ka_pairs.hip -- spatial four-point sums (gfx950).
//
// Method: Boccagna, arXiv 1710.05155, Sec. 2.2 (g4(r, t) and chi4 = sum_r g4) and Sec. 3.3
// (Phi(r, t) as the popcount of the AND of the words n_i(t), n_i(0), n_j(t), n_j(0)).  With
// Q_i = n_i(t) & n_i(0) per word (one bit per replica), for every minimum-image displacement
// delta with |delta|^2 = r2 <= r2_max:
//     S2[r2]  += popcount(Q_i & Q_{i+delta})            summed over sites i and words,
//     S11[r2] += popcount(Q_i) * popcount(Q_{i+delta})  with popcounts over all words,
// i.e. the replica sums of q_i q_j and the products of the replica sums, over ordered pairs.
// One thread per site holds its Q words in registers; a workgroup takes a chunk of
// displacements, reduces each one over the wave with shuffles and adds it into 64-bit LDS
// shell accumulators, which go to global memory once per workgroup.
#include "ka_device.h"

namespace ka {
namespace {

using namespace dev;

constexpr int kPairBlock = 256;
constexpr int kPairChunk = 32;     // displacements per workgroup
constexpr int kMaxWords = 16;      // up to 1024 replicas

__device__ __forceinline__ unsigned wave_sum(unsigned v)
{
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += (unsigned)__shfl_xor((int)v, off);
  return v;
}

// element index of canonical coordinates in the sublattice layout
__device__ __forceinline__ int element_of(const LatticeGeom &g, const int (&x)[3])
{
  int sub = 0, pos = 0, sm = 1, pm = 1;
  for (int k = 0; k < g.d; ++k) {
    sub += (x[k] & 3) * sm;
    pos += (x[k] >> 2) * pm;
    sm *= 4;
    pm *= g.Q;
  }
  return sub * g.P + pos;
}

template <int WPT>
__global__ __launch_bounds__(kPairBlock) void k_pairs(PairArgs a)
{
  __shared__ unsigned long long acc2[kMaxPairShells];
  __shared__ unsigned long long acc11[kMaxPairShells];
  const int tid = (int)threadIdx.x;
  for (int q = tid; q <= a.r2_max; q += kPairBlock) {
    acc2[q] = 0;
    acc11[q] = 0;
  }
  __syncthreads();
  const int idx = (int)blockIdx.x * kPairBlock + tid;
  const bool valid = idx < a.g.N;
  const int e = valid ? idx : 0;
  const int sub = e / a.g.P, pos = e - (e / a.g.P) * a.g.P;
  const Site s = decode(a.g, a.g.d, sub, pos);
  int x[3];
  for (int k = 0; k < 3; ++k) x[k] = 4 * s.p[k] + s.a[k];
  const size_t plane_words = (size_t)a.g.N * WPT;
  u64 qi[kMaxWords];
  unsigned pci = 0;
#pragma unroll
  for (int q = 0; q < kMaxWords; ++q) {
    qi[q] = 0;
    const int p = q / WPT, w = q % WPT;
    if (p < a.planes) {
      const size_t off = (size_t)p * plane_words + (size_t)e * WPT + w;
      qi[q] = a.n[off] & a.n0[off];
      pci += (unsigned)__popcll(qi[q]);
    }
  }
  const int d0 = (int)blockIdx.y * kPairChunk;
  const int d1 = min(a.n_disp, d0 + kPairChunk);
  for (int dq = d0; dq < d1; ++dq) {
    const int4 dv = a.disp[dq];
    int y[3] = {x[0] + dv.x, x[1] + dv.y, x[2] + dv.z};
    for (int k = 0; k < a.g.d; ++k) {
      if (y[k] < 0) y[k] += a.g.L;
      else if (y[k] >= a.g.L) y[k] -= a.g.L;
    }
    const int j = element_of(a.g, y);
    unsigned c2 = 0, pcj = 0;
#pragma unroll
    for (int q = 0; q < kMaxWords; ++q) {
      const int p = q / WPT, w = q % WPT;
      if (p < a.planes) {
        const size_t off = (size_t)p * plane_words + (size_t)j * WPT + w;
        const u64 qj = a.n[off] & a.n0[off];
        c2 += (unsigned)__popcll(qi[q] & qj);
        pcj += (unsigned)__popcll(qj);
      }
    }
    unsigned c11 = pci * pcj;
    if (!valid) c2 = c11 = 0;
    c2 = wave_sum(c2);
    c11 = wave_sum(c11);
    if (__lane_id() == 0) {
      atomicAdd(&acc2[dv.w], (unsigned long long)c2);
      atomicAdd(&acc11[dv.w], (unsigned long long)c11);
    }
  }
  __syncthreads();
  for (int q = tid; q <= a.r2_max; q += kPairBlock) {
    if (acc2[q]) atomicAdd(&a.S2[q], acc2[q]);
    if (acc11[q]) atomicAdd(&a.S11[q], acc11[q]);
  }
}

// Graphs without a geometry (Sec. 3.3: distance 0 for i = j, 1 otherwise): only the per-site
// replica sums Q_i = sum_b q_i^b are needed, through sum_i Q_i and sum_i Q_i^2 (out[0], out[1]).
template <int WPT>
__global__ __launch_bounds__(kPairBlock) void k_pairs_graph(PairGraphArgs a)
{
  const int i = (int)blockIdx.x * kPairBlock + (int)threadIdx.x;
  unsigned q = 0;
  if (i < a.N) {
    const size_t plane_words = (size_t)a.N * WPT;
    for (int p = 0; p < a.planes; ++p)
#pragma unroll
      for (int w = 0; w < WPT; ++w) {
        const size_t off = (size_t)p * plane_words + (size_t)i * WPT + w;
        q += (unsigned)__popcll(a.n[off] & a.n0[off]);
      }
  }
  // per wave: sum Q <= 64 * 1024 and sum Q^2 <= 64 * 2^20, both within 32 bits
  const unsigned s1 = wave_sum(q);
  const unsigned s2 = wave_sum(q * q);
  if (__lane_id() == 0 && s1) {
    atomicAdd(&a.out[0], (unsigned long long)s1);
    atomicAdd(&a.out[1], (unsigned long long)s2);
  }
}

}  // namespace

hipError_t launch_pairs_graph(const PairGraphArgs &a, int wpt, hipStream_t s)
{
  const dim3 grid((unsigned)((a.N + kPairBlock - 1) / kPairBlock));
  if (wpt == 2)
    hipLaunchKernelGGL((k_pairs_graph<2>), grid, dim3(kPairBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_pairs_graph<1>), grid, dim3(kPairBlock), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_pairs(const PairArgs &a, int wpt, hipStream_t s)
{
  const dim3 grid((unsigned)((a.g.N + kPairBlock - 1) / kPairBlock), (unsigned)((a.n_disp + kPairChunk - 1) / kPairChunk));
  if (wpt == 2)
    hipLaunchKernelGGL((k_pairs<2>), grid, dim3(kPairBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_pairs<1>), grid, dim3(kPairBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace ka
