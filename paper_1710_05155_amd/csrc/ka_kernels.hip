// ka_kernels.hip -- CDNA4 (gfx950) kernels of the multispin Kob-Andersen sweep.
//
// Method: Boccagna, arXiv 1710.05155.  The state of 64 replicas of one site is one 64-bit
// word (Sec. 3.1, multispin coding).  An edge (i, j) is updated for all replicas of a word
// at once with bitwise logic (Sec. 3.2): A_k = "at most m occupied neighbours of k other
// than the partner" per replica, computed with a bit-sliced adder (one bit of the sum per
// word, every replica in its own bit lane) and a comparison with m; the exchange mask is
//     d = (n_i ^ n_j) & A_i & A_j & r,   n_i ^= d, n_j ^= d, f_i |= d, f_j |= d,
// where r holds the per-replica Bernoulli(1/2) acceptance bits from Philox4x32-10.  This
// equals the paper's Table 1 update with s_i = s_{i4} & s_{j5}, s_j = s_{j4} & s_{i5}
// (Sec. 3.2): a particle at i may hop to an empty j iff i has at most m occupied
// neighbours (j empty) and j at most m+1 (i occupied), i.e. both counts that exclude the
// partner are at most m.  f marks sites whose occupation ever changed (persistence).
//
// All hot-path work is integer bit logic: there is no dense contraction, so no MFMA.
#include "ka_internal.h"

namespace ka {
namespace {

constexpr int kPassBlock = 256;
constexpr int kLdsBlock = 1024;
constexpr int kObsBlock = 256;

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The round keys depend only on the
// seed, so they stay in scalar registers; each round is two 32x32->64 multiplies and xors.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const u64 p0 = (u64)0xD2511F53u * (u64)c.x;
    const u64 p1 = (u64)0xCD9E8D57u * (u64)c.z;
    uint4 y;
    y.x = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    y.y = (uint32_t)p1;
    y.z = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    y.w = (uint32_t)p0;
    c = y;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ u64 lo_half(uint4 o) { return (u64)o.x | ((u64)o.y << 32); }
__device__ __forceinline__ u64 hi_half(uint4 o) { return (u64)o.z | ((u64)o.w << 32); }

// Acceptance words of the WPT words of plane `plane` for edge e of class c in sweep t:
// word w uses half (w & 1) of Philox(t, c, e, w >> 1).
template <int WPT>
__device__ __forceinline__ void accept_words(uint32_t t, uint32_t c, uint32_t e, int plane,
                                             uint32_t k0, uint32_t k1, u64 (&r)[WPT])
{
  if constexpr (WPT == 2) {
    const uint4 o = philox10(make_uint4(t, c, e, (uint32_t)plane), k0, k1);
    r[0] = lo_half(o);
    r[1] = hi_half(o);
  } else {
    const uint4 o = philox10(make_uint4(t, c, e, (uint32_t)plane >> 1), k0, k1);
    r[0] = (plane & 1) ? hi_half(o) : lo_half(o);
  }
}

// ------------------------------------------------------------------------------------
// Element = the WPT words of one site in one plane.
// ------------------------------------------------------------------------------------
template <int WPT>
struct Elem {
  u64 w[WPT];
};

template <int WPT>
__device__ __forceinline__ Elem<WPT> ld(const u64 *base, int idx)
{
  Elem<WPT> e;
  if constexpr (WPT == 2) {
    const ulonglong2 v = reinterpret_cast<const ulonglong2 *>(base)[idx];
    e.w[0] = v.x;
    e.w[1] = v.y;
  } else {
    e.w[0] = base[idx];
  }
  return e;
}

template <int WPT>
__device__ __forceinline__ void st(u64 *base, int idx, const Elem<WPT> &e)
{
  if constexpr (WPT == 2) {
    ulonglong2 v;
    v.x = e.w[0];
    v.y = e.w[1];
    reinterpret_cast<ulonglong2 *>(base)[idx] = v;
  } else {
    base[idx] = e.w[0];
  }
}

// ------------------------------------------------------------------------------------
// Bit-sliced neighbour count and threshold (replaces the paper's Karnaugh subset-OR forms
// of Sec. 3.2 for general z and m): (s2 s1 s0) is, in every bit lane, the number of set
// inputs; at_most(m) is the per-lane predicate "sum <= m".
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void full_add(u64 a, u64 b, u64 c, u64 &s, u64 &carry)
{
  const u64 t = a ^ b;
  s = t ^ c;
  carry = (t & c) | (~t & a);
}

template <int K>
__device__ __forceinline__ void bitsum(const u64 (&x)[K], u64 &s0, u64 &s1, u64 &s2)
{
  static_assert(K >= 3 && K <= 7, "bit-sliced sum supports 3..7 inputs");
  if constexpr (K == 3) {
    full_add(x[0], x[1], x[2], s0, s1);
    s2 = 0;
  } else if constexpr (K == 4) {
    u64 a0, a1;
    full_add(x[0], x[1], x[2], a0, a1);
    s0 = a0 ^ x[3];
    const u64 b1 = a0 & x[3];
    s1 = a1 ^ b1;
    s2 = a1 & b1;
  } else if constexpr (K == 5) {
    u64 a0, a1, b1;
    full_add(x[0], x[1], x[2], a0, a1);
    full_add(x[3], x[4], a0, s0, b1);
    s1 = a1 ^ b1;
    s2 = a1 & b1;
  } else if constexpr (K == 6) {
    u64 a0, a1, b0, b1;
    full_add(x[0], x[1], x[2], a0, a1);
    full_add(x[3], x[4], x[5], b0, b1);
    s0 = a0 ^ b0;
    const u64 c1 = a0 & b0;
    full_add(a1, b1, c1, s1, s2);
  } else {
    u64 a0, a1, b0, b1, c1;
    full_add(x[0], x[1], x[2], a0, a1);
    full_add(x[3], x[4], x[5], b0, b1);
    full_add(a0, b0, x[6], s0, c1);
    full_add(a1, b1, c1, s1, s2);
  }
}

// m is wave-uniform, so the branches below are scalar.
__device__ __forceinline__ u64 at_most(u64 s0, u64 s1, u64 s2, int m)
{
  if (m >= 7) return ~0ull;
  u64 gt = 0, eq = ~0ull;
  if (m & 4) {
    eq = s2;
  } else {
    gt = s2;
    eq = ~s2;
  }
  if (m & 2) {
    eq &= s1;
  } else {
    gt |= eq & s1;
    eq &= ~s1;
  }
  if (!(m & 1)) gt |= eq & s0;
  return ~gt;
}

template <int K>
__device__ __forceinline__ u64 activity(const u64 (&x)[K], int m)
{
  u64 s0, s1, s2;
  bitsum<K>(x, s0, s1, s2);
  return at_most(s0, s1, s2, m);
}

// Exchange for one element pair; returns d per word.
template <int K, int WPT>
__device__ __forceinline__ void exchange(Elem<WPT> &ni, Elem<WPT> &nj, const Elem<WPT> (&xi)[K],
                                         const Elem<WPT> (&xj)[K], const u64 (&r)[WPT], int m,
                                         u64 (&d)[WPT])
{
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    u64 ai[K], aj[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ai[k] = xi[k].w[w];
      aj[k] = xj[k].w[w];
    }
    const u64 Ai = activity<K>(ai, m);
    const u64 Aj = activity<K>(aj, m);
    d[w] = (ni.w[w] ^ nj.w[w]) & Ai & Aj & r[w];
    ni.w[w] ^= d[w];
    nj.w[w] ^= d[w];
  }
}

// ------------------------------------------------------------------------------------
// Workgroup -> tile mapping aware of the 8 XCDs: the hardware hands consecutive
// workgroups to XCDs round-robin; renumber so that each XCD gets one contiguous range of
// tiles, whose stencil halos then meet in that XCD's own L2.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, q = b >> 3;
  return (x < rem) ? x * (per + 1) + q : rem * (per + 1) + (x - rem) * per + q;
}

// ------------------------------------------------------------------------------------
// Lattice indexing in the sublattice layout (see ka_internal.h).
// ------------------------------------------------------------------------------------
struct Site {
  int a[3];  // residues x_nu mod 4
  int p[3];  // block coordinates x_nu / 4
  int idx;   // element index sub*P + pos
};

__device__ __forceinline__ Site decode(const LatticeGeom &g, int D, int sub, int pos)
{
  Site s;
  s.a[0] = sub & 3;
  s.a[1] = (sub >> 2) & 3;
  s.a[2] = (sub >> 4) & 3;
  s.p[0] = pos % g.Q;
  const int rest = pos / g.Q;
  if (D == 3) {
    s.p[1] = rest % g.Q;
    s.p[2] = rest / g.Q;
  } else {
    s.p[1] = rest;
    s.p[2] = 0;
  }
  s.idx = sub * g.P + pos;
  return s;
}

__device__ __forceinline__ int qpow(const LatticeGeom &g, int nu)
{
  return nu == 0 ? 1 : (nu == 1 ? g.Q : g.Q * g.Q);
}

// element index of s + e_nu
__device__ __forceinline__ int step_up(const LatticeGeom &g, const Site &s, int nu)
{
  const int sub_stride = g.P << (2 * nu);
  if (s.a[nu] < 3) return s.idx + sub_stride;
  const int ps = qpow(g, nu);
  return s.idx - 3 * sub_stride + ((s.p[nu] + 1 < g.Q) ? ps : -(g.Q - 1) * ps);
}

// element index of s - e_nu
__device__ __forceinline__ int step_dn(const LatticeGeom &g, const Site &s, int nu)
{
  const int sub_stride = g.P << (2 * nu);
  if (s.a[nu] > 0) return s.idx - sub_stride;
  const int ps = qpow(g, nu);
  return s.idx + 3 * sub_stride + ((s.p[nu] > 0) ? -ps : (g.Q - 1) * ps);
}

__device__ __forceinline__ Site move_up(const LatticeGeom &g, const Site &s, int nu)
{
  Site t = s;
  t.idx = step_up(g, s, nu);
  if (s.a[nu] < 3) {
    t.a[nu] = s.a[nu] + 1;
  } else {
    t.a[nu] = 0;
    t.p[nu] = (s.p[nu] + 1 < g.Q) ? s.p[nu] + 1 : 0;
  }
  return t;
}

__device__ __forceinline__ int canonical(const LatticeGeom &g, int D, const Site &s)
{
  const int x0 = 4 * s.p[0] + s.a[0];
  const int x1 = 4 * s.p[1] + s.a[1];
  if (D == 2) return x0 + g.L * x1;
  const int x2 = 4 * s.p[2] + s.a[2];
  return x0 + g.L * (x1 + g.L * x2);
}

// Element indices of the 2D-1 neighbours of i other than j = i + e_MU, and of j other than i.
template <int D, int MU>
__device__ __forceinline__ void lattice_stencil(const LatticeGeom &g, const Site &si,
                                                const Site &sj, int (&ii)[2 * D - 1],
                                                int (&jj)[2 * D - 1])
{
  int q = 0;
#pragma unroll
  for (int nu = 0; nu < D; ++nu) {
    if (nu == MU) {
      ii[q] = step_dn(g, si, nu);
      jj[q] = step_up(g, sj, nu);
      ++q;
    } else {
      ii[q] = step_up(g, si, nu);
      jj[q] = step_up(g, sj, nu);
      ++q;
      ii[q] = step_dn(g, si, nu);
      jj[q] = step_dn(g, sj, nu);
      ++q;
    }
  }
}

// One lattice edge on the plane at base (global memory or LDS); shared by both paths.
template <int D, int MU, int WPT>
__device__ __forceinline__ void lattice_edge(u64 *nb, u64 *fb, const LatticeGeom &g, int sub,
                                             int pos, int plane, int m, uint32_t t, uint32_t c,
                                             uint32_t k0, uint32_t k1)
{
  constexpr int K = 2 * D - 1;
  const Site si = decode(g, D, sub, pos);
  const Site sj = move_up(g, si, MU);
  int ii[K], jj[K];
  lattice_stencil<D, MU>(g, si, sj, ii, jj);
  Elem<WPT> ni = ld<WPT>(nb, si.idx);
  Elem<WPT> nj = ld<WPT>(nb, sj.idx);
  Elem<WPT> xi[K], xj[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    xi[k] = ld<WPT>(nb, ii[k]);
    xj[k] = ld<WPT>(nb, jj[k]);
  }
  const uint32_t e = (uint32_t)canonical(g, D, si) * (uint32_t)D + (uint32_t)MU;
  u64 r[WPT];
  accept_words<WPT>(t, c, e, plane, k0, k1, r);
  u64 d[WPT];
  exchange<K, WPT>(ni, nj, xi, xj, r, m, d);
  u64 any = 0;
#pragma unroll
  for (int w = 0; w < WPT; ++w) any |= d[w];
  if (any) {
    st<WPT>(nb, si.idx, ni);
    st<WPT>(nb, sj.idx, nj);
    Elem<WPT> fi = ld<WPT>(fb, si.idx);
    Elem<WPT> fj = ld<WPT>(fb, sj.idx);
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      fi.w[w] |= d[w];
      fj.w[w] |= d[w];
    }
    st<WPT>(fb, si.idx, fi);
    st<WPT>(fb, sj.idx, fj);
  }
}

// One general-graph edge (u, v, e).  The 2z neighbour words are gathered; the partner's
// word is picked out of the other endpoint's row and zeroed there, so the bit-sliced sum
// over z inputs counts exactly the z-1 neighbours other than the partner.
template <int Z, int WPT>
__device__ __forceinline__ void graph_edge(u64 *nb, u64 *fb, const int32_t *adj, int4 E,
                                           int plane, int m, uint32_t t, uint32_t c,
                                           uint32_t k0, uint32_t k1)
{
  const int u = E.x, v = E.y;
  int nu[Z], nv[Z];
#pragma unroll
  for (int q = 0; q < Z; ++q) {
    nu[q] = adj[(size_t)u * Z + q];
    nv[q] = adj[(size_t)v * Z + q];
  }
  Elem<WPT> xu[Z], xv[Z];
#pragma unroll
  for (int q = 0; q < Z; ++q) {
    xu[q] = ld<WPT>(nb, nu[q]);
    xv[q] = ld<WPT>(nb, nv[q]);
  }
  Elem<WPT> ni, nj;
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    ni.w[w] = 0;
    nj.w[w] = 0;
  }
#pragma unroll
  for (int q = 0; q < Z; ++q) {
    const bool is_v = nu[q] == v;
    const bool is_u = nv[q] == u;
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      nj.w[w] |= is_v ? xu[q].w[w] : 0ull;
      xu[q].w[w] = is_v ? 0ull : xu[q].w[w];
      ni.w[w] |= is_u ? xv[q].w[w] : 0ull;
      xv[q].w[w] = is_u ? 0ull : xv[q].w[w];
    }
  }
  u64 r[WPT];
  accept_words<WPT>(t, c, (uint32_t)E.z, plane, k0, k1, r);
  u64 d[WPT];
  exchange<Z, WPT>(ni, nj, xu, xv, r, m, d);
  u64 any = 0;
#pragma unroll
  for (int w = 0; w < WPT; ++w) any |= d[w];
  if (any) {
    st<WPT>(nb, u, ni);
    st<WPT>(nb, v, nj);
    Elem<WPT> fu = ld<WPT>(fb, u);
    Elem<WPT> fv = ld<WPT>(fb, v);
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      fu.w[w] |= d[w];
      fv.w[w] |= d[w];
    }
    st<WPT>(fb, u, fu);
    st<WPT>(fb, v, fv);
  }
}

// ------------------------------------------------------------------------------------
// Global-memory class pass kernels: one launch per (class, sweep), all planes at once.
// ------------------------------------------------------------------------------------
// Thread order: a wave covers 64 consecutive positions of one lower-endpoint sublattice
// (coalesced 64 x 16 B loads); consecutive waves cover the class's other lower-endpoint
// sublattices at the same positions, so the neighbour sublattices they share are fetched
// once and then served from L2 (together with the XCD-contiguous block order).
template <int D, int MU, int WPT>
__global__ __launch_bounds__(kPassBlock) void k_pass_lattice(PassLattice a, int m)
{
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int plane = lin / a.blocks_per_plane;
  const int blk = lin - plane * a.blocks_per_plane;
  const int gid = blk * kPassBlock + (int)threadIdx.x;
  const int span = a.nsub * 64;            // threads per 64-position chunk
  const int chunk = gid / span;
  const int rem = gid - chunk * span;
  const int q = rem >> 6;
  const int pos = chunk * 64 + (rem & 63);
  if (pos >= a.g.P) return;
  const size_t off = (size_t)plane * (size_t)a.g.N * WPT;
  lattice_edge<D, MU, WPT>(a.n + off, a.f + off, a.g, a.sub[q], pos, plane, m, a.t, a.c,
                           a.key0, a.key1);
}

template <int Z, int WPT>
__global__ __launch_bounds__(kPassBlock) void k_pass_graph(PassGraph a, int m)
{
  const int lin = xcd_remap(blockIdx.x, gridDim.x);
  const int plane = lin / a.blocks_per_plane;
  const int blk = lin - plane * a.blocks_per_plane;
  const int k = blk * kPassBlock + (int)threadIdx.x;
  if (k >= a.count) return;
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  graph_edge<Z, WPT>(a.n + off, a.f + off, a.adj, a.edges[k], plane, m, a.t, a.c, a.key0,
                     a.key1);
}

// ------------------------------------------------------------------------------------
// Vertical (per-replica) population counts with wavefront ballots: lane l of the wave
// accumulates, for replica bit l, the number of the wave's 64 sites whose bit l is set.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void ballot_count(u64 x, unsigned &acc)
{
  const int lane = (int)__lane_id();
#pragma unroll
  for (int l = 0; l < 64; ++l) {
    const unsigned c = (unsigned)__popcll(__ballot((int)((x >> l) & 1ull)));
    acc += (lane == l) ? c : 0u;
  }
}

template <int WPT>
__global__ __launch_bounds__(kObsBlock) void k_observe(ObserveArgs a)
{
  const int plane = blockIdx.y;
  const int lane = (int)__lane_id();
  const int wave = (int)(blockIdx.x * (kObsBlock / 64) + threadIdx.x / 64);
  const int nwaves = (int)(gridDim.x * (kObsBlock / 64));
  const size_t off = (size_t)plane * (size_t)a.N * WPT;
  unsigned acc[3][WPT];
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int w = 0; w < WPT; ++w) acc[o][w] = 0;
  for (int base = wave * 64; base < a.N; base += nwaves * 64) {  // wave-uniform loop
    const int idx = base + lane;
    Elem<WPT> x, x0, xf;
    if (idx < a.N) {
      x = ld<WPT>(a.n + off, idx);
      x0 = ld<WPT>(a.n0 + off, idx);
      xf = ld<WPT>(a.f + off, idx);
    } else {
#pragma unroll
      for (int w = 0; w < WPT; ++w) x.w[w] = x0.w[w] = xf.w[w] = 0;
    }
#pragma unroll
    for (int w = 0; w < WPT; ++w) {
      ballot_count(x.w[w], acc[0][w]);
      ballot_count(x.w[w] & x0.w[w], acc[1][w]);
      ballot_count(x0.w[w] & ~xf.w[w], acc[2][w]);
    }
  }
#pragma unroll
  for (int o = 0; o < 3; ++o)
#pragma unroll
    for (int w = 0; w < WPT; ++w)
      if (acc[o][w])
        atomicAdd(&a.out[(size_t)o * a.R + (size_t)(plane * WPT + w) * 64 + lane],
                  (unsigned long long)acc[o][w]);
}

// ------------------------------------------------------------------------------------
// LDS-resident sweep loop: one workgroup owns one plane of a small instance, keeps n and f
// in LDS across all class passes of all requested sweeps (a barrier between passes) and
// records observations in place; only the first load and the final store touch HBM.
// ------------------------------------------------------------------------------------
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
      ballot_count(x.w[w], acc[0][w]);
      ballot_count(x.w[w] & x0.w[w], acc[1][w]);
      ballot_count(x0.w[w] & ~xf.w[w], acc[2][w]);
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

template <int WPT>
__device__ void lds_observe_due(const SweepLds &a, const u64 *sn, const u64 *sf, int plane,
                                int &qo, int64_t t_now, unsigned *cnt)
{
  while (qo < a.n_obs && a.obs_times[qo] == t_now) {
    lds_observe<WPT>(a, sn, sf, plane, qo, cnt);
    ++qo;
  }
}

template <int D, int WPT>
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
  const int per_class = a.cls.nsub * a.g.P;
  for (int s = 0; s < a.n_sweeps; ++s) {
    const uint32_t t = a.t0 + (uint32_t)s;
    for (int c = 0; c < a.C; ++c) {
      const int mu = c >> 2;
      for (int k = (int)threadIdx.x; k < per_class; k += (int)blockDim.x) {
        const int q = k / a.g.P;
        const int pos = k - q * a.g.P;
        const int sub = a.cls.sub[c][q];
        if (mu == 0)
          lattice_edge<D, 0, WPT>(sn, sf, a.g, sub, pos, plane, m, t, (uint32_t)c, a.key0, a.key1);
        else if (mu == 1)
          lattice_edge<D, 1, WPT>(sn, sf, a.g, sub, pos, plane, m, t, (uint32_t)c, a.key0, a.key1);
        else if constexpr (D == 3)
          lattice_edge<D, 2, WPT>(sn, sf, a.g, sub, pos, plane, m, t, (uint32_t)c, a.key0, a.key1);
      }
      __syncthreads();
    }
    lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)t + 1, cnt);
  }
  lds_store<WPT>(a, sn, sf, plane);
}

template <int Z, int WPT>
__global__ __launch_bounds__(kLdsBlock) void k_sweep_lds_graph(SweepLds a, int m)
{
  extern __shared__ u64 lds[];
  __shared__ unsigned cnt[3 * 64 * WPT];
  u64 *sn = lds;
  u64 *sf = lds + (size_t)a.N * WPT;
  const int plane = blockIdx.x;
  lds_load<WPT>(a, sn, sf, plane);
  int qo = 0;
  lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)a.t0, cnt);
  for (int s = 0; s < a.n_sweeps; ++s) {
    const uint32_t t = a.t0 + (uint32_t)s;
    for (int c = 0; c < a.C; ++c) {
      const int b0 = a.class_start[c], b1 = a.class_start[c + 1];
      for (int k = b0 + (int)threadIdx.x; k < b1; k += (int)blockDim.x)
        graph_edge<Z, WPT>(sn, sf, a.adj, a.edges[k], plane, m, t, (uint32_t)c, a.key0, a.key1);
      __syncthreads();
    }
    lds_observe_due<WPT>(a, sn, sf, plane, qo, (int64_t)t + 1, cnt);
  }
  lds_store<WPT>(a, sn, sf, plane);
}

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

__device__ __forceinline__ bool key_matches(u64 u, u64 prefix, int pbits)
{
  return pbits == 0 || (u >> (64 - pbits)) == prefix;
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
    __syncthreads();
    if (tid < 2 && !done[tid]) {
      const int h = tid;
      const int pb = pbits[h];
      const int dig = (64 - pb) < kDig ? (64 - pb) : kDig;
      long long cum = 0;
      int beta = 0;
      for (beta = 0; beta < (1 << dig); ++beta) {
        const long long c = hist[h][beta];
        if (cum + c >= need[h]) break;
        cum += c;
      }
      if (beta >= (1 << dig)) {  // unreachable: need <= keys under the prefix
        beta = (1 << dig) - 1;
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
  if (!a.is_lattice) return idx;
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

template <typename Kern>
hipError_t set_lds(Kern k, size_t bytes)
{
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
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

hipError_t launch_pass_graph(const PassGraph &a, int z, int m, int wpt, hipStream_t s)
{
  const dim3 grid((unsigned)(a.blocks_per_plane * a.planes));
  const dim3 block(kPassBlock);
#define KA_GR(Z, W) hipLaunchKernelGGL((k_pass_graph<Z, W>), grid, block, 0, s, a, m)
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

size_t sweep_lds_bytes(int N, int wpt) { return (size_t)2 * (size_t)N * (size_t)wpt * 8u; }

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
#define KA_LDS_L(D, W)                                                            \
  do {                                                                            \
    e = set_lds(k_sweep_lds_lattice<D, W>, lds_bytes);                            \
    if (e == hipSuccess)                                                          \
      hipLaunchKernelGGL((k_sweep_lds_lattice<D, W>), grid, block, lds_bytes, s, a, m); \
  } while (0)
#define KA_LDS_G(Z, W)                                                            \
  do {                                                                            \
    e = set_lds(k_sweep_lds_graph<Z, W>, lds_bytes);                              \
    if (e == hipSuccess)                                                          \
      hipLaunchKernelGGL((k_sweep_lds_graph<Z, W>), grid, block, lds_bytes, s, a, m); \
  } while (0)
  if (lattice) {
    if (a.g.d == 2) {
      if (wpt == 2) KA_LDS_L(2, 2); else KA_LDS_L(2, 1);
    } else {
      if (wpt == 2) KA_LDS_L(3, 2); else KA_LDS_L(3, 1);
    }
  } else {
    switch (zdeg * 4 + wpt) {
      case 3 * 4 + 1: KA_LDS_G(3, 1); break;
      case 3 * 4 + 2: KA_LDS_G(3, 2); break;
      case 4 * 4 + 1: KA_LDS_G(4, 1); break;
      case 4 * 4 + 2: KA_LDS_G(4, 2); break;
      case 5 * 4 + 1: KA_LDS_G(5, 1); break;
      case 5 * 4 + 2: KA_LDS_G(5, 2); break;
      case 6 * 4 + 1: KA_LDS_G(6, 1); break;
      case 6 * 4 + 2: KA_LDS_G(6, 2); break;
      default: return hipErrorInvalidValue;
    }
  }
#undef KA_LDS_L
#undef KA_LDS_G
  if (e != hipSuccess) return e;
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

hipError_t launch_observe(const ObserveArgs &a, int wpt, hipStream_t s)
{
  int bx = (a.N + kObsBlock - 1) / kObsBlock;
  if (bx > 512) bx = 512;
  const dim3 grid((unsigned)bx, (unsigned)a.planes);
  if (wpt == 2)
    hipLaunchKernelGGL((k_observe<2>), grid, dim3(kObsBlock), 0, s, a);
  else
    hipLaunchKernelGGL((k_observe<1>), grid, dim3(kObsBlock), 0, s, a);
  return hipGetLastError();
}

}  // namespace ka
