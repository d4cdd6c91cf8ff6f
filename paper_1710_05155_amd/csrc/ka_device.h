// ka_device.h -- device-side building blocks shared by the libka kernels.
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
#pragma once

#include <type_traits>

#include "ka_internal.h"

namespace ka {
namespace dev {


// ------------------------------------------------------------------------------------
// Three-input bitwise functions in one gfx950 instruction (v_bitop3_b32) per 32 bits.  The
// 8-bit truth table is the function evaluated on the byte patterns 0xF0, 0xCC, 0xAA standing
// for its first, second and third input.
// ------------------------------------------------------------------------------------
constexpr uint32_t kTTXor3 = (0xF0u ^ 0xCCu ^ 0xAAu) & 0xFFu;                           // a ^ b ^ c
constexpr uint32_t kTTMaj = ((0xF0u & 0xCCu) | (0xF0u & 0xAAu) | (0xCCu & 0xAAu)) & 0xFFu; // majority
constexpr uint32_t kTTAnd3 = (0xF0u & 0xCCu & 0xAAu) & 0xFFu;                           // a & b & c
constexpr uint32_t kTTXorAnd = ((0xF0u ^ 0xCCu) & 0xAAu) & 0xFFu;                       // (a ^ b) & c
constexpr uint32_t kTTXorOfAnd = (0xF0u ^ (0xCCu & 0xAAu)) & 0xFFu;                     // a ^ (b & c)
// one step of a bit-serial "greater than" from the low bit up: a = bit of x, b = bit of y (as
// an all-ones / all-zeros mask), c = "the lower bits of x exceed those of y"
constexpr uint32_t kTTGt = ((0xF0u & ~0xCCu) | (~(0xF0u ^ 0xCCu) & 0xAAu)) & 0xFFu;
constexpr uint32_t kTTNotGt = ~kTTGt & 0xFFu;

template <uint32_t TT>
__device__ __forceinline__ uint32_t bit3(uint32_t a, uint32_t b, uint32_t c)
{
  return __builtin_amdgcn_bitop3_b32(a, b, c, TT);
}

template <uint32_t TT>
__device__ __forceinline__ u64 bit3(u64 a, u64 b, u64 c)
{
  return (u64)bit3<TT>((uint32_t)a, (uint32_t)b, (uint32_t)c) |
         ((u64)bit3<TT>((uint32_t)(a >> 32), (uint32_t)(b >> 32), (uint32_t)(c >> 32)) << 32);
}

// ------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  The round keys depend only on the
// seed, so they stay in scalar registers; each round is two 32x32->64 multiplies and two
// three-way xors.
// ------------------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const u64 p0 = (u64)0xD2511F53u * (u64)c.x;
    const u64 p1 = (u64)0xCD9E8D57u * (u64)c.z;
    uint4 y;
    y.x = bit3<kTTXor3>((uint32_t)(p1 >> 32), c.y, k0);
    y.y = (uint32_t)p1;
    y.z = bit3<kTTXor3>((uint32_t)(p0 >> 32), c.w, k1);
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
// word w uses half (w & 1) of Philox(t, c, e, w >> 1).  With shared noise (noise != 0) every
// replica takes the same bit: bit 0 of output word 0 of Philox(t, c, e, 0xFFFFFFFF).  One
// Philox call either way; only its counter and the final selection differ.
template <int WPT>
__device__ __forceinline__ void accept_words(uint32_t t, uint32_t c, uint32_t e, int plane,
                                             uint32_t k0, uint32_t k1, int noise, u64 (&r)[WPT])
{
  const uint32_t w3 = noise ? 0xFFFFFFFFu : (WPT == 2 ? (uint32_t)plane : (uint32_t)plane >> 1);
  const uint4 o = philox10(make_uint4(t, c, e, w3), k0, k1);
  const u64 all = (o.x & 1u) ? ~0ull : 0ull;
  if constexpr (WPT == 2) {
    r[0] = noise ? all : lo_half(o);
    r[1] = noise ? all : hi_half(o);
  } else {
    r[0] = noise ? all : ((plane & 1) ? hi_half(o) : lo_half(o));
  }
}

// ------------------------------------------------------------------------------------
// Element = the WPT words of one site in one plane.
// ------------------------------------------------------------------------------------
template <int WPT>
struct Elem {
  u64 w[WPT];
};

// A word pair as one 16-byte vector, so that every load and store of an element is a single
// 128-bit memory instruction.
typedef u64 u64x2 __attribute__((ext_vector_type(2)));

template <int WPT>
__device__ __forceinline__ Elem<WPT> ld(const u64 *base, int idx)
{
  Elem<WPT> e;
  if constexpr (WPT == 2) {
    const u64x2 v = reinterpret_cast<const u64x2 *>(base)[idx];
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
    u64x2 v;
    v.x = e.w[0];
    v.y = e.w[1];
    reinterpret_cast<u64x2 *>(base)[idx] = v;
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
  s = bit3<kTTXor3>(a, b, c);
  carry = bit3<kTTMaj>(a, b, c);
}

template <int K>
__device__ __forceinline__ void bitsum(const u64 (&x)[K], u64 &s0, u64 &s1, u64 &s2)
{
  static_assert(K >= 2 && K <= 7, "bit-sliced sum supports 2..7 inputs");
  if constexpr (K == 2) {
    s0 = x[0] ^ x[1];
    s1 = x[0] & x[1];
    s2 = 0;
  } else if constexpr (K == 3) {
    full_add(x[0], x[1], x[2], s0, s1);
    s2 = 0;
  } else if constexpr (K == 4) {
    u64 a0, a1;
    full_add(x[0], x[1], x[2], a0, a1);
    s0 = a0 ^ x[3];
    s1 = bit3<kTTXorOfAnd>(a1, a0, x[3]);   // a1 ^ (a0 & x3)
    s2 = bit3<kTTAnd3>(a1, a0, x[3]);
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

// Per lane, sum (s2 s1 s0) <= m for a wave-uniform m in [0, 7]: a bit-serial comparison from
// the low bit up with one three-input instruction per bit; the bits of m become all-ones /
// all-zeros masks, which stay in scalar registers.  (Written with branches on m, the compiler
// turned the comparison into selects, about eight instructions per 32-bit half.)
__device__ __forceinline__ u64 at_most(u64 s0, u64 s1, u64 s2, int m)
{
  const u64 m0 = (m & 1) ? ~0ull : 0ull, m1 = (m & 2) ? ~0ull : 0ull, m2 = (m & 4) ? ~0ull : 0ull;
  const u64 g0 = s0 & ~m0;
  const u64 g1 = bit3<kTTGt>(s1, m1, g0);
  return bit3<kTTNotGt>(s2, m2, g1);
}

// The same for sums of at most three inputs (s2 = 0), where m <= 3.
__device__ __forceinline__ u64 at_most2(u64 s0, u64 s1, int m)
{
  const u64 m0 = (m & 1) ? ~0ull : 0ull, m1 = (m & 2) ? ~0ull : 0ull;
  return bit3<kTTNotGt>(s1, m1, s0 & ~m0);
}

// m <= z - 1 = K, so a sum of at most three inputs is compared with an m below 4.
template <int K>
__device__ __forceinline__ u64 activity(const u64 (&x)[K], int m)
{
  u64 s0, s1, s2;
  bitsum<K>(x, s0, s1, s2);
  if constexpr (K <= 3) return at_most2(s0, s1, m);
  else return at_most(s0, s1, s2, m);
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
    d[w] = bit3<kTTAnd3>(bit3<kTTXorAnd>(ni.w[w], nj.w[w], Ai), Aj, r[w]);   // (ni ^ nj) & Ai & Aj & r
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

// Lower-endpoint sublattice number q of lattice class (mu, r): the residues of the other
// directions are the base-4 digits of q (in increasing direction), and
// a_mu = (r - 2 * their sum) mod 4.  A class owns 4^(D-1) such sublattices; any enumeration
// of them gives the same result, since the class's edges commute.
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

// n / Q for 0 <= n < 2^31, by the multiply in lattice_qinv.
__device__ __forceinline__ int div_q(const LatticeGeom &g, int n)
{
  return (int)__umul64hi((u64)(unsigned)n << 1, g.qinv);
}

__device__ __forceinline__ Site decode(const LatticeGeom &g, int D, int sub, int pos)
{
  Site s;
  s.a[0] = sub & 3;
  s.a[1] = (sub >> 2) & 3;
  s.a[2] = (sub >> 4) & 3;
  const int rest = div_q(g, pos);
  s.p[0] = pos - rest * g.Q;
  if (D == 3) {
    s.p[2] = div_q(g, rest);
    s.p[1] = rest - s.p[2] * g.Q;
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

// Optional summary of the moved-ever words: bit (base + element) of `bits` is set once every
// word of the element's f is all ones, after which f can no longer change there and the
// exchange skips reading it.  A clear bit only means "not known to be full": f is read as
// usual.  NoSat disables the summary (f is always read where an exchange happens).
struct NoSat {};
struct FSat {
  uint32_t *bits;
  int base;    // bit index of element 0 of this plane
};

// f |= d at element i, reading f only if the summary does not already know it is full; the
// store happens only when f gains a bit, and a store that makes f all ones sets the summary
// bit (fire-and-forget atomic: other bits of the word belong to other sites).
template <int WPT, typename SatT>
__device__ __forceinline__ void moved_ever_or(u64 *fb, int i, const u64 (&d)[WPT], const Elem<WPT> &fi,
                                              SatT sat)
{
  Elem<WPT> fn = fi;
  u64 gain = 0, full = ~0ull;
#pragma unroll
  for (int w = 0; w < WPT; ++w) {
    gain |= d[w] & ~fn.w[w];
    fn.w[w] |= d[w];
    full &= fn.w[w];
  }
  if (gain) {
    st<WPT>(fb, i, fn);
    if constexpr (!std::is_same<SatT, NoSat>::value) {
      if (full == ~0ull) {
        const unsigned b = (unsigned)(sat.base + i);
        __hip_atomic_fetch_or(sat.bits + (b >> 5), 1u << (b & 31u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// The exchange across one edge (i, j) on the plane at base nb (moved-ever words at fb;
// global memory or LDS), given the element indices of i, j and of their K neighbours other
// than the partner; draw(r) supplies the edge's acceptance words once the state loads are
// issued.  Shared by every path.
template <int K, int WPT, typename Draw, typename SatT = NoSat>
__device__ __forceinline__ void edge_update_with(u64 *nb, u64 *fb, int i, int j, const int (&ii)[K],
                                                 const int (&jj)[K], int m, Draw draw, SatT sat = SatT{})
{
  Elem<WPT> ni = ld<WPT>(nb, i);
  Elem<WPT> nj = ld<WPT>(nb, j);
  Elem<WPT> xi[K], xj[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    xi[k] = ld<WPT>(nb, ii[k]);
    xj[k] = ld<WPT>(nb, jj[k]);
  }
  bool full_i = false, full_j = false;
  if constexpr (!std::is_same<SatT, NoSat>::value) {
    // issued with the state loads; the summary is small and stays in L2
    const unsigned bi = (unsigned)(sat.base + i), bj = (unsigned)(sat.base + j);
    full_i = (sat.bits[bi >> 5] >> (bi & 31u)) & 1u;
    full_j = (sat.bits[bj >> 5] >> (bj & 31u)) & 1u;
  }
  u64 r[WPT];
  draw(r);
  u64 d[WPT];
  exchange<K, WPT>(ni, nj, xi, xj, r, m, d);
  u64 any = 0;
#pragma unroll
  for (int w = 0; w < WPT; ++w) any |= d[w];
  if (any) {
    st<WPT>(nb, i, ni);
    st<WPT>(nb, j, nj);
    // f only gains a bit the first time a site changes in a replica, so it is stored
    // only then: over a run a word is rewritten at most 64 times.  Both loads are issued
    // before either is used.
    Elem<WPT> fi, fj;
    if (!full_i) fi = ld<WPT>(fb, i);
    if (!full_j) fj = ld<WPT>(fb, j);
    if (!full_i) moved_ever_or<WPT>(fb, i, d, fi, sat);
    if (!full_j) moved_ever_or<WPT>(fb, j, d, fj, sat);
  }
}

// The same exchange for the edge with canonical id e, class c, sweep t: its acceptance words
// are drawn here.
template <int K, int WPT, typename SatT = NoSat>
__device__ __forceinline__ void edge_update(u64 *nb, u64 *fb, int i, int j, const int (&ii)[K],
                                            const int (&jj)[K], uint32_t e, int plane, int m,
                                            uint32_t t, uint32_t c, uint32_t k0, uint32_t k1,
                                            int noise, SatT sat = SatT{})
{
  edge_update_with<K, WPT>(nb, fb, i, j, ii, jj, m, [&](u64 (&r)[WPT]) {
    accept_words<WPT>(t, c, e, plane, k0, k1, noise, r);
  }, sat);
}

// Element indices and canonical id of the lattice edge (si, si + e_MU): i, j, the 2D-1
// other neighbours of each, and e = i_canonical * D + MU.
template <int D, int MU>
__device__ __forceinline__ void lattice_edge_indices(const LatticeGeom &g, const Site &si, int &i,
                                                     int &j, int (&ii)[2 * D - 1],
                                                     int (&jj)[2 * D - 1], uint32_t &e)
{
  const Site sj = move_up(g, si, MU);
  lattice_stencil<D, MU>(g, si, sj, ii, jj);
  i = si.idx;
  j = sj.idx;
  e = (uint32_t)canonical(g, D, si) * (uint32_t)D + (uint32_t)MU;
}

// One lattice edge (si, si + e_MU), with si already decoded.
template <int D, int MU, int WPT>
__device__ __forceinline__ void lattice_edge_at(u64 *nb, u64 *fb, const LatticeGeom &g,
                                                const Site &si, int plane, int m, uint32_t t,
                                                uint32_t c, uint32_t k0, uint32_t k1, int noise)
{
  constexpr int K = 2 * D - 1;
  int i, j, ii[K], jj[K];
  uint32_t e;
  lattice_edge_indices<D, MU>(g, si, i, j, ii, jj, e);
  edge_update<K, WPT>(nb, fb, i, j, ii, jj, e, plane, m, t, c, k0, k1, noise);
}

// The same edge given by its sublattice and position.
template <int D, int MU, int WPT>
__device__ __forceinline__ void lattice_edge(u64 *nb, u64 *fb, const LatticeGeom &g, int sub,
                                             int pos, int plane, int m, uint32_t t, uint32_t c,
                                             uint32_t k0, uint32_t k1, int noise)
{
  lattice_edge_at<D, MU, WPT>(nb, fb, g, decode(g, D, sub, pos), plane, m, t, c, k0, k1, noise);
}

// One general-graph edge: entry k of the class-sorted edge list, record (u, v, e, 0) and
// its neighbour lists in slot-major arrays of stride `stride`: slots 0..z-2 hold the
// neighbours of u other than v, slots z-1..2z-3 those of v other than u.  All 2z state
// words are gathered at once, with no dependent adjacency-row load in front of them.
template <int Z, int WPT, typename SatT = NoSat>
__device__ __forceinline__ void graph_edge(u64 *nb, u64 *fb, const int4 *edges, const int32_t *nbr,
                                           size_t stride, int k, int plane, int m, uint32_t t,
                                           uint32_t c, uint32_t k0, uint32_t k1, int noise,
                                           SatT sat = SatT{})
{
  constexpr int K = Z - 1;
  const int4 E = edges[k];
  int iu[K], iv[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    iu[q] = nbr[(size_t)q * stride + (size_t)k];
    iv[q] = nbr[(size_t)(K + q) * stride + (size_t)k];
  }
  edge_update<K, WPT>(nb, fb, E.x, E.y, iu, iv, (uint32_t)E.z, plane, m, t, c, k0, k1, noise, sat);
}

// ------------------------------------------------------------------------------------
// Vertical (per-replica) population counts: the wave's 64 words (one site per lane) are
// transposed as a 64 x 64 bit matrix in six butterfly stages (lanes i and i ^ s swap the
// off-diagonal s x s blocks), after which lane l holds bit l of every lane's word, and its
// popcount is the number of the wave's sites whose bit l is set; lane l accumulates that
// into acc.  All 64 lanes must take part (wave-uniform control flow).
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void vertical_count(u64 x, unsigned &acc)
{
  const int lane = (int)__lane_id();
  constexpr u64 kMask[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                            0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int sh = 32 >> k;
    const u64 m = kMask[k];
    const u64 y = __shfl_xor(x, sh);
    const u64 lo = (x & m) | ((y & m) << sh);     // lanes with bit sh clear
    const u64 hi = ((y >> sh) & m) | (x & ~m);    // lanes with bit sh set
    const u64 sel = 0ull - (u64)((lane >> (5 - k)) & 1);   // all ones where bit sh is set
    x = (lo & ~sel) | (hi & sel);
  }
  acc += (unsigned)__popcll(x);
}

}  // namespace dev
}  // namespace ka
