"""Python driver for the oracle (liboracle.so, built from ka_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the benchmark's
CPU-baseline leg.  The product package never imports this module.

The oracle follows the paper (Boccagna, arXiv 1710.05155) step by step, one replica at a
time: Sec. 2.1 rules (a)-(c) for the exchange, Sec. 2.2 for the overlap observables and
Sec. 3.3 for their word-level (popcount) form.  The numpy helpers below only marshal
arrays, count occupied sites (plain sums) and pack bits into the canonical export layout.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# KA_ORACLE_LIB names another build of the same source (the sanitizer test uses it)
LIB_PATH = os.environ.get("KA_ORACLE_LIB") or os.path.join(HERE, "liboracle.so")

_lib = None


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b  # type: ignore
            _b.build()
        _lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int
        U64 = ctypes.c_uint64
        _lib.ko_philox_many.argtypes = [I64, P, P, P]
        _lib.ko_lattice.argtypes = [I32, I32, P, P, P, P]
        _lib.ko_lattice.restype = I32
        _lib.ko_rrg.argtypes = [I64, I32, U64, I64, P, P]
        _lib.ko_rrg.restype = I32
        _lib.ko_edges.argtypes = [I64, I32, P, P, P]
        _lib.ko_edges.restype = I64
        _lib.ko_colour.argtypes = [I64, I32, P, I64, P, P, P]
        _lib.ko_colour.restype = I32
        _lib.ko_init_replica.argtypes = [I64, I64, U64, I64, P]
        _lib.ko_exchange.argtypes = [I32, I32, I32, I32, P, P, I32, P, P]
        _lib.ko_pass.argtypes = [I64, I32, P, I64, P, P, P, I32, I32, I64, P, P, P]
        _lib.ko_accept_bit.argtypes = [U64, I64, I32, I64, I64]
        _lib.ko_accept_bit.restype = I32
        _lib.ko_accept_bit_shared.argtypes = [U64, I64, I32, I64]
        _lib.ko_accept_bit_shared.restype = I32
        _lib.ko_run.argtypes = [I64, I32, P, I64, P, P, P, I32, I32, U64, I64, P, I64, I64, P, P, I32]
        _lib.ko_threads.restype = I32
        _lib.ko_layered.argtypes = [I32, I32, I32, U64, P]
        _lib.ko_layered.restype = I32
        _lib.ko_layered_classes.argtypes = [I32, I32, I64, I64, P, P, P]
        _lib.ko_rs_targets.argtypes = [I64, I32, P, I32, I64, P, P]
        _lib.ko_rs_run.argtypes = [I64, I32, P, I32, U64, I64, P, U64, U64, P, P]
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------- Philox
def philox(ctr, key) -> np.ndarray:
    """Philox4x32-10 (Salmon et al., SC'11) on an (n, 4) array of counters."""
    lib = load()
    ctr = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32).reshape(-1, 4))
    key = np.ascontiguousarray(np.asarray(key, dtype=np.uint32).reshape(2))
    out = np.empty_like(ctr)
    lib.ko_philox_many(ctr.shape[0], _p(ctr), _p(key), _p(out))
    return out


# ----------------------------------------------------------------------------- graphs
@dataclass
class Graph:
    N: int
    z: int
    adj: np.ndarray    # (N, z) int32
    eu: np.ndarray     # (E,) int32, canonical edge order
    ev: np.ndarray
    ecls: np.ndarray   # (E,) int32 class of each edge
    C: int
    kind: str = "graph"
    d: int = 0
    L: int = 0

    @property
    def E(self) -> int:
        return int(self.eu.shape[0])


def lattice(d: int, L: int) -> Graph:
    """Periodic hypercubic lattice (Sec. 2.1) with the mod-4 coordinate edge classes."""
    lib = load()
    N = L ** d
    z = 2 * d
    adj = np.empty((N, z), dtype=np.int32)
    eu = np.empty(N * d, dtype=np.int32)
    ev = np.empty(N * d, dtype=np.int32)
    ecls = np.empty(N * d, dtype=np.int32)
    rc = lib.ko_lattice(d, L, _p(adj), _p(eu), _p(ev), _p(ecls))
    if rc != 0:
        raise ValueError(f"oracle: bad lattice d={d} L={L}")
    return Graph(N, z, adj, eu, ev, ecls, 4 * d, kind="lattice", d=d, L=L)


def rrg_adjacency(N: int, z: int, graph_seed: int, max_attempts: int = 1_000_000):
    """Configuration-model random regular graph with whole-pairing rejection (Sec. 2.1)."""
    lib = load()
    adj = np.empty((N, z), dtype=np.int32)
    used = ctypes.c_int64(0)
    rc = lib.ko_rrg(N, z, graph_seed, max_attempts, _p(adj), ctypes.byref(used))
    if rc != 0:
        raise ValueError(f"oracle: rrg failed rc={rc} (N={N}, z={z})")
    return adj, int(used.value)


def graph_from_adjacency(adj: np.ndarray) -> Graph:
    """Canonical edges ({u<v}, lexicographic) and greedy distance-2 edge colouring."""
    lib = load()
    adj = np.ascontiguousarray(adj, dtype=np.int32)
    N, z = adj.shape
    E = N * z // 2
    eu = np.empty(E, dtype=np.int32)
    ev = np.empty(E, dtype=np.int32)
    got = lib.ko_edges(N, z, _p(adj), _p(eu), _p(ev))
    if got != E:
        raise ValueError("oracle: adjacency is not a simple z-regular graph")
    ecls = np.empty(E, dtype=np.int32)
    C = lib.ko_colour(N, z, _p(adj), E, _p(eu), _p(ev), _p(ecls))
    return Graph(N, z, adj, eu, ev, ecls, int(C), kind="graph")


def rrg(N: int, z: int, graph_seed: int) -> Graph:
    adj, _ = rrg_adjacency(N, z, graph_seed)
    g = graph_from_adjacency(adj)
    g.kind = "rrg"
    return g


def layered_adjacency(d: int, L: int, M: int, graph_seed: int) -> np.ndarray:
    """Layered random graph (Sec. 5.2): M lattice copies, a random permutation per bond."""
    lib = load()
    N = L ** d * M
    adj = np.empty((N, 2 * d), dtype=np.int32)
    if lib.ko_layered(d, L, M, graph_seed, _p(adj)) != 0:
        raise ValueError("oracle: bad layered graph arguments")
    return adj


def layered(d: int, L: int, M: int, graph_seed: int) -> Graph:
    """Layered graph with canonical edges; classes by projection to the lattice when
    L % 4 == 0, otherwise the greedy distance-2 colouring."""
    lib = load()
    adj = layered_adjacency(d, L, M, graph_seed)
    g = graph_from_adjacency(adj)
    if L % 4 == 0:
        ecls = np.empty(g.E, dtype=np.int32)
        lib.ko_layered_classes(d, L, L ** d, g.E, _p(g.eu), _p(g.ev), _p(ecls))
        g.ecls = ecls
        g.C = 4 * d
    g.kind = "layered"
    return g


# ----------------------------------------------------------------------------- dynamics
def k_from_rho(N: int, rho: float) -> int:
    """Particle number at density rho: floor(rho*N + 1/2) in IEEE double."""
    return int(math.floor(float(rho) * float(N) + 0.5))


def init(g: Graph, K: int, seed: int, replicas) -> np.ndarray:
    """Initial occupations (nrep, N) uint8: K sites per replica (uniform K-subset)."""
    lib = load()
    reps = [int(b) for b in replicas]
    occ = np.zeros((len(reps), g.N), dtype=np.uint8)
    for q, b in enumerate(reps):
        row = np.zeros(g.N, dtype=np.uint8)
        lib.ko_init_replica(g.N, int(K), seed, b, _p(row))
        occ[q] = row
    return occ


def exchange(z: int, m: int, ni: int, nj: int, nbr_i, nbr_j, r: int):
    lib = load()
    a = np.ascontiguousarray(np.asarray(nbr_i, dtype=np.uint8))
    b = np.ascontiguousarray(np.asarray(nbr_j, dtype=np.uint8))
    oi = ctypes.c_int(0)
    oj = ctypes.c_int(0)
    lib.ko_exchange(z, m, ni, nj, _p(a), _p(b), r, ctypes.byref(oi), ctypes.byref(oj))
    return oi.value, oj.value


def class_pass(g: Graph, c: int, m: int, occ: np.ndarray, moved: np.ndarray,
               accept: np.ndarray) -> None:
    """One pass over class c with explicit acceptance bits accept[(R, E)] (in place)."""
    lib = load()
    R = occ.shape[0]
    assert occ.shape == (R, g.N) and moved.shape == (R, g.N) and accept.shape == (R, g.E)
    lib.ko_pass(g.N, g.z, _p(g.adj), g.E, _p(g.eu), _p(g.ev), _p(g.ecls), c, m, R,
                _p(occ), _p(moved), _p(accept))


def accept_bit(seed: int, t: int, c: int, e: int, b: int) -> int:
    return int(load().ko_accept_bit(seed, t, c, e, b))


def accept_bit_shared(seed: int, t: int, c: int, e: int) -> int:
    """Shared-noise variant: the one acceptance bit of edge e, class c, sweep t for every
    replica."""
    return int(load().ko_accept_bit_shared(seed, t, c, e))


def run(g: Graph, m: int, seed: int, replicas, occ: np.ndarray, moved: np.ndarray,
        t0: int, n_sweeps: int, shared: bool = False) -> None:
    """Sweeps t0 .. t0+n_sweeps-1 in place on occ/moved (rows = listed replicas); shared
    selects the shared-noise acceptance bits (one per edge for all replicas)."""
    lib = load()
    reps = np.ascontiguousarray(np.asarray(list(replicas), dtype=np.int64))
    assert occ.shape == (reps.shape[0], g.N) and moved.shape == occ.shape
    assert occ.flags["C_CONTIGUOUS"] and moved.flags["C_CONTIGUOUS"]
    lib.ko_run(g.N, g.z, _p(g.adj), g.E, _p(g.eu), _p(g.ev), _p(g.ecls), g.C, m, seed,
               reps.shape[0], _p(reps), t0, n_sweeps, _p(occ), _p(moved), 1 if shared else 0)


def threads() -> int:
    return int(load().ko_threads())


# ----------------------------------------------------------------------------- random sequential
def rs_targets(g: Graph, m: int, occ: np.ndarray) -> np.ndarray:
    """Paper's random-sequential rule (Sec. 2.1 (a)-(c)) for every state row of occ
    (n, N), site i and neighbour slot k: the target site of the move, or -1."""
    occ = np.ascontiguousarray(occ, dtype=np.uint8)
    n = occ.shape[0]
    out = np.empty((n, g.N, g.z), dtype=np.int64)
    load().ko_rs_targets(g.N, g.z, _p(g.adj), m, n, _p(occ), _p(out))
    return out


def rs_run(g: Graph, m: int, seed: int, replicas, occ: np.ndarray, moved: np.ndarray,
           a0: int, n_attempts: int) -> None:
    """Random-sequential attempts a0 .. a0+n_attempts-1 in place (rows = listed replicas):
    a uniform particle, a uniform neighbour, the move made if rules (a)-(c) allow it.
    For statistical cross-checks only; its time unit is attempts (K attempts = one
    attempt per particle)."""
    lib = load()
    reps = np.ascontiguousarray(np.asarray(list(replicas), dtype=np.int64))
    assert occ.shape == (reps.shape[0], g.N) and moved.shape == occ.shape
    assert occ.flags["C_CONTIGUOUS"] and moved.flags["C_CONTIGUOUS"]
    lib.ko_rs_run(g.N, g.z, _p(g.adj), m, seed, reps.shape[0], _p(reps), int(a0),
                  int(n_attempts), _p(occ), _p(moved))


# ----------------------------------------------------------------------------- observables
def observe(occ: np.ndarray, occ0: np.ndarray, moved: np.ndarray):
    """Per-replica integer counts (Sec. 2.2 overlap q_i = n_i(t) n_i(0); Sec. 3.3):
    density_b = sum_i n_i, overlap_b = sum_i n_i(t) n_i(0),
    persistence_b = sum_i n_i(0) (1 - moved_i)  (occupied at t=0 and never vacated)."""
    o = occ.astype(np.int64)
    o0 = occ0.astype(np.int64)
    mv = moved.astype(np.int64)
    density = o.sum(axis=1)
    overlap = (o * o0).sum(axis=1)
    persistence = (o0 * (1 - mv)).sum(axis=1)
    return density, overlap, persistence


def derived(N: int, K: int, overlap: np.ndarray, persistence: np.ndarray):
    """Replica averages: C = mean_b q_b with q_b = (overlap_b/N - rho^2)/(rho(1-rho))
    (Sec. 2.2, with the 1/N that makes q(0)=1), chi4 = N (mean q^2 - (mean q)^2), and
    the mean persistence fraction P = mean_b persistence_b / K."""
    rho = K / N
    ov = np.asarray(overlap, dtype=np.float64)
    if 0 < K < N:
        q = (ov / N - rho * rho) / (rho * (1.0 - rho))
        C = float(q.mean())
        chi4 = float(N * ((q * q).mean() - q.mean() ** 2))
    else:
        C, chi4 = float("nan"), float("nan")
    P = float(np.asarray(persistence, dtype=np.float64).mean() / K) if K > 0 else float("nan")
    return C, chi4, P


def pack(occ: np.ndarray) -> np.ndarray:
    """Canonical export layout: (R, N) 0/1 -> uint64 (W, N), bit b&63 of word b>>6 is
    replica b (least significant bit = replica 0 of the word)."""
    R, N = occ.shape
    assert R % 64 == 0
    W = R // 64
    bits = occ.astype(np.uint64).reshape(W, 64, N)
    shifts = np.arange(64, dtype=np.uint64).reshape(1, 64, 1)
    return np.bitwise_or.reduce(bits << shifts, axis=1)


def unpack(words: np.ndarray) -> np.ndarray:
    """Inverse of pack: uint64 (W, N) -> (64W, N) uint8."""
    W, N = words.shape
    shifts = np.arange(64, dtype=np.uint64).reshape(1, 64, 1)
    bits = (words.reshape(W, 1, N) >> shifts) & np.uint64(1)
    return bits.reshape(W * 64, N).astype(np.uint8)


class Sim:
    """Convenience: a set of replicas of one (graph, m, K, seed) run by the oracle."""

    def __init__(self, g: Graph, m: int, K: int, seed: int, replicas, shared: bool = False):
        self.g, self.m, self.K, self.seed = g, m, int(K), seed
        self.shared = bool(shared)
        self.replicas = [int(b) for b in replicas]
        self.occ = init(g, K, seed, self.replicas)
        self.occ0 = self.occ.copy()
        self.moved = np.zeros_like(self.occ)
        self.t = 0

    def sweep(self, n: int) -> None:
        if n > 0:
            run(self.g, self.m, self.seed, self.replicas, self.occ, self.moved, self.t, n,
                self.shared)
            self.t += n

    def observe(self):
        return observe(self.occ, self.occ0, self.moved)


class RSim:
    """Replicas of one (graph, m, K, seed) under the random-sequential dynamics, started
    from the same initial states as Sim; t counts attempts."""

    def __init__(self, g: Graph, m: int, K: int, seed: int, replicas):
        self.g, self.m, self.K, self.seed = g, m, int(K), seed
        self.replicas = [int(b) for b in replicas]
        self.occ = init(g, K, seed, self.replicas)
        self.occ0 = self.occ.copy()
        self.moved = np.zeros_like(self.occ)
        self.t = 0

    def attempt(self, n: int) -> None:
        if n > 0:
            rs_run(self.g, self.m, self.seed, self.replicas, self.occ, self.moved, self.t, n)
            self.t += n

    def observe(self):
        return observe(self.occ, self.occ0, self.moved)


# ----------------------------------------------------------------------------- spatial pairs
def displacement_shells(d: int, L: int, r2_max: int):
    """Every displacement of the periodic lattice once (components taken in the minimum
    image, |c| <= L/2), with its squared Euclidean norm, for norms <= r2_max."""
    import itertools
    out = []
    for comps in itertools.product(range(L), repeat=d):
        v = [c if c <= L // 2 else c - L for c in comps]
        r2 = sum(c * c for c in v)
        if r2 <= r2_max:
            out.append((tuple(v), r2))
    return out


def pair_sums(occ: np.ndarray, occ0: np.ndarray, d: int, L: int, r2_max: int):
    """Four-point sums of Sec. 2.2 / Sec. 3.3 over ordered site pairs (i, i+delta) with
    |delta|^2 = r2, where q_i^b = n_i^b(t) n_i^b(0):
        S2[r2]  = sum_i sum_delta sum_b q_i^b q_{i+delta}^b          (Phi(r, t))
        S11[r2] = sum_i sum_delta (sum_b q_i^b) (sum_b q_{i+delta}^b)
    and count[r2] = number of displacements in the shell.  Plain numpy rolls."""
    R = occ.shape[0]
    shape = (R,) + (L,) * d                      # x fastest -> last axis
    q = (occ.astype(np.int64) * occ0.astype(np.int64)).reshape(shape)
    qs = q.sum(axis=0)                           # sum over replicas, per site
    S2 = np.zeros(r2_max + 1, dtype=np.int64)
    S11 = np.zeros(r2_max + 1, dtype=np.int64)
    count = np.zeros(r2_max + 1, dtype=np.int64)
    for v, r2 in displacement_shells(d, L, r2_max):
        # site i at coordinates x (axis order reversed: last array axis is x_0)
        shift = tuple(-c for c in reversed(v))
        axes = tuple(range(1, d + 1))
        qj = np.roll(q, shift, axis=axes)        # qj[..., x] = q[..., x + v]
        S2[r2] += int((q * qj).sum())
        qsj = np.roll(qs, shift, axis=tuple(range(d)))
        S11[r2] += int((qs * qsj).sum())
        count[r2] += 1
    return S2, S11, count


def graph_distance_tree(i: int, j: int) -> int:
    """Distance on a graph without a geometry (Sec. 3.3): 0 for i = j, 1 otherwise."""
    return 0 if i == j else 1


def pair_sums_graph_bruteforce(occ: np.ndarray, occ0: np.ndarray, r2_max: int):
    """S2, S11, count of Sec. 2.2 / Sec. 3.3 on a graph without a geometry by an explicit
    loop over every ordered site pair (i, j), shell graph_distance_tree(i, j).  Tiny N only."""
    R, N = occ.shape
    q = occ.astype(np.int64) * occ0.astype(np.int64)
    S2 = np.zeros(r2_max + 1, dtype=np.int64)
    S11 = np.zeros(r2_max + 1, dtype=np.int64)
    count = np.zeros(r2_max + 1, dtype=np.int64)
    for i in range(N):
        for j in range(N):
            r = graph_distance_tree(i, j)
            if r > r2_max:
                continue
            S2[r] += int((q[:, i] * q[:, j]).sum())
            S11[r] += int(q[:, i].sum()) * int(q[:, j].sum())
            if i == 0:
                count[r] += 1
    return S2, S11, count


def pair_sums_graph(occ: np.ndarray, occ0: np.ndarray, r2_max: int):
    """The same sums for any N: shell 0 is the pairs (i, i), shell 1 every ordered pair with
    i != j, whose sums are the sums over all ordered pairs less the diagonal,
    sum_{i != j} a_i b_j = (sum_i a_i)(sum_j b_j) - sum_i a_i b_i."""
    R, N = occ.shape
    q = occ.astype(np.int64) * occ0.astype(np.int64)     # (R, N)
    Q = q.sum(axis=0)                                      # per site, summed over replicas
    O = q.sum(axis=1)                                      # per replica, summed over sites
    S2 = np.zeros(r2_max + 1, dtype=np.int64)
    S11 = np.zeros(r2_max + 1, dtype=np.int64)
    count = np.zeros(r2_max + 1, dtype=np.int64)
    S2[0] = int((q * q).sum())
    S11[0] = int((Q * Q).sum())
    count[0] = 1
    if r2_max >= 1:
        S2[1] = int((O.astype(object) ** 2).sum()) - int((q * q).sum())
        S11[1] = int(Q.sum()) ** 2 - int((Q * Q).sum())
        count[1] = N - 1
    return S2, S11, count


def g4_from_pairs(N: int, K: int, R: int, S2, S11):
    """g4(r) = sum over pairs at r of the replica covariance of q_i, q_j, divided by
    N rho^2 (1-rho)^2 (the normalisation under which sum_r g4 = chi4 of Sec. 2.2)."""
    rho = K / N
    cov = np.asarray(S2, dtype=np.float64) / R - np.asarray(S11, dtype=np.float64) / (R * R)
    return cov / (N * rho * rho * (1.0 - rho) ** 2)
