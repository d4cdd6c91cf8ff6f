"""Pins of the oracle's random-sequential mode: the paper's own algorithm (Sec. 2.1), one
uniformly chosen particle and neighbour per attempt, moved under rules (a)-(c).  The mode
exists for statistical cross-checks of the class schedule, never for parity.

- its one-attempt transition matrix, enumerated exhaustively over all 2^16 states of the
  2D L=4 lattice, is symmetric for every m (the reversibility remarked after rule (c));
- its rule agrees with the class schedule's exchange rule on every local configuration;
- at m = z-1 (no constraint) it is the exclusion process, whose one-point function is
  linear: E[n(a+1) | n(a)] = M n(a) with M = I + (A/z - I)/K, so E[overlap(a)] =
  n0^T M^a n0 exactly (K = 1: a simple random walk);
- blocked configurations stay frozen under it too;
- cross-check: after one fitted time scale its C(t) follows the class schedule's C(t),
  including the plateau left by particles that can never move.
"""
import math

import numpy as np
import pytest


def _states(N):
    S = 1 << N
    states = np.arange(S, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(N)) & 1).astype(np.uint8)
    return states, bits


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_rs_transition_matrix_symmetric_2d_L4(oracle, m):
    g = oracle.lattice(2, 4)  # N = 16: 65536 states
    states, bits = _states(g.N)
    tgt = oracle.rs_targets(g, m, bits)                    # (S, N, z)
    S = states.shape[0]
    src = np.repeat(states, g.N * g.z)
    i = np.tile(np.repeat(np.arange(g.N), g.z), S)
    j = tgt.reshape(-1)
    occupied = ((src >> i) & 1) == 1                        # an attempt picks a particle
    src, i, j = src[occupied], i[occupied], j[occupied]
    succ = np.where(j >= 0, src ^ (1 << i) ^ (1 << np.maximum(j, 0)), src)
    # every attempt has weight 1/(K z) and K is conserved: compare the multisets
    pc = np.array([bin(x).count("1") for x in range(S)])
    assert np.array_equal(pc[src], pc[succ])
    fwd = np.unique(src * S + succ, return_counts=True)
    bwd = np.unique(succ * S + src, return_counts=True)
    assert np.array_equal(fwd[0], bwd[0]) and np.array_equal(fwd[1], bwd[1])
    assert (j >= 0).any() or m == 0


def test_rs_rule_matches_class_exchange_rule(oracle):
    """(a)-(c) with the counts over all neighbours is the class rule's 'at most m
    occupied neighbours other than the partner, on both ends' (2D L=4 lattice: 429 of
    3000 sampled states, every particle and neighbour in them, every m)."""
    g = oracle.lattice(2, 4)
    _, bits = _states(g.N)
    rng = np.random.default_rng(2)
    rows = bits[rng.choice(bits.shape[0], 3000, replace=False)]
    for m in range(g.z):
        tgt = oracle.rs_targets(g, m, rows)
        for s in range(0, rows.shape[0], 7):
            occ = rows[s]
            for i in np.flatnonzero(occ):
                for k in range(g.z):
                    j = int(g.adj[i, k])
                    if occ[j]:
                        assert tgt[s, i, k] == -1
                        continue
                    nbr_i = [occ[a] for a in g.adj[i] if a != j]
                    nbr_j = [occ[b] for b in g.adj[j] if b != i]
                    ni, nj = oracle.exchange(g.z, m, 1, 0, nbr_i, nbr_j, 1)
                    assert (tgt[s, i, k] == j) == (ni == 0 and nj == 1)


@pytest.mark.parametrize("K", [1, 2, 32])
def test_rs_exclusion_one_point_function(oracle, K):
    """m = z-1: E[overlap(a)] = n0^T M^a n0, M = I + (A/z - I)/K, after a attempts (the
    particle of each attempt uniform among the K, its neighbour uniform among the z)."""
    g = oracle.lattice(2, 8)
    R = 2048
    s = oracle.RSim(g, g.z - 1, K, 17, range(R))
    A = np.zeros((g.N, g.N))
    for i in range(g.N):
        for j in g.adj[i]:
            A[i, j] += 1.0
    M = np.eye(g.N) + (A / g.z - np.eye(g.N)) / K
    n0 = s.occ0.astype(np.float64)
    done = 0
    for a in sorted({1, 2, 5, K, 2 * K, 4 * K}):
        s.attempt(a - done)
        done = a
        _, ov, _ = s.observe()
        expect = np.einsum("bi,ij,bj->b", n0, np.linalg.matrix_power(M, a), n0)
        diff = ov - expect
        sd = diff.std(ddof=1)
        if sd == 0:
            assert abs(diff.mean()) < 1e-9, (a, diff.mean())
            continue
        zsc = diff.mean() / (sd / math.sqrt(R))
        assert abs(zsc) < 5.0, (a, zsc)


def test_rs_conservation_split_and_bounds(oracle):
    g = oracle.rrg(200, 4, 9)
    K = oracle.k_from_rho(g.N, 0.6)
    a = oracle.RSim(g, 2, K, 5, range(16))
    a.attempt(3000)
    b = oracle.RSim(g, 2, K, 5, range(16))
    b.attempt(1000)
    b.attempt(2000)
    assert np.array_equal(a.occ, b.occ) and np.array_equal(a.moved, b.moved)
    dens, ov, pers = a.observe()
    assert (dens == K).all() and (pers <= ov).all() and (ov <= K).all()
    assert a.moved.sum() > 0
    # every site whose occupation differs from the start has been marked as moved
    assert (a.moved[a.occ != a.occ0] == 1).all()


def test_rs_frozen_double_row_2d(oracle):
    """2D, m=2: a fully occupied pair of adjacent periodic rows never moves."""
    g = oracle.lattice(2, 12)
    y = np.arange(g.N) // g.L
    block = (y == 3) | (y == 4)
    rng = np.random.default_rng(8)
    R = 32
    occ = (rng.random((R, g.N)) < 0.4).astype(np.uint8)
    occ[:, block] = 1
    moved = np.zeros_like(occ)
    oracle.rs_run(g, 2, 3, range(R), occ, moved, 0, 20000)
    assert (occ[:, block] == 1).all() and (moved[:, block] == 0).all()
    assert moved[:, ~block].sum() > 0


@pytest.mark.parametrize("m,rho", [(1, 0.5), (2, 0.7)])
def test_rs_cross_check_class_schedule(oracle, m, rho):
    """The class schedule and the paper's random-sequential dynamics are the same model up
    to the time unit: with one fitted scale (attempts per particle per sweep), the
    random-sequential C(t) follows the class schedule's at every sampled time.  The fitted
    scale lies above the naive 2 hops per sweep, because a sweep's four classes along one
    direction visit its residues in increasing order, so a particle can advance up to four
    sites along that direction in one sweep."""
    g = oracle.lattice(2, 16)
    K = oracle.k_from_rho(g.N, rho)
    R = 256
    cls = oracle.Sim(g, m, K, 7, range(R))
    ts = [1, 2, 4, 8, 16, 32, 64]
    Cc, done = [], 0
    for t in ts:
        cls.sweep(t - done)
        done = t
        _, ov, _ = cls.observe()
        Cc.append(oracle.derived(g.N, K, ov, ov)[0])
    rs = oracle.RSim(g, m, K, 7, range(R, 2 * R))
    taus = np.arange(0.25, 8 * 64 + 0.01, 0.25)
    Cr, done = [], 0
    for tau in taus:
        a = int(round(tau * K))
        rs.attempt(a - done)
        done = a
        _, ov, _ = rs.observe()
        Cr.append(oracle.derived(g.N, K, ov, ov)[0])
    Cr = np.asarray(Cr)
    best = None
    for alpha in np.arange(0.5, 8.0, 0.01):
        r = np.array([Cc[q] - np.interp(alpha * t, taus, Cr) for q, t in enumerate(ts)])
        rms = float(np.sqrt((r * r).mean()))
        if best is None or rms < best[1]:
            best = (alpha, rms)
    alpha, rms = best
    assert 1.0 < alpha < 7.5, alpha
    assert rms < 0.03, (alpha, rms)
