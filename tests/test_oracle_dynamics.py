"""Pins of the oracle's initial state and dynamics against what the paper and the
mathematics fix (no implementation exists to compare against):

- initial state: exactly K particles per replica, uniform over K-subsets (chi-square on a
  tiny system), the occupied sites carry the K smallest keys;
- particle-number conservation (Sec. 2.1);
- detailed balance / flat measure (Sec. 2.1 remark after rule (c), Sec. 2.2): the one-pass
  transition matrix of every class, enumerated exhaustively over all 2^N states, is
  symmetric, hence doubly stochastic, so the uniform measure on each particle-number
  sector is stationary;
- blocked configurations stay frozen forever (Sec. 2.2, dynamical arrest);
- single particle (K=1): a random walk whose return probability is the trace of the
  product of one-walker class matrices; m = z-1 (no constraint): the exclusion process is
  a stirring process, so E[overlap] = sum_ij n0_i P_t(i,j) n0_j (self-duality);
- schedule bookkeeping: split invariance and replica independence;
- observables at t = 0: overlap = persistence = density = K, C(0) = 1;
- shared-noise variant (one acceptance bit per edge for all replicas, as the paper's
  multispin step applies one random choice to all replicas of a word): replicas started
  equal stay equal, and at m = z-1 every replica is moved by one and the same permutation of
  the sites, found by following single particles.
"""
import itertools
import math

import numpy as np
import pytest


# ------------------------------------------------------------------------ initial state
def test_init_exact_count_and_extremes(oracle):
    g = oracle.lattice(2, 8)
    for K in (0, 1, 17, 63, 64):
        occ = oracle.init(g, K, 5, range(8))
        assert (occ.sum(axis=1) == K).all()


def test_init_uniform_k_subsets(oracle):
    """N=4 sites (any graph: init ignores edges), K=2: six subsets, each w.p. 1/6."""
    adj = np.array([[1, 3], [0, 2], [1, 3], [0, 2]], dtype=np.int32)
    g = oracle.graph_from_adjacency(adj)
    R = 6000
    occ = oracle.init(g, 2, 77, range(R))
    codes = occ @ np.array([1, 2, 4, 8])
    vals, counts = np.unique(codes, return_counts=True)
    assert len(vals) == 6
    exp = R / 6
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 30.0, chi2  # 5 dof; 30 is p ~ 1.5e-5


def test_particle_count_from_density(oracle):
    """K = floor(rho N + 1/2) in IEEE double: the counts of the measured workloads (2D L=64
    at rho=0.70; 3D L=128 at 0.80, 0.85, 0.88; RRG N=2^20 at 0.50..0.75), and ties at an
    exact half round up (never to even)."""
    assert oracle.k_from_rho(64 ** 2, 0.70) == 2867
    assert [oracle.k_from_rho(128 ** 3, r) for r in (0.80, 0.85, 0.88)] == [1677722, 1782579, 1845494]
    assert [oracle.k_from_rho(2 ** 20, r) for r in (0.50, 0.55, 0.60, 0.65, 0.70, 0.75)] == \
        [524288, 576717, 629146, 681574, 734003, 786432]
    assert oracle.k_from_rho(2, 0.25) == 1          # rho N = 0.5
    assert oracle.k_from_rho(8, 0.3125) == 3        # 2.5
    assert oracle.k_from_rho(16, 0.90625) == 15     # 14.5
    assert oracle.k_from_rho(10, 0.0) == 0 and oracle.k_from_rho(10, 1.0) == 10


def test_init_occupies_smallest_keys(oracle):
    g = oracle.lattice(2, 8)
    seed, K = 123456789, 20
    for b in (0, 1, 2, 63, 64, 200):
        occ = oracle.init(g, K, seed, [b])[0]
        ctr = np.array([[0, 0xFFFFFFFF, i, b >> 1] for i in range(g.N)], dtype=np.uint32)
        out = oracle.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32]).astype(np.uint64)
        h = b & 1
        u = out[:, 2 * h] | (out[:, 2 * h + 1] << np.uint64(32))
        occupied = u[occ == 1]
        empty = u[occ == 0]
        assert occupied.max() < empty.min()


# ------------------------------------------------------------------------ conservation
@pytest.mark.parametrize("kind", ["2d", "3d", "rrg"])
def test_particle_number_conserved(oracle, kind):
    if kind == "2d":
        g, m = oracle.lattice(2, 12), 2
    elif kind == "3d":
        g, m = oracle.lattice(3, 8), 3
    else:
        g, m = oracle.rrg(200, 4, 9), 2
    for rho in (0.3, 0.7, 0.9):
        K = oracle.k_from_rho(g.N, rho)
        s = oracle.Sim(g, m, K, 31, range(0, 256, 37))
        for _ in range(4):
            s.sweep(5)
            dens, ov, pers = s.observe()
            assert (dens == K).all()
            assert (pers <= ov).all() and (ov <= K).all()


# ------------------------------------------------------------------------ detailed balance
def _class_transition_pairs(oracle, g, c, m):
    """All (state, successor) pairs of one class pass with each acceptance pattern."""
    edges = [e for e in range(g.E) if g.ecls[e] == c]
    n_pat = 1 << len(edges)
    S = 1 << g.N
    states = np.arange(S, dtype=np.int64)
    bits = ((states[:, None] >> np.arange(g.N)) & 1).astype(np.uint8)
    occ = np.repeat(bits, n_pat, axis=0)
    moved = np.zeros_like(occ)
    accept = np.zeros((S * n_pat, g.E), dtype=np.uint8)
    pats = np.arange(n_pat)
    for q, e in enumerate(edges):
        accept[:, e] = np.tile((pats >> q) & 1, S)
    oracle.class_pass(g, c, m, occ, moved, accept)
    succ = (occ.astype(np.int64) << np.arange(g.N)).sum(axis=1)
    src = np.repeat(states, n_pat)
    return src, succ, n_pat


def _assert_symmetric(src, succ, S):
    fwd = np.unique(src * S + succ, return_counts=True)
    bwd = np.unique(succ * S + src, return_counts=True)
    assert np.array_equal(fwd[0], bwd[0]) and np.array_equal(fwd[1], bwd[1])


@pytest.mark.parametrize("m", [0, 1, 2, 3])
def test_detailed_balance_2d_L4_exhaustive(oracle, m):
    g = oracle.lattice(2, 4)  # N = 16: 65536 states
    for c in range(g.C):
        src, succ, n_pat = _class_transition_pairs(oracle, g, c, m)
        _assert_symmetric(src, succ, 1 << g.N)
        # particle number conserved by every transition
        pc = np.array([bin(x).count("1") for x in range(1 << g.N)])
        assert np.array_equal(pc[src], pc[succ])


@pytest.mark.parametrize("z,m", [(3, 0), (3, 1), (3, 2), (4, 1), (4, 2)])
def test_detailed_balance_rrg_exhaustive(oracle, z, m):
    g = oracle.rrg(10 if z == 3 else 8, z, 4)
    for c in range(g.C):
        src, succ, _ = _class_transition_pairs(oracle, g, c, m)
        _assert_symmetric(src, succ, 1 << g.N)


# ------------------------------------------------------------------------ frozen configurations
def _run_custom(oracle, g, m, occ0, seed, n):
    occ = occ0.copy()
    moved = np.zeros_like(occ)
    oracle.run(g, m, seed, range(occ.shape[0]), occ, moved, 0, n)
    return occ, moved


def _coords(g):
    idx = np.arange(g.N)
    return [(idx // g.L ** k) % g.L for k in range(g.d)]


def test_frozen_double_row_2d(oracle):
    """2D, m=2: a fully occupied pair of adjacent periodic rows can never move."""
    g = oracle.lattice(2, 12)
    x, y = _coords(g)
    block = (y == 3) | (y == 4)
    rng = np.random.default_rng(3)
    occ0 = (rng.random((64, g.N)) < 0.4).astype(np.uint8)
    occ0[:, block] = 1
    occ, moved = _run_custom(oracle, g, 2, occ0, 11, 30)
    assert (occ[:, block] == 1).all() and (moved[:, block] == 0).all()
    assert (occ.sum(1) == occ0.sum(1)).all()
    assert (moved[:, ~block].sum() > 0)  # the background does move


@pytest.mark.parametrize("shape", ["rod", "planes"])
def test_frozen_blocks_3d(oracle, shape):
    """3D, m=3: a full periodic 2x2 rod, or a full pair of adjacent planes, is frozen."""
    g = oracle.lattice(3, 8)
    x, y, zc = _coords(g)
    block = ((x == 2) | (x == 3)) & ((y == 5) | (y == 6)) if shape == "rod" else ((zc == 1) | (zc == 2))
    rng = np.random.default_rng(4)
    occ0 = (rng.random((16, g.N)) < 0.5).astype(np.uint8)
    occ0[:, block] = 1
    occ, moved = _run_custom(oracle, g, 3, occ0, 12, 10)
    assert (occ[:, block] == 1).all() and (moved[:, block] == 0).all()


def test_full_empty_and_single_hole(oracle):
    g = oracle.lattice(2, 8)
    for K in (0, g.N):
        s = oracle.Sim(g, 2, K, 1, range(64))
        s.sweep(5)
        assert (s.moved == 0).all()
    # one hole and m < z-1: every neighbour of the hole has z-1 occupied other neighbours
    for m in range(g.z - 1):
        s = oracle.Sim(g, m, g.N - 1, 1, range(64))
        s.sweep(5)
        assert (s.moved == 0).all()
    s = oracle.Sim(g, g.z - 1, g.N - 1, 1, range(64))
    s.sweep(5)
    assert s.moved.sum() > 0


# ------------------------------------------------------------------------ exact statistics
def _walker_matrix(g, c):
    """Single-walker kernel of one class pass: on a class edge the walker hops w.p. 1/2."""
    P = np.eye(g.N)
    for e in range(g.E):
        if g.ecls[e] == c:
            i, j = int(g.eu[e]), int(g.ev[e])
            P[i, i] = P[j, j] = 0.5
            P[i, j] = P[j, i] = 0.5
    return P


def _sweep_matrix(g):
    P = np.eye(g.N)
    for c in range(g.C):
        P = P @ _walker_matrix(g, c)
    return P


@pytest.mark.parametrize("kind", ["2d", "rrg"])
def test_single_particle_return_probability(oracle, kind):
    g = oracle.lattice(2, 8) if kind == "2d" else oracle.rrg(48, 3, 2)
    R = 4096
    s = oracle.Sim(g, 0, 1, 2024, range(R))
    Ps = _sweep_matrix(g)
    Pt = np.eye(g.N)
    for t in range(1, 6):
        s.sweep(1)
        Pt = Pt @ Ps
        _, ov, _ = s.observe()
        # start sites are uniform (K=1 uniform subset); E[overlap] = tr(P_t)/N
        p = np.trace(Pt) / g.N
        est = ov.mean()
        se = math.sqrt(p * (1 - p) / R)
        assert abs(est - p) < 5 * se + 1e-12, (t, est, p)


def test_stirring_self_duality_unconstrained(oracle):
    """m = z-1: the exclusion process with swap probability 1/2 on each class edge is a
    stirring process; E[overlap_b(t)] = n0_b^T P_t n0_b with P_t the walker kernel."""
    g = oracle.lattice(2, 8)
    K = g.N // 2
    R = 2048
    s = oracle.Sim(g, g.z - 1, K, 99, range(R))
    Ps = _sweep_matrix(g)
    Pt = np.eye(g.N)
    n0 = s.occ0.astype(np.float64)
    for t in range(1, 5):
        s.sweep(1)
        Pt = Pt @ Ps
        _, ov, _ = s.observe()
        expect = np.einsum("bi,ij,bj->b", n0, Pt, n0)
        diff = ov - expect
        z = diff.mean() / (diff.std(ddof=1) / math.sqrt(R))
        assert abs(z) < 5.0, (t, z)


def test_stirring_two_point_stationary(oracle):
    """After many unconstrained sweeps the state is uniform on the K-sector:
    P(n_i n_j = 1) = K(K-1)/(N(N-1)) for a neighbour pair."""
    g = oracle.lattice(2, 8)
    K = 24
    R = 4096
    s = oracle.Sim(g, g.z - 1, K, 5, range(R))
    s.sweep(40)
    occ = s.occ.astype(np.float64)
    pair = (occ[:, g.eu] * occ[:, g.ev]).mean()  # averaged over replicas and edges
    p = K * (K - 1) / (g.N * (g.N - 1))
    # edges within a replica are correlated; use the replica means for the error bar
    per_rep = (occ[:, g.eu] * occ[:, g.ev]).mean(axis=1)
    se = per_rep.std(ddof=1) / math.sqrt(R)
    assert abs(pair - p) < 5 * se
    site = occ.mean()
    assert abs(site - K / g.N) < 1e-12  # exact: conservation


# ------------------------------------------------------------------------ bookkeeping
def test_split_invariance_and_replica_independence(oracle):
    g = oracle.lattice(3, 8)
    K = oracle.k_from_rho(g.N, 0.6)
    a = oracle.Sim(g, 3, K, 8, [0, 5, 64, 130, 255])
    a.sweep(7)
    b = oracle.Sim(g, 3, K, 8, [0, 5, 64, 130, 255])
    b.sweep(3)
    b.sweep(4)
    assert np.array_equal(a.occ, b.occ) and np.array_equal(a.moved, b.moved)
    c = oracle.Sim(g, 3, K, 8, [130])
    c.sweep(7)
    assert np.array_equal(c.occ[0], a.occ[3]) and np.array_equal(c.moved[0], a.moved[3])


def test_observables_at_time_zero(oracle):
    g = oracle.rrg(128, 4, 3)
    K = oracle.k_from_rho(g.N, 0.55)
    s = oracle.Sim(g, 2, K, 3, range(64))
    dens, ov, pers = s.observe()
    assert (dens == K).all() and (ov == K).all() and (pers == K).all()
    C, chi4, P = oracle.derived(g.N, K, ov, pers)
    assert abs(C - 1.0) < 1e-12 and abs(chi4) < 1e-9 and P == 1.0
    s.sweep(10)
    _, ov2, pers2 = s.observe()
    assert (pers2 <= pers).all()
    s.sweep(10)
    _, ov3, pers3 = s.observe()
    assert (pers3 <= pers2).all()


def test_pack_roundtrip(oracle):
    rng = np.random.default_rng(0)
    occ = (rng.random((128, 37)) < 0.5).astype(np.uint8)
    w = oracle.pack(occ)
    assert w.shape == (2, 37) and w.dtype == np.uint64
    assert np.array_equal(oracle.unpack(w), occ)
    # replica 65 is bit 1 of word 1
    assert ((w[1] >> np.uint64(1)) & np.uint64(1)).astype(np.uint8).tolist() == occ[65].tolist()


def test_every_replica_has_its_own_noise(oracle):
    """Replicas are independent chains: 256 replicas started from one and the same state
    must all follow different trajectories, and 256 initial states must all differ.  A
    counter or half-word mix-up that lets two replicas share random bits fails this."""
    g = oracle.lattice(2, 8)
    rng = np.random.default_rng(1)
    start = (rng.random(g.N) < 0.5).astype(np.uint8)
    occ = np.repeat(start[None, :], 256, axis=0)
    moved = np.zeros_like(occ)
    oracle.run(g, g.z - 1, 42, range(256), occ, moved, 0, 3)
    assert len({row.tobytes() for row in occ}) == 256
    occ0 = oracle.init(g, 20, 42, range(256))
    assert len({row.tobytes() for row in occ0}) == 256


@pytest.mark.parametrize("kind", ["lattice", "rrg"])
def test_shared_noise_couples_equal_replicas(oracle, kind):
    """With shared noise, replicas started from the same state stay identical for ever,
    while with independent noise they separate; replicas started apart stay conserved."""
    g = oracle.lattice(2, 8) if kind == "lattice" else oracle.rrg(60, 4, 3)
    rng = np.random.default_rng(5)
    start = (rng.random(g.N) < 0.55).astype(np.uint8)
    other = (rng.random(g.N) < 0.55).astype(np.uint8)
    for shared in (True, False):
        occ = np.stack([start, start, other, start]).astype(np.uint8)
        moved = np.zeros_like(occ)
        oracle.run(g, 2, 17, [0, 1, 2, 63], occ, moved, 0, 25, shared=shared)
        same = [np.array_equal(occ[0], occ[k]) and np.array_equal(moved[0], moved[k]) for k in (1, 3)]
        assert all(same) if shared else not any(same)
        assert int(occ[2].sum()) == int(other.sum()) and int(occ[0].sum()) == int(start.sum())
        assert not np.array_equal(occ[0], start)


@pytest.mark.parametrize("kind", ["lattice", "rrg"])
def test_shared_noise_stirring_is_one_permutation(oracle, kind):
    """At m = z-1 an accepted edge always swaps its two sites' contents (equal contents make
    the swap a no-op), so with shared noise every replica is moved by one permutation pi of
    the sites.  pi is found by following a single particle from each site (K = 1 replicas);
    then a many-particle replica must end as its start moved by pi, and its moved-ever mask
    must cover every site whose final content differs from its start."""
    g = oracle.lattice(2, 8) if kind == "lattice" else oracle.rrg(48, 3, 9)
    N = g.N
    rng = np.random.default_rng(11)
    many = (rng.random(N) < 0.5).astype(np.uint8)
    occ = np.zeros((N + 1, N), dtype=np.uint8)
    occ[np.arange(N), np.arange(N)] = 1
    occ[N] = many
    moved = np.zeros_like(occ)
    oracle.run(g, g.z - 1, 23, range(N + 1), occ, moved, 0, 7, shared=True)
    pi = occ[:N].argmax(axis=1)
    assert (occ[:N].sum(axis=1) == 1).all()
    assert sorted(pi.tolist()) == list(range(N)), "not a permutation"
    expect = np.zeros(N, dtype=np.uint8)
    expect[pi] = many
    assert np.array_equal(occ[N], expect)
    assert (moved[N][occ[N] != many] == 1).all()
    assert (pi != np.arange(N)).any()


# ------------------------------------------------------------------------ four-point sums
def test_pair_sums_brute_force_tiny(oracle):
    """S2, S11 against an explicit double loop over site pairs (2D L=4, r2 <= 8)."""
    g = oracle.lattice(2, 4)
    s = oracle.Sim(g, 2, 9, 5, range(64))
    s.sweep(3)
    S2, S11, count = oracle.pair_sums(s.occ, s.occ0, 2, 4, 8)
    q = (s.occ.astype(np.int64) * s.occ0)
    L = 4
    bS2 = np.zeros(9, dtype=np.int64)
    bS11 = np.zeros(9, dtype=np.int64)
    for i in range(16):
        for j in range(16):
            dx = abs(i % L - j % L)
            dy = abs(i // L - j // L)
            dx, dy = min(dx, L - dx), min(dy, L - dy)
            r2 = dx * dx + dy * dy
            if r2 <= 8:
                bS2[r2] += int((q[:, i] * q[:, j]).sum())
                bS11[r2] += int(q[:, i].sum() * q[:, j].sum())
    assert np.array_equal(S2, bS2) and np.array_equal(S11, bS11)
    assert count.sum() == 16 and count[0] == 1 and count[1] == 4


@pytest.mark.parametrize("d,L", [(2, 8), (3, 4)])
def test_pair_sums_cover_chi4(oracle, d, L):
    """Summed over every displacement: sum S2 = sum_b overlap_b^2, sum S11 =
    (sum_b overlap_b)^2, S2[0] = sum_b overlap_b; hence sum_r g4(r) = chi4."""
    g = oracle.lattice(d, L)
    K = oracle.k_from_rho(g.N, 0.6)
    s = oracle.Sim(g, g.z // 2, K, 7, range(128))
    s.sweep(4)
    _, ov, pers = s.observe()
    r2_all = d * (L // 2) ** 2
    S2, S11, count = oracle.pair_sums(s.occ, s.occ0, d, L, r2_all)
    assert count.sum() == g.N
    assert S2.sum() == int((ov.astype(np.int64) ** 2).sum())
    assert S11.sum() == int(ov.sum()) ** 2
    assert S2[0] == int(ov.sum())
    g4 = oracle.g4_from_pairs(g.N, K, 128, S2, S11)
    _, chi4, _ = oracle.derived(g.N, K, ov, pers)
    assert abs(g4.sum() - chi4) < 1e-9 * max(1.0, abs(chi4))


@pytest.mark.parametrize("N,z,R", [(12, 3, 64), (20, 4, 128)])
def test_pair_sums_graph_brute_force_tiny(oracle, N, z, R):
    """Graphs without a geometry (Sec. 3.3: distance 0 for i = j, 1 otherwise): the closed
    form used at any size equals the explicit loop over every ordered site pair; the shells
    cover all pairs, so sum S2 = sum_b overlap_b^2, sum S11 = (sum_b overlap_b)^2, and
    sum_r g4(r) = chi4."""
    adj, _ = oracle.rrg_adjacency(N, z, 5)
    g = oracle.graph_from_adjacency(adj)
    K = oracle.k_from_rho(N, 0.5)
    s = oracle.Sim(g, 1, K, 3, range(R))
    s.sweep(3)
    for r2_max in (0, 1, 3):
        got = oracle.pair_sums_graph(s.occ, s.occ0, r2_max)
        want = oracle.pair_sums_graph_bruteforce(s.occ, s.occ0, r2_max)
        for a, b in zip(got, want):
            assert np.array_equal(a, b), r2_max
    S2, S11, count = oracle.pair_sums_graph(s.occ, s.occ0, 1)
    _, ov, pers = s.observe()
    assert count.tolist() == [1, N - 1]
    assert S2.sum() == int((ov.astype(np.int64) ** 2).sum()) and S2[0] == int(ov.sum())
    assert S11.sum() == int(ov.sum()) ** 2
    g4 = oracle.g4_from_pairs(N, K, R, S2, S11)
    _, chi4, _ = oracle.derived(N, K, ov, pers)
    assert abs(g4.sum() - chi4) < 1e-9 * max(1.0, abs(chi4))
