"""GPU parity: the HIP path (through the C ABI) against the oracle, bit for bit.

The state is integer bit data and the observables are integer counts, so the bar is exact
equality: packed occupations n, the t=0 copy n0, the moved-ever mask f, and the per-replica
density / overlap / persistence counts.  Cases span both kernel paths (one launch per
class pass over global memory, and the LDS-resident sweep loop), word layouts with one and
two words per thread (R = 64, 128, 192, 256, 320), lattices whose side is not a power of
two, random regular graphs of degree 3..6, every activation number m, and the degenerate
particle numbers K = 0, 1, N-1, N.
"""
import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _state_equal(sim, orc):
    n, n0, f, t = ka.ka_get_state(sim)
    assert t == orc.t
    from oracle import oracle as o
    assert np.array_equal(n0, o.pack(orc.occ0)), "n0 differs"
    assert np.array_equal(n, o.pack(orc.occ)), "n differs"
    assert np.array_equal(f, o.pack(orc.moved)), "f differs"


def _observe_equal(sim, orc):
    t, dens, ov, pers = ka.ka_observe(sim)
    odens, oov, opers = orc.observe()
    assert t == orc.t
    assert np.array_equal(dens, odens) and np.array_equal(ov, oov) and np.array_equal(pers, opers)


def _check_case(oracle, lib_graph, or_graph, m, K, seed, R, chunks, path, options=()):
    _say(f"N={or_graph.N} z={or_graph.z} m={m} K={K} R={R} path={path} chunks={chunks} options={options}")
    sim = ka.ka_init_k(lib_graph, m, K, seed, R)
    for opt, value in options:
        ka.ka_set_option(sim, opt, value)
    if path:
        try:
            ka.ka_set_option(sim, ka.KA_OPT_PATH, path)
        except ka.KaError:
            sim.free()
            pytest.skip("this instance does not fit the LDS-resident path on this device")
    orc = oracle.Sim(or_graph, m, K, seed, range(R))
    _state_equal(sim, orc)
    _observe_equal(sim, orc)
    for n in chunks:
        ka.ka_sweep(sim, n)
        orc.sweep(n)
        _state_equal(sim, orc)
        _observe_equal(sim, orc)
    sim.free()


LATTICE_CASES = [
    # d, L, m, rho, R
    (2, 4, 2, 0.5, 64),
    (2, 8, 0, 0.3, 64),
    (2, 8, 3, 0.6, 128),
    (2, 12, 1, 0.55, 192),
    (2, 12, 2, 0.7, 320),
    (2, 64, 2, 0.7, 64),
    (2, 64, 2, 0.85, 256),
    (3, 4, 3, 0.6, 64),
    (3, 8, 3, 0.8, 128),
    (3, 8, 5, 0.5, 64),
    (3, 12, 2, 0.6, 192),
    (3, 16, 3, 0.85, 256),
    # classes of more than 1024 edges: 2 or 3 edges per thread in the LDS path
    (2, 96, 2, 0.7, 64),
    (2, 68, 1, 0.6, 128),
    (3, 20, 3, 0.85, 64),
]


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("d,L,m,rho,R", LATTICE_CASES)
def test_lattice_parity(oracle, d, L, m, rho, R, path):
    g = ka.ka_graph_lattice(d, L)
    og = oracle.lattice(d, L)
    K = oracle.k_from_rho(og.N, rho)
    _check_case(oracle, g, og, m, K, 1234 + L, R, [1, 2, 4], path)


RRG_CASES = [
    # N, z, m, rho, R
    (64, 3, 1, 0.5, 64),
    (100, 4, 2, 0.6, 128),
    (512, 5, 3, 0.7, 64),
    (300, 6, 3, 0.8, 256),
    (300, 6, 0, 0.4, 64),
    (2000, 4, 2, 0.65, 192),
    # complete graphs K4 and K6: every pair of edges conflicts, so each class is one edge
    (4, 3, 1, 0.5, 64),
    (6, 5, 2, 0.5, 128),
]


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("N,z,m,rho,R", RRG_CASES)
def test_rrg_parity(oracle, N, z, m, rho, R, path):
    g = ka.ka_graph_rrg(N, z, 17)
    oadj, _ = oracle.rrg_adjacency(N, z, 17)
    og = oracle.graph_from_adjacency(oadj)
    K = oracle.k_from_rho(N, rho)
    _check_case(oracle, g, og, m, K, 99 + N, R, [1, 3, 5], path)


@pytest.mark.parametrize("N,z,m,rho,R", RRG_CASES)
def test_rrg_parity_one_launch_per_class(oracle, N, z, m, rho, R):
    """The same cases on the global path with every class in a launch of its own (these
    graphs' classes are all small, so by default a whole sweep is one merged launch)."""
    g = ka.ka_graph_rrg(N, z, 17)
    oadj, _ = oracle.rrg_adjacency(N, z, 17)
    og = oracle.graph_from_adjacency(oadj)
    K = oracle.k_from_rho(N, rho)
    _check_case(oracle, g, og, m, K, 99 + N, R, [1, 3, 5], 1, options=((ka.KA_OPT_TAIL, 0),))


def _tail_first(class_sizes, most=512):
    """First class of the trailing run of classes with at most `most` edges each, or the
    class count if that run holds fewer than two classes."""
    C = len(class_sizes)
    c = C
    while c > 0 and class_sizes[c - 1] <= most:
        c -= 1
    return c if C - c >= 2 else C


@pytest.mark.parametrize("N,z,m,rho,R,mixed", [
    (16384, 4, 2, 0.6, 64, True),
    (16384, 5, 3, 0.7, 192, True),
    (8192, 3, 1, 0.55, 128, True),
    (2000, 4, 2, 0.65, 192, False),
])
def test_tail_classes_one_launch(oracle, N, z, m, rho, R, mixed):
    """Greedy colourings end in a few classes of a few hundred edges or fewer; on the global
    path that trailing run is one launch with one workgroup per word plane.  Runs with and
    without the merge equal the oracle, and the launch counts show which ran."""
    g = ka.ka_graph_rrg(N, z, 23)
    adj, _, _, ec = ka.ka_graph_export(g)
    og = oracle.graph_from_adjacency(adj)
    sizes = np.bincount(ec, minlength=og.C)
    assert N * 8 * (2 if R % 128 == 0 else 1) <= 1 << 20    # small enough for the merge
    tail = _tail_first(sizes)
    if mixed:
        assert 0 < tail <= og.C - 2, sizes        # large classes, then a merged run
    else:
        assert tail == 0, sizes                    # every class small: one launch per sweep
    K = oracle.k_from_rho(N, rho)
    _say(f"tail classes: RRG N={N} z={z} R={R} classes={og.C} tail from {tail}")
    sims = []
    for opt in (1, 0):
        sim = ka.ka_init_k(g, m, K, 5, R)
        ka.ka_set_option(sim, ka.KA_OPT_PATH, 1)
        ka.ka_set_option(sim, ka.KA_OPT_TAIL, opt)
        sims.append(sim)
    orc = oracle.Sim(og, m, K, 5, range(R))
    for n in (1, 4):
        for sim in sims:
            ka.ka_sweep(sim, n)
        orc.sweep(n)
        for sim in sims:
            _state_equal(sim, orc)
            _observe_equal(sim, orc)
    assert [ka.ka_timing(sim)[0] for sim in sims] == [5 * (tail + 1), 5 * og.C]
    for sim in sims:
        sim.free()


LAYERED_CASES = [
    # d, L, M, m, rho, R
    (2, 8, 3, 2, 0.7, 64),
    (3, 4, 4, 3, 0.8, 128),
    (2, 6, 2, 1, 0.6, 64),      # L % 4 != 0: greedy classes
    (3, 8, 2, 3, 0.85, 256),
]


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("d,L,M,m,rho,R", LAYERED_CASES)
def test_layered_parity(oracle, d, L, M, m, rho, R, path):
    g = ka.ka_graph_layered(d, L, M, 5)
    og = oracle.layered(d, L, M, 5)
    K = oracle.k_from_rho(og.N, rho)
    _check_case(oracle, g, og, m, K, 71 + M, R, [1, 2, 3], path)


@pytest.mark.parametrize("path", [1, 2])
def test_degenerate_particle_numbers(oracle, path):
    g = ka.ka_graph_lattice(2, 8)
    og = oracle.lattice(2, 8)
    for K in (0, 1, og.N - 1, og.N):
        for m in (0, 2, 3):
            _check_case(oracle, g, og, m, K, 5, 64, [3], path)


def test_every_m_both_geometries(oracle):
    for d, L in [(2, 8), (3, 8)]:
        g = ka.ka_graph_lattice(d, L)
        og = oracle.lattice(d, L)
        for m in range(og.z):
            _check_case(oracle, g, og, m, oracle.k_from_rho(og.N, 0.6), 3 + m, 128, [2], 1)


@pytest.mark.parametrize("path", [1, 2])
def test_run_observation_grid(oracle, path):
    """ka_run records observations on the device; rows must equal the oracle's counts."""
    g = ka.ka_graph_lattice(2, 16)
    og = oracle.lattice(2, 16)
    K = oracle.k_from_rho(og.N, 0.7)
    _say(f"ka_run grid path={path}")
    sim = ka.ka_init_k(g, 2, K, 77, 128)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, path)
    times = [0, 0, 1, 2, 3, 5, 8, 8, 13, 21]
    dens, ov, pers = ka.ka_run(sim, times)
    orc = oracle.Sim(og, 2, K, 77, range(128))
    for q, t in enumerate(times):
        orc.sweep(t - orc.t)
        od, oo, op = orc.observe()
        assert np.array_equal(dens[q], od) and np.array_equal(ov[q], oo) and np.array_equal(pers[q], op), q
    assert sim.t == 21
    _state_equal(sim, orc)


def test_paths_agree_and_split_invariance(oracle):
    g = ka.ka_graph_lattice(3, 12)
    _say("paths agree 3D L=12")
    a = ka.ka_init(g, 3, 0.75, 8, 256)
    ka.ka_set_option(a, ka.KA_OPT_PATH, 1)
    ka.ka_sweep(a, 7)
    b = ka.ka_init(g, 3, 0.75, 8, 256)
    ka.ka_set_option(b, ka.KA_OPT_PATH, 2)
    ka.ka_sweep(b, 3)
    ka.ka_sweep(b, 4)
    sa, sb = ka.ka_get_state(a), ka.ka_get_state(b)
    for x, y in zip(sa, sb):
        assert np.array_equal(np.asarray(x), np.asarray(y))


@pytest.mark.parametrize("d,L,R", [(3, 12, 256), (2, 16, 192), (2, 16, 320)])
def test_plane_streams_identical(oracle, d, L, R):
    """Word planes on two streams of the sim's own (KA_OPT_PLANE_STREAMS), all planes in one
    launch (the default), and the timed mode with plane streams asked for (which keeps one
    stream) end in the same state; with plane streams every plane and class step is one
    launch.  A few replicas are also checked against the oracle."""
    g = ka.ka_graph_lattice(d, L)
    _say(f"plane streams d={d} L={L} R={R}")
    states, launches = [], []
    for opts in ([(ka.KA_OPT_PLANE_STREAMS, 1)], [], [(ka.KA_OPT_PLANE_STREAMS, 1), (ka.KA_OPT_TIMING, 3)]):
        s = ka.ka_init(g, d, 0.7, 12, R)
        ka.ka_set_option(s, ka.KA_OPT_PATH, 1)
        for o, v in opts:
            ka.ka_set_option(s, o, v)
        ka.ka_sweep(s, 3)
        ka.ka_run(s, [4, 6])
        states.append(ka.ka_get_state(s))
        launches.append(ka.ka_timing(s)[0])
        s.free()
    for other in states[1:]:
        for x, y in zip(states[0], other):
            assert np.array_equal(np.asarray(x), np.asarray(y))
    W = R // 64
    planes = W // 2 if W % 2 == 0 else W
    C = 4 * d
    assert launches == [6 * C * planes, 6 * C, 6 * C]
    og = oracle.lattice(d, L)
    orc = oracle.Sim(og, d, oracle.k_from_rho(og.N, 0.7), 12, [0, R - 1])
    orc.sweep(6)
    n = states[0][0]
    for q, b in enumerate([0, R - 1]):
        row = (n[b // 64] >> np.uint64(b % 64)) & np.uint64(1)
        assert np.array_equal(row.astype(np.uint8), orc.occ[q])


@pytest.mark.parametrize("d,L,R,group", [(3, 12, 256, 1), (2, 16, 192, 2), (3, 8, 320, 2), (2, 12, 128, 1)])
def test_plane_groups_match_oracle(oracle, d, L, R, group):
    """Word planes run group by group (each group through the whole call's sweeps, as large
    lattices do to keep a group's n and f in the Infinity Cache): the result equals the
    oracle's, with groups of one or two planes, a short last group, and the ordinary
    all-planes launch in between; the launch count shows the grouping."""
    g = ka.ka_graph_lattice(d, L)
    og = oracle.lattice(d, L)
    m = d + 1 if d == 3 else 2
    K = oracle.k_from_rho(og.N, 0.8)
    _say(f"plane groups: {d}D L={L} R={R} group={group}")
    sim = ka.ka_init_k(g, m, K, 21, R)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, 1)
    W = R // 64
    planes = W // 2 if W % 2 == 0 else W
    orc = oracle.Sim(og, m, K, 21, range(R))
    expected = 0
    for n, grp in ((3, group), (2, 0), (4, group)):
        ka.ka_set_option(sim, ka.KA_OPT_PLANE_GROUPS, grp)
        ka.ka_sweep(sim, n)
        orc.sweep(n)
        _state_equal(sim, orc)
        _observe_equal(sim, orc)
        expected += n * og.C * (-(-planes // grp) if grp else 1)
    assert ka.ka_timing(sim)[0] == expected
    for bad in (-2, planes + 1):
        with pytest.raises(ka.KaError) as err:
            ka.ka_set_option(sim, ka.KA_OPT_PLANE_GROUPS, bad)
        assert err.value.code == ka.KA_EINVAL
    sim.free()


@pytest.mark.parametrize("N,z,R,group", [(3000, 4, 256, 1), (2000, 5, 192, 2), (16384, 4, 320, 3)])
def test_plane_groups_graph_match_oracle(oracle, N, z, R, group):
    """The same grouping on random regular graphs, with the trailing tiny classes merged into
    one launch per group (the merged launch takes only its group's planes)."""
    g = ka.ka_graph_rrg(N, z, 29)
    adj, _, _, _ = ka.ka_graph_export(g)
    og = oracle.graph_from_adjacency(adj)
    K = oracle.k_from_rho(N, 0.6)
    _say(f"plane groups: RRG N={N} z={z} R={R} group={group}")
    sim = ka.ka_init_k(g, 2, K, 23, R)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, 1)
    orc = oracle.Sim(og, 2, K, 23, range(R))
    for n, grp in ((2, group), (1, 0), (3, group)):
        ka.ka_set_option(sim, ka.KA_OPT_PLANE_GROUPS, grp)
        ka.ka_sweep(sim, n)
        orc.sweep(n)
        _state_equal(sim, orc)
        _observe_equal(sim, orc)
    sim.free()


def test_set_state_resume(oracle):
    """Checkpoint/resume: a state put back with ka_set_state continues exactly."""
    g = ka.ka_graph_lattice(2, 12)
    og = oracle.lattice(2, 12)
    K = oracle.k_from_rho(og.N, 0.6)
    _say("set_state resume")
    orc = oracle.Sim(og, 2, K, 4, range(128))
    orc.sweep(5)
    sim = ka.ka_init_k(g, 2, K, 4, 128)
    ka.ka_set_state(sim, oracle.pack(orc.occ), oracle.pack(orc.occ0), oracle.pack(orc.moved), orc.t)
    ka.ka_sweep(sim, 6)
    orc.sweep(6)
    _state_equal(sim, orc)
    _observe_equal(sim, orc)


@pytest.mark.parametrize("tail", [1, 0])
@pytest.mark.parametrize("R", [64, 128])
def test_full_moved_ever_summary_cleared_by_set_state(oracle, R, tail):
    """General graphs keep a bit per vertex once its moved-ever words are all ones and then
    skip reading them.  After enough sweeps at m = z-1 (no constraint) every vertex is full;
    ka_set_state then puts back a state whose f has been cleared, and the run must mark moves
    again exactly as the oracle does from the same state (global path, one and two words per
    thread, with the trailing tiny classes merged into one launch or not).  The same run
    without the reset checks the summary's steady state."""
    N, z, m = 3000, 4, 3
    g = ka.ka_graph_rrg(N, z, 17)
    adj, _, _, _ = ka.ka_graph_export(g)
    og = oracle.graph_from_adjacency(adj)
    K = oracle.k_from_rho(N, 0.5)
    _say(f"moved-ever summary: RRG N={N} R={R} tail={tail}")
    sim = ka.ka_init_k(g, m, K, 8, R)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, 1)
    ka.ka_set_option(sim, ka.KA_OPT_TAIL, tail)
    orc = oracle.Sim(og, m, K, 8, range(R))
    ka.ka_sweep(sim, 60)
    orc.sweep(60)
    _state_equal(sim, orc)
    n, n0, f, t = ka.ka_get_state(sim)
    assert (f == np.uint64(0xFFFFFFFFFFFFFFFF)).mean() > 0.99     # the summary is in use
    ka.ka_sweep(sim, 3)                                           # full: f reads skipped
    orc.sweep(3)
    _state_equal(sim, orc)
    _observe_equal(sim, orc)
    n, n0, f, t = ka.ka_get_state(sim)
    zero = np.zeros_like(f)
    ka.ka_set_state(sim, n, n0, zero, t)
    orc.moved[:] = 0
    ka.ka_sweep(sim, 2)
    orc.sweep(2)
    _state_equal(sim, orc)
    _observe_equal(sim, orc)
    sim.free()


def test_replica_subset_independence(oracle):
    """Replica b's trajectory does not depend on how many replicas run beside it."""
    g = ka.ka_graph_lattice(2, 16)
    _say("replica subset")
    small = ka.ka_init(g, 2, 0.7, 3, 64)
    big = ka.ka_init(g, 2, 0.7, 3, 256)
    ka.ka_sweep(small, 9)
    ka.ka_sweep(big, 9)
    ns = ka.ka_get_state(small)[0]
    nb = ka.ka_get_state(big)[0]
    assert np.array_equal(ns[0], nb[0])


# ------------------------------------------------------------------------ four-point pair sums
PAIR_CASES = [
    # d, L, m, rho, R, sweeps, r2_max
    (2, 8, 2, 0.7, 64, 3, 32),        # full coverage: 2 * 4^2
    (2, 12, 1, 0.55, 128, 2, 9),
    (3, 4, 3, 0.6, 256, 4, 12),       # full coverage: 3 * 2^2
    (3, 8, 3, 0.8, 192, 2, 6),
]


@pytest.mark.parametrize("d,L,m,rho,R,sweeps,r2_max", PAIR_CASES)
def test_pair_sums_parity(oracle, d, L, m, rho, R, sweeps, r2_max):
    g = ka.ka_graph_lattice(d, L)
    og = oracle.lattice(d, L)
    K = oracle.k_from_rho(og.N, rho)
    _say(f"pair sums d={d} L={L} R={R} r2_max={r2_max}")
    sim = ka.ka_init_k(g, m, K, 13, R)
    ka.ka_sweep(sim, sweeps)
    S2, S11, cnt = ka.ka_observe_pairs(sim, r2_max)
    orc = oracle.Sim(og, m, K, 13, range(R))
    orc.sweep(sweeps)
    oS2, oS11, ocnt = oracle.pair_sums(orc.occ, orc.occ0, d, L, r2_max)
    assert np.array_equal(cnt, ocnt)
    assert np.array_equal(S2, oS2) and np.array_equal(S11, oS11)


def test_pair_sums_cover_chi4_gpu(oracle):
    """All displacements of 3D L=16 x 256 replicas: sum S2 = sum_b overlap_b^2, sum S11 =
    (sum_b overlap_b)^2, S2[0] = sum_b overlap_b, so the library's g4 (ka_g4) sums to the
    chi4 that the oracle's own formula gives for the oracle's overlaps of the same run, and
    the library's ka_derived equals the oracle's formula too."""
    g = ka.ka_graph_lattice(3, 16)
    _say("pair sums full coverage 3D L=16")
    sim = ka.ka_init(g, 3, 0.75, 5, 256)
    ka.ka_sweep(sim, 20)
    S2, S11, cnt = ka.ka_observe_pairs(sim, 3 * 8 * 8)
    _, dens, ov, pers = ka.ka_observe(sim)
    assert cnt.sum() == g.N
    assert S2.sum() == int((ov.astype(object) ** 2).sum())
    assert S11.sum() == int(ov.sum()) ** 2
    assert S2[0] == int(ov.sum())
    orc = oracle.Sim(oracle.lattice(3, 16), 3, sim.K, 5, range(256))
    orc.sweep(20)
    _, o_ov, o_pers = orc.observe()
    assert np.array_equal(ov, o_ov) and np.array_equal(pers, o_pers)
    oC, o_chi4, oP = oracle.derived(g.N, sim.K, o_ov, o_pers)
    g4 = ka.ka_g4(g.N, sim.K, 256, S2, S11)
    assert abs(g4.sum() - o_chi4) < 1e-9 * max(1.0, abs(o_chi4))
    C, chi4, P = ka.ka_derived(g.N, sim.K, ov, pers)
    assert abs(C[0] - oC) < 1e-12 and abs(chi4[0] - o_chi4) < 1e-9 * max(1.0, abs(o_chi4))
    assert abs(P[0] - oP) < 1e-12


GRAPH_PAIR_CASES = [
    # kind, N or (d, L, M), z, m, rho, R, sweeps, r2_max
    ("rrg", 300, 4, 2, 0.6, 64, 5, 0),
    ("rrg", 500, 3, 1, 0.5, 128, 4, 1),
    ("rrg", 1000, 5, 3, 0.7, 192, 3, 6),
    ("layered", (2, 8, 3), 4, 2, 0.65, 64, 6, 2),
    ("rrg", 20000, 4, 2, 0.75, 64, 2, 1),       # global path
]


@pytest.mark.parametrize("kind,size,z,m,rho,R,sweeps,r2_max", GRAPH_PAIR_CASES)
def test_pair_sums_graph_parity(oracle, kind, size, z, m, rho, R, sweeps, r2_max):
    """Graphs without a geometry use the distance 0 for i = j and 1 otherwise (Sec. 3.3):
    the library's shells equal the oracle's explicit pair loop."""
    if kind == "rrg":
        g = ka.ka_graph_rrg(size, z, 31)
        adj, _, _, _ = ka.ka_graph_export(g)
        og = oracle.graph_from_adjacency(adj)
    else:
        g = ka.ka_graph_layered(*size, 31)
        og = oracle.layered(*size, 31)       # classes projected from the lattice (L % 4 == 0)
    K = oracle.k_from_rho(og.N, rho)
    _say(f"graph pair sums {kind} {size} z={z} R={R} r2_max={r2_max}")
    sim = ka.ka_init_k(g, m, K, 17, R)
    ka.ka_sweep(sim, sweeps)
    S2, S11, cnt = ka.ka_observe_pairs(sim, r2_max)
    orc = oracle.Sim(og, m, K, 17, range(R))
    orc.sweep(sweeps)
    oS2, oS11, ocnt = oracle.pair_sums_graph(orc.occ, orc.occ0, r2_max)
    assert np.array_equal(cnt, ocnt)
    assert np.array_equal(S2, oS2) and np.array_equal(S11, oS11)


def test_pair_sums_full_workload_properties():
    """3D L=128 x 256 replicas (the benchmark workload) out to r = 6 (the paper's range):
    at t = 0, S2[0] equals the summed overlap K*R, S11[0] = sum_i popcount(n0_i)^2 >= S2[0];
    after sweeps S2[0] still equals the summed overlap."""
    g = ka.ka_graph_lattice(3, 128)
    _say("pair sums 3D L=128 x 256")
    sim = ka.ka_init(g, 3, 0.85, 1, 256)
    S2, S11, cnt = ka.ka_observe_pairs(sim, 36)
    assert S2[0] == sim.K * 256 and S11[0] >= S2[0]
    assert cnt[1] == 6 and cnt[2] == 12 and cnt[36] > 0
    ka.ka_sweep(sim, 3)
    S2, S11, cnt = ka.ka_observe_pairs(sim, 36)
    _, dens, ov, pers = ka.ka_observe(sim)
    assert S2[0] == int(ov.sum())
    assert (S2 >= 0).all() and (S11 >= 0).all()


def test_graph_schedule_reused_and_outlives_graph(oracle):
    """The device schedule of a general graph is built on the first ka_init and reused by
    later ones; a sim keeps working after its graph is freed.  Two sims of one graph (the
    second built from the cached schedule, the graph then freed under both) equal the
    oracle bit for bit."""
    N, z, m, R, seed = 3000, 4, 2, 128, 9
    g = ka.ka_graph_rrg(N, z, seed)
    adj, _, _, _ = ka.ka_graph_export(g)
    og = oracle.graph_from_adjacency(adj)
    K = ka.ka_particles(N, 0.6)
    _say(f"schedule reuse: RRG N={N} z={z} K={K} R={R}")
    sims = [ka.ka_init_k(g, m, K, s, R) for s in (3, 4)]
    ka.load().ka_graph_free(g.handle)
    g._h = None
    for s in sims:
        s.graph = None
    orcs = [oracle.Sim(og, m, K, s, range(R)) for s in (3, 4)]
    for sim, orc in zip(sims, orcs):
        ka.ka_sweep(sim, 7)
        orc.sweep(7)
        _state_equal(sim, orc)
        _observe_equal(sim, orc)
        sim.free()


SHARED_CASES = [
    # kind, size, z-or-d, m, rho, R
    ("lattice", 12, 2, 2, 0.6, 128),
    ("lattice", 8, 3, 3, 0.8, 64),
    ("lattice", 64, 2, 2, 0.7, 256),
    ("rrg", 300, 4, 2, 0.6, 192),
    ("rrg", 200, 6, 5, 0.5, 64),
]


@pytest.mark.parametrize("path", [1, 2])
@pytest.mark.parametrize("kind,size,zd,m,rho,R", SHARED_CASES)
def test_shared_noise_parity(oracle, kind, size, zd, m, rho, R, path):
    """KA_OPT_NOISE = 1 (one acceptance bit per edge for all replicas) equals the oracle's
    shared-noise run bit for bit, on both kernel paths."""
    if kind == "lattice":
        g, og = ka.ka_graph_lattice(zd, size), oracle.lattice(zd, size)
    else:
        g = ka.ka_graph_rrg(size, zd, 5)
        og = oracle.graph_from_adjacency(oracle.rrg_adjacency(size, zd, 5)[0])
    K = oracle.k_from_rho(og.N, rho)
    _say(f"shared noise: {kind} {size} m={m} R={R} path={path}")
    sim = ka.ka_init_k(g, m, K, 77, R)
    try:
        ka.ka_set_option(sim, ka.KA_OPT_PATH, path)
    except ka.KaError:
        sim.free()
        pytest.skip("this instance does not fit the LDS-resident path on this device")
    ka.ka_set_option(sim, ka.KA_OPT_NOISE, 1)
    orc = oracle.Sim(og, m, K, 77, range(R), shared=True)
    for n in (1, 3, 5):
        ka.ka_sweep(sim, n)
        orc.sweep(n)
        _state_equal(sim, orc)
        _observe_equal(sim, orc)
    sim.free()


def test_shared_noise_couples_equal_replicas_on_gpu():
    """With shared noise, replicas set to the same state stay equal (checked over all word
    positions of a 3-word state), and switching back to independent noise separates them."""
    g = ka.ka_graph_lattice(3, 12)
    sim = ka.ka_init(g, 3, 0.8, 9, 192)
    n, n0, f, _ = ka.ka_get_state(sim)
    first = (n[0] & np.uint64(1)).astype(bool)
    word = np.where(first, np.uint64(0xFFFFFFFFFFFFFFFF), np.uint64(0))
    same = np.repeat(word[None, :], 3, axis=0)
    ka.ka_set_state(sim, same, same, np.zeros_like(same), 0)
    ka.ka_set_option(sim, ka.KA_OPT_NOISE, 1)
    ka.ka_sweep(sim, 20)
    n, _, f, _ = ka.ka_get_state(sim)
    for arr in (n, f):
        assert ((arr == np.uint64(0)) | (arr == np.uint64(0xFFFFFFFFFFFFFFFF))).all()
        assert (arr == arr[0][None, :]).all()
    assert not np.array_equal(n[0], word)
    ka.ka_set_option(sim, ka.KA_OPT_NOISE, 0)
    ka.ka_sweep(sim, 5)
    n, _, _, _ = ka.ka_get_state(sim)
    assert not ((n == np.uint64(0)) | (n == np.uint64(0xFFFFFFFFFFFFFFFF))).all()
    sim.free()


def test_valu_probe():
    """The calibration probe runs, reports positive rates, and rejects bad arguments."""
    _say("valu probe")
    for kind in (0, 1):
        ips, lops = ka.ka_probe_valu(kind, iters=200, blocks=512)
        assert ips > 0 and lops == pytest.approx(64 * ips)
    with pytest.raises(ka.KaError):
        ka.ka_probe_valu(2)
    with pytest.raises(ka.KaError):
        ka.ka_probe_valu(0, iters=0)


@pytest.mark.parametrize("R", [64, 256])
def test_lds_chunk_boundaries(oracle, R):
    """The LDS-resident lattice sweep runs in chunks of sweeps whose acceptance words are
    generated ahead (128 sweeps per chunk for one 2D L=64 plane, 32 for two), counted from
    the time a call starts: sweeps and observations that start, end or sit exactly at chunk
    boundaries match the oracle."""
    g = ka.ka_graph_lattice(2, 64)
    og = oracle.lattice(2, 64)
    K = oracle.k_from_rho(og.N, 0.7)
    chunk = 128 if R == 64 else 32
    _say(f"LDS chunk boundaries R={R}")
    sim = ka.ka_init_k(g, 2, K, 3, R)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, 2)
    replicas = [0, R - 1]
    orc = oracle.Sim(og, 2, K, 3, replicas)
    ka.ka_sweep(sim, chunk - 1)
    orc.sweep(chunk - 1)
    # the run starts at t0 = chunk - 1, so its chunks end at t0 + chunk, t0 + 2 chunk, ...
    times = [chunk, chunk, chunk + 1, 2 * chunk - 1, 2 * chunk, 3 * chunk - 1, 3 * chunk, 4 * chunk]
    dens, ov, pers = ka.ka_run(sim, times)
    for q, t in enumerate(times):
        orc.sweep(t - orc.t)
        od, oo, op = orc.observe()
        for k, b in enumerate(replicas):
            assert (dens[q, b], ov[q, b], pers[q, b]) == (od[k], oo[k], op[k]), (t, b)
    ka.ka_sweep(sim, chunk + 3)
    orc.sweep(chunk + 3)
    n, n0, f, t = ka.ka_get_state(sim)
    assert t == orc.t
    for k, b in enumerate(replicas):
        assert np.array_equal(((n[b // 64] >> np.uint64(b % 64)) & np.uint64(1)).astype(np.uint8), orc.occ[k])
        assert np.array_equal(((f[b // 64] >> np.uint64(b % 64)) & np.uint64(1)).astype(np.uint8), orc.moved[k])
    sim.free()


def test_lds_observations_snapshot_and_in_place(oracle):
    """The LDS-resident path takes observations as snapshots counted on the whole device when
    they fit its snapshot budget (4 MiB: 64 rows of 64 KiB for 2D L=64 x 64), and counts them
    in place on its one workgroup otherwise.  Both give the oracle's counts."""
    g = ka.ka_graph_lattice(2, 64)
    og = oracle.lattice(2, 64)
    K = oracle.k_from_rho(og.N, 0.7)
    replicas = list(range(64))
    for times in (list(range(0, 60)) + [70, 90], list(range(0, 101))):
        _say(f"LDS observations: {len(times)} in one chunk")
        sim = ka.ka_init_k(g, 2, K, 8, 64)
        ka.ka_set_option(sim, ka.KA_OPT_PATH, 2)
        dens, ov, pers = ka.ka_run(sim, times)
        orc = oracle.Sim(og, 2, K, 8, replicas)
        for q, t in enumerate(times):
            orc.sweep(t - orc.t)
            od, oo, op = orc.observe()
            assert np.array_equal(dens[q], od) and np.array_equal(ov[q], oo) and np.array_equal(pers[q], op), t
        _state_equal(sim, orc)
        sim.free()


@pytest.mark.parametrize("z,R", [(4, 64), (3, 128)])
def test_lds_graph_chunk_boundaries(oracle, z, R):
    """The LDS-resident graph sweep with acceptance words generated ahead per chunk of sweeps
    (8 MiB of words: 128 sweeps for N=4096, z=4 x 64 replicas; 85 for z=3 x 128): sweeps and
    observations that start, end or sit on chunk boundaries match the oracle."""
    N = 4096
    g = ka.ka_graph_rrg(N, z, 23)
    oadj, _ = oracle.rrg_adjacency(N, z, 23)
    og = oracle.graph_from_adjacency(oadj)
    K = oracle.k_from_rho(N, 0.6)
    chunk = min(20000, (8 << 20) // (g.E * (R // 64) * 8))
    _say(f"LDS graph chunk boundaries z={z} R={R} chunk={chunk}")
    sim = ka.ka_init_k(g, 2, K, 5, R)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, 2)
    replicas = [0, R - 1]
    orc = oracle.Sim(og, 2, K, 5, replicas)
    ka.ka_sweep(sim, chunk - 1)
    orc.sweep(chunk - 1)
    times = [chunk, chunk + 1, 2 * chunk - 1, 2 * chunk, 2 * chunk + 3]
    dens, ov, pers = ka.ka_run(sim, times)
    for q, t in enumerate(times):
        orc.sweep(t - orc.t)
        od, oo, op = orc.observe()
        for k, b in enumerate(replicas):
            assert (dens[q, b], ov[q, b], pers[q, b]) == (od[k], oo[k], op[k]), (t, b)
    ka.ka_sweep(sim, chunk + 2)
    orc.sweep(chunk + 2)
    n, n0, f, t = ka.ka_get_state(sim)
    assert t == orc.t
    for k, b in enumerate(replicas):
        assert np.array_equal(((n[b // 64] >> np.uint64(b % 64)) & np.uint64(1)).astype(np.uint8), orc.occ[k])
        assert np.array_equal(((f[b // 64] >> np.uint64(b % 64)) & np.uint64(1)).astype(np.uint8), orc.moved[k])
    sim.free()


@pytest.mark.parametrize("z,R", [(3, 64), (4, 64), (3, 192), (4, 192)])
def test_lds_graph_two_edges_per_thread(oracle, z, R):
    """Random regular graphs of 8192 vertices fit the LDS-resident sweep with classes of more
    than 1024 edges, so a thread takes a second edge slot of every large class.  With one and
    with three word planes (one workgroup each), across chunks of acceptance words generated
    ahead, every replica matches the oracle at every observation and in the final state."""
    N = 8192
    g = ka.ka_graph_rrg(N, z, 29)
    oadj, _ = oracle.rrg_adjacency(N, z, 29)
    og = oracle.graph_from_adjacency(oadj)
    _, _, _, ec = ka.ka_graph_export(g)
    assert np.bincount(ec).max() > 1024
    K = oracle.k_from_rho(N, 0.6)
    chunk = min(20000, (8 << 20) // (g.E * (R // 64) * 8))
    _say(f"LDS graph two slots z={z} R={R} chunk={chunk}")
    sim = ka.ka_init_k(g, 2, K, 6, R)
    ka.ka_set_option(sim, ka.KA_OPT_PATH, 2)
    orc = oracle.Sim(og, 2, K, 6, range(R))
    times = [1, chunk - 1, chunk, chunk + 1, 2 * chunk, 2 * chunk + 5]
    dens, ov, pers = ka.ka_run(sim, times)
    for q, t in enumerate(times):
        orc.sweep(t - orc.t)
        od, oo, op = orc.observe()
        assert np.array_equal(dens[q], od) and np.array_equal(ov[q], oo) and np.array_equal(pers[q], op), t
    _state_equal(sim, orc)
    sim.free()
