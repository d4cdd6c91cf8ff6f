"""GPU parity at the full workload sizes, in the launch configuration the benchmark times.

- 2D square lattice L=64, z=4, m=2, rho=0.70 (K=2867), 64 replicas, seed 1, 1000 sweeps,
  observations every 10 sweeps: every replica, every observation and the final state are
  compared with the oracle (the whole run is small enough for it).
- 3D cubic lattice L=128, z=6, m=3, 256 replicas (4 words per site), seed 1, observation on
  the 38-point log grid: replicas {0, 63, 64, 255} (first and last bit of the first and last
  word) are compared with the oracle bit for bit at every grid point up to 31 sweeps; the run
  then goes on to 10^4 sweeps and properties that hold at any size are checked on every
  replica.
- Random regular graph N=2^20, z=4, m=2, graph seed 1, 64 replicas: the library's graph
  and classes equal the oracle's; replicas {0, 63} are compared at every grid point up to 31
  sweeps at rho = 0.50 and 0.75; invariants after 10^4 sweeps on every replica.
"""
import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _replica_bits(words, b):
    return ((words[b >> 6] >> np.uint64(b & 63)) & np.uint64(1)).astype(np.uint8)


def _check_invariants(K, dens, ov, pers):
    assert (dens == K).all(), "particle number not conserved"
    assert (ov <= K).all() and (pers <= ov).all()
    assert (np.diff(pers, axis=0) <= 0).all(), "persistence increased"
    assert (ov[0] == K).all() and (pers[0] == K).all()


def test_square64_full_run(oracle):
    g = ka.ka_graph_lattice(2, 64)
    og = oracle.lattice(2, 64)
    K = oracle.k_from_rho(og.N, 0.70)
    assert K == 2867
    times = list(range(0, 1001, 10))
    _say("square64 full: 64 replicas x 1000 sweeps, observations every 10")
    sim = ka.ka_init(g, 2, 0.70, 1, 64)
    dens, ov, pers = ka.ka_run(sim, times)
    n, n0, f, t = ka.ka_get_state(sim)
    orc = oracle.Sim(og, 2, K, 1, range(64))
    for q, tt in enumerate(times):
        orc.sweep(tt - orc.t)
        od, oo, op = orc.observe()
        assert np.array_equal(dens[q], od) and np.array_equal(ov[q], oo) and np.array_equal(pers[q], op), tt
    assert t == 1000
    assert np.array_equal(n, oracle.pack(orc.occ))
    assert np.array_equal(n0, oracle.pack(orc.occ0))
    assert np.array_equal(f, oracle.pack(orc.moved))


@pytest.mark.parametrize("rho", [0.80, 0.85, 0.88])
def test_cubic128_sampled_replicas(oracle, rho):
    g = ka.ka_graph_lattice(3, 128)
    og = oracle.lattice(3, 128)
    K = oracle.k_from_rho(og.N, rho)
    grid = ka.log_time_grid(10_000)
    head = [t for t in grid if t <= 31]
    sample = [0, 63, 64, 255]
    _say(f"cubic128 rho={rho}: head {head}, sampled replicas {sample}")
    sim = ka.ka_init(g, 3, rho, 1, 256)
    assert ka.ka_sim_path(sim) == 1
    dens, ov, pers = ka.ka_run(sim, head)
    n, n0, f, t = ka.ka_get_state(sim)
    orc = oracle.Sim(og, 3, K, 1, sample)
    for q, tt in enumerate(head):
        orc.sweep(tt - orc.t)
        od, oo, op = orc.observe()
        for k, b in enumerate(sample):
            assert (dens[q, b], ov[q, b], pers[q, b]) == (od[k], oo[k], op[k]), (tt, b)
    for k, b in enumerate(sample):
        assert np.array_equal(_replica_bits(n, b), orc.occ[k]), b
        assert np.array_equal(_replica_bits(n0, b), orc.occ0[k]), b
        assert np.array_equal(_replica_bits(f, b), orc.moved[k]), b
    _say(f"cubic128 rho={rho}: continuing to 10^4 sweeps")
    rest = [t for t in grid if t > 31]
    d2, o2, p2 = ka.ka_run(sim, rest)
    _check_invariants(K, np.vstack([dens, d2]), np.vstack([ov, o2]), np.vstack([pers, p2]))
    assert sim.t == 10_000


def test_rrg20_graph_and_sampled_replicas(oracle):
    N, z = 1 << 20, 4
    _say("rrg N=2^20: graph build (library and oracle)")
    g = ka.ka_graph_rrg(N, z, 1)
    oadj, _ = oracle.rrg_adjacency(N, z, 1)
    adj, eu, ev, ec = ka.ka_graph_export(g)
    assert np.array_equal(adj, oadj)
    og = oracle.graph_from_adjacency(oadj)
    assert np.array_equal(eu, og.eu) and np.array_equal(ev, og.ev) and np.array_equal(ec, og.ecls)
    for rho in (0.50, 0.75):
        K = oracle.k_from_rho(N, rho)
        head = [t for t in ka.log_time_grid(10_000) if t <= 31]
        _say(f"rrg N=2^20 rho={rho}: {head[-1]} sweeps, replicas 0 and 63")
        sim = ka.ka_init(g, 2, rho, 1, 64)
        assert ka.ka_sim_path(sim) == 1
        dens, ov, pers = ka.ka_run(sim, head)
        n, n0, f, t = ka.ka_get_state(sim)
        orc = oracle.Sim(og, 2, K, 1, [0, 63])
        for q, tt in enumerate(head):
            orc.sweep(tt - orc.t)
            od, oo, op = orc.observe()
            for k, b in enumerate([0, 63]):
                assert (dens[q, b], ov[q, b], pers[q, b]) == (od[k], oo[k], op[k]), (tt, b)
        for k, b in enumerate([0, 63]):
            assert np.array_equal(_replica_bits(n, b), orc.occ[k])
            assert np.array_equal(_replica_bits(f, b), orc.moved[k])
        grid = [t for t in ka.log_time_grid(10_000) if t > 31]
        d2, o2, p2 = ka.ka_run(sim, grid)
        _check_invariants(K, np.vstack([dens, d2]), np.vstack([ov, o2]), np.vstack([pers, p2]))
        sim.free()


@pytest.mark.parametrize("R,groups", [(256, 4), (128, 2), (64, 1)])
def test_cubic256_tiled_order_sampled_replicas(oracle, R, groups):
    """3D L=256 (Q = 64): the class pass visits chunk rows in tiles along p1 (a permutation
    of the edges of a class, which commute), and with more than one 64-replica word the n and
    f of all words exceed the 256 MiB Infinity Cache, so the words run one at a time (one
    word per plane, one launch per word and class step).  Replicas 0, 64 (when present) and
    R-1 match the oracle bit for bit after 2 sweeps."""
    g = ka.ka_graph_lattice(3, 256)
    og = oracle.lattice(3, 256)
    K = oracle.k_from_rho(og.N, 0.85)
    reps = sorted({0, min(64, R - 1), R - 1})
    _say(f"cubic256 R={R}: 2 sweeps, replicas {reps}")
    sim = ka.ka_init(g, 3, 0.85, 7, R)
    assert ka.ka_sim_path(sim) == 1
    dens, ov, pers = ka.ka_run(sim, [1, 2])
    assert ka.ka_timing(sim)[0] == 2 * 12 * groups     # one launch per word group and class
    n, n0, f, t = ka.ka_get_state(sim)
    sim.free()
    orc = oracle.Sim(og, 3, K, 7, reps)
    for q, tt in enumerate([1, 2]):
        orc.sweep(tt - orc.t)
        od, oo, op = orc.observe()
        for k, b in enumerate(reps):
            assert (dens[q, b], ov[q, b], pers[q, b]) == (od[k], oo[k], op[k]), (tt, b)
    for k, b in enumerate(reps):
        assert np.array_equal(_replica_bits(n, b), orc.occ[k]), b
        assert np.array_equal(_replica_bits(f, b), orc.moved[k]), b
