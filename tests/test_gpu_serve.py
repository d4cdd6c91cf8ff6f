"""Serving with continuous batching: jobs submitted while others run are admitted as slots
and device memory free up, share the batch's step kernels, and each job's observations and
final state are bit-identical to running it alone; four of them (2D, 3D with four words per
site, a random regular graph, and one admitted while others run) are also compared with the
oracle at every observation and in the final state."""
import random
import time

import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


JOBS = [
    # graph key, m, rho, R, seed, sweeps, obs
    (("lat", 2, 8), 2, 0.6, 64, 1, 12, [0, 3, 12]),
    (("lat", 2, 16), 1, 0.5, 128, 2, 20, None),
    (("lat", 3, 8), 3, 0.8, 256, 3, 9, [0, 1, 2, 5, 9]),
    (("rrg", 300, 4), 2, 0.65, 64, 4, 15, [7, 15]),
    (("rrg", 64, 3), 1, 0.5, 192, 5, 30, [0, 30]),
    (("lat", 2, 64), 2, 0.7, 64, 6, 25, [0, 5, 10, 15, 20, 25]),
    (("rrg", 500, 5), 3, 0.7, 128, 7, 8, None),
    (("lat", 3, 12), 2, 0.6, 64, 8, 6, [6]),
    (("rrg", 200, 6), 3, 0.8, 64, 9, 11, [0, 11]),
    (("lat", 2, 12), 3, 0.85, 320, 10, 4, [0, 2, 4]),
    (("lat", 2, 8), 0, 0.4, 64, 11, 0, None),
    (("rrg", 1000, 4), 2, 0.6, 64, 12, 18, [9, 18]),
]


@pytest.fixture(scope="module")
def graphs():
    out = {}
    for j in JOBS:
        key = j[0]
        if key in out:
            continue
        out[key] = ka.ka_graph_lattice(key[1], key[2]) if key[0] == "lat" else ka.ka_graph_rrg(key[1], key[2], 40 + key[1])
    return out


def _solo(g, m, rho, R, seed, sweeps, obs):
    s = ka.ka_init(g, m, rho, seed, R)
    times = obs if obs is not None else [sweeps]
    dens, ov, pers = ka.ka_run(s, times)
    if s.t < sweeps:
        ka.ka_sweep(s, sweeps - s.t)
    state = ka.ka_get_state(s)
    s.free()
    return (dens, ov, pers), state


def _run_server(graphs, budget, max_active, jitter):
    sv = ka.ka_server_create(budget, max_active)
    rng = random.Random(3)
    ids = []
    for (key, m, rho, R, seed, sweeps, obs) in JOBS:
        ids.append(ka.ka_server_submit(sv, graphs[key], m, rho, seed, R, sweeps, obs_times=obs, keep_sim=True))
        if jitter:
            time.sleep(rng.uniform(0.0, 0.004))
    ka.ka_server_wait_idle(sv)
    out = []
    for jid in ids:
        res = ka.ka_server_result(sv, jid)
        sim = ka.ka_server_take_sim(sv, jid)
        out.append((res, ka.ka_get_state(sim)))
        sim.free()
    stats = ka.ka_server_stats(sv)
    done = set(ka.ka_server_poll(sv))
    sv.free()
    assert done == set(ids)
    return out, stats


# Served jobs also compared with the oracle directly: a 2D lattice, a 3D lattice with four
# words per site, a random regular graph, and the last job, which with 3 slots is admitted
# only after earlier jobs complete, while others still run.
ORACLE_JOBS = (0, 2, 3, 11)


def _oracle_graph(oracle, graphs, key):
    if key[0] == "lat":
        return oracle.lattice(key[1], key[2])
    adj, _ = oracle.rrg_adjacency(key[1], key[2], 40 + key[1])
    exported, _, _, _ = ka.ka_graph_export(graphs[key])
    assert np.array_equal(adj, exported)
    return oracle.graph_from_adjacency(adj)


def _oracle_equal(oracle, graphs, job, res, state):
    key, m, rho, R, seed, sweeps, obs = job
    og = _oracle_graph(oracle, graphs, key)
    orc = oracle.Sim(og, m, oracle.k_from_rho(og.N, rho), seed, range(R))
    for q, t in enumerate(obs if obs is not None else [sweeps]):
        orc.sweep(t - orc.t)
        d, o, p = orc.observe()
        assert np.array_equal(res["density"][q], d), t
        assert np.array_equal(res["overlap"][q], o), t
        assert np.array_equal(res["persistence"][q], p), t
    orc.sweep(sweeps - orc.t)
    n, n0, f, t = state
    assert t == sweeps
    assert np.array_equal(n, oracle.pack(orc.occ))
    assert np.array_equal(n0, oracle.pack(orc.occ0))
    assert np.array_equal(f, oracle.pack(orc.moved))


@pytest.mark.parametrize("budget,max_active,jitter", [(1 << 34, 64, True), (1 << 34, 3, False)])
def test_served_jobs_equal_solo(oracle, graphs, budget, max_active, jitter):
    _say(f"serve budget={budget} max_active={max_active}")
    served, stats = _run_server(graphs, budget, max_active, jitter)
    assert stats["jobs_done"] == len(JOBS)
    assert stats["peak_active"] <= max_active
    for k, ((key, m, rho, R, seed, sweeps, obs), (res, state)) in enumerate(zip(JOBS, served)):
        (dens, ov, pers), solo_state = _solo(graphs[key], m, rho, R, seed, sweeps, obs)
        assert np.array_equal(res["density"], dens), k
        assert np.array_equal(res["overlap"], ov), k
        assert np.array_equal(res["persistence"], pers), k
        for a, b in zip(state, solo_state):
            assert np.array_equal(np.asarray(a), np.asarray(b)), k
        assert res["latency_s"] >= res["wait_s"] >= 0.0
    if max_active == 3:
        assert served[ORACLE_JOBS[-1]][0]["wait_s"] > 0.0    # admitted while others ran
    for k in ORACLE_JOBS:
        _say(f"serve: job {k} against the oracle")
        _oracle_equal(oracle, graphs, JOBS[k], *served[k])


def test_admission_by_footprint(graphs):
    """A budget that holds only the largest job alone still runs every job, within it."""
    big = max(ka.ka_footprint(graphs[j[0]], j[3]) for j in JOBS)
    budget = int(big * 1.05) + (1 << 20)
    _say("serve: budget for the largest job")
    served, stats = _run_server(graphs, budget, 64, False)
    assert stats["peak_bytes"] <= budget
    for k, ((key, m, rho, R, seed, sweeps, obs), (res, state)) in enumerate(zip(JOBS, served)):
        (dens, ov, pers), solo_state = _solo(graphs[key], m, rho, R, seed, sweeps, obs)
        assert np.array_equal(res["overlap"], ov) and np.array_equal(res["persistence"], pers), k


def test_server_rejects_oversized_job(graphs):
    sv = ka.ka_server_create(1 << 12, 4)
    with pytest.raises(ka.KaError) as e:
        ka.ka_server_submit(sv, graphs[("lat", 2, 64)], 2, 0.7, 1, 64, 10)
    assert e.value.code == ka.KA_EINVAL
    sv.free()


def test_release_and_taken_sim_outlives_server(graphs):
    """ka_server_release forgets a completed job (results and untaken kept sim); a taken
    sim moves off the server's own stream, so it keeps running after the server is freed and
    still equals the solo run."""
    g = graphs[("lat", 2, 16)]
    m, rho, R, sweeps = 1, 0.5, 128, 10
    _say("serve: release and a taken sim after ka_server_free")
    sv = ka.ka_server_create(1 << 34, 8)
    a = ka.ka_server_submit(sv, g, m, rho, 21, R, sweeps, obs_times=[0, sweeps], keep_sim=True)
    b = ka.ka_server_submit(sv, g, m, rho, 22, R, sweeps, keep_sim=True)
    c = ka.ka_server_submit(sv, g, m, rho, 23, R, sweeps)
    ka.ka_server_wait_idle(sv)
    res_a = ka.ka_server_result(sv, a)
    sim_a = ka.ka_server_take_sim(sv, a)
    ka.ka_server_release(sv, b)            # kept sim never taken: freed here
    ka.ka_server_release(sv, c)
    for jid in (b, c):
        with pytest.raises(ka.KaError) as e:
            ka.ka_server_result(sv, jid)
        assert e.value.code == ka.KA_ESTATE
    with pytest.raises(ka.KaError):
        ka.ka_server_release(sv, c)
    assert set(ka.ka_server_poll(sv)) == {a}
    sv.free()
    ka.ka_sweep(sim_a, 5)
    _, dens, ov, pers = ka.ka_observe(sim_a)
    state = ka.ka_get_state(sim_a)
    sim_a.free()
    (d0, o0, p0), _ = _solo(g, m, rho, R, 21, sweeps, [0, sweeps])
    assert np.array_equal(res_a["overlap"], o0) and np.array_equal(res_a["persistence"], p0)
    (d1, o1, p1), solo_state = _solo(g, m, rho, R, 21, sweeps + 5, [sweeps + 5])
    assert np.array_equal(ov, o1[0]) and np.array_equal(pers, p1[0]) and np.array_equal(dens, d1[0])
    for x, y in zip(state, solo_state):
        assert np.array_equal(np.asarray(x), np.asarray(y))


def test_take_and_release_while_others_run(graphs):
    """Completed jobs are taken (and swept further) or released from the caller's thread while
    the worker keeps running later jobs; every taken sim equals its solo run."""
    _say("serve: take / release while running")
    sv = ka.ka_server_create(1 << 34, 3)
    ids = {}
    done, taken = 0, {}
    try:
        for k, (key, m, rho, R, seed, sweeps, obs) in enumerate(JOBS):
            ids[ka.ka_server_submit(sv, graphs[key], m, rho, seed, R, sweeps, obs_times=obs,
                                    keep_sim=True)] = k
        deadline = time.time() + 120
        while done < len(ids):
            assert time.time() < deadline, "jobs did not complete"
            for jid in ka.ka_server_poll(sv):
                k = ids[jid]
                done += 1
                if k % 2 == 0:
                    sim = ka.ka_server_take_sim(sv, jid)
                    ka.ka_sweep(sim, 2)
                    taken[k] = ka.ka_get_state(sim)
                    sim.free()
                ka.ka_server_release(sv, jid)
            time.sleep(0.001)
    finally:
        sv.free()
    for k, state in taken.items():
        key, m, rho, R, seed, sweeps, obs = JOBS[k]
        _, solo_state = _solo(graphs[key], m, rho, R, seed, sweeps + 2, None)
        for a, b in zip(state, solo_state):
            assert np.array_equal(np.asarray(a), np.asarray(b)), k


SOLO_JOBS = [
    # 3D L=128 x 64 replicas: n and f take 32 MiB, so the server's batch runs these two one at
    # a time through their own passes (the default KA_BOPT_SOLO_BYTES) next to the small jobs
    (("lat", 3, 128), 3, 0.85, 64, 21, 6, [0, 2, 6]),
    (("lat", 2, 16), 1, 0.5, 128, 22, 20, [5, 20]),
    (("lat", 3, 128), 3, 0.80, 64, 23, 4, [1, 4]),
    (("rrg", 300, 4), 2, 0.65, 64, 24, 15, [7, 15]),
]


def test_served_solo_jobs_equal_solo():
    """Jobs large enough to fill the device alone are solo members of the server's batch:
    each job's observations and final state still equal its run alone."""
    _say("serve: jobs run one at a time inside the server's batch")
    graphs = {}
    for key, *_ in SOLO_JOBS:
        if key not in graphs:
            graphs[key] = ka.ka_graph_lattice(key[1], key[2]) if key[0] == "lat" else ka.ka_graph_rrg(key[1], key[2], 40 + key[1])
    sv = ka.ka_server_create(1 << 34, 8)
    ids = [ka.ka_server_submit(sv, graphs[key], m, rho, seed, R, sweeps, obs_times=obs, keep_sim=True)
           for (key, m, rho, R, seed, sweeps, obs) in SOLO_JOBS]
    ka.ka_server_wait_idle(sv)
    for jid, (key, m, rho, R, seed, sweeps, obs) in zip(ids, SOLO_JOBS):
        res = ka.ka_server_result(sv, jid)
        sim = ka.ka_server_take_sim(sv, jid)
        state = ka.ka_get_state(sim)
        sim.free()
        (dens, ov, pers), ref = _solo(graphs[key], m, rho, R, seed, sweeps, obs)
        assert np.array_equal(res["density"], dens) and np.array_equal(res["overlap"], ov), key
        assert np.array_equal(res["persistence"], pers), key
        for x, y in zip(state, ref):
            assert np.array_equal(np.asarray(x), np.asarray(y)), key
    sv.free()
