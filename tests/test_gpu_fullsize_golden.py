"""GPU parity for the full 10^4 sweeps of the 3D L=128 and random-regular-graph workloads,
against stored oracle values (tests/golden/fullsize_*.json, written on the CPU by
oracle/make_fullsize_golden.py, which calls only the oracle).

- 3D cubic lattice L=128, z=6, m=3, 256 replicas, seed 1, in the launch configuration the
  benchmark times (global class passes): replicas {0, 63, 64, 255} at rho = 0.80, 0.85, 0.88,
  every count at all 38 log-grid points to 10^4 sweeps and the final n, n(0), f rows; all 256
  replicas at rho = 0.85 for the first 100 sweeps (every count at the 18 grid points, and the
  whole state at t = 100).
- Random regular graph N=2^20, z=4, m=2, graph seed 1, 64 replicas: replicas {0, 63} at
  rho = 0.50 and 0.75 to 10^4 sweeps; all 64 replicas at both densities for 100 sweeps.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _load(name):
    path = os.path.join(GOLDEN, f"fullsize_{name}.json")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (python -m oracle.make_fullsize_golden)")
    with open(path) as fh:
        return json.load(fh)


def _sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _row(words, b):
    return ((words[b >> 6] >> np.uint64(b & 63)) & np.uint64(1)).astype(np.uint8)


def _check_prefix(gold, rho, dens, ov, pers, state):
    pre = [p for p in gold["prefix"] if p["rho"] == rho]
    if not pre:
        return False
    p = pre[0]
    for q, t in enumerate(gold["prefix_grid"]):
        c = np.stack([dens[q], ov[q], pers[q]]).astype("<i8")
        assert _sha(c) == p["counts_sha256"][q], f"all-replica counts differ at t={t}"
        assert int(dens[q].sum()) == p["density_total"][q]
    n, n0, f, t = state
    assert t == gold["prefix_grid"][-1]
    assert _sha(n0.astype("<u8")) == p["n0_sha256"], "n(0) differs"
    assert _sha(n.astype("<u8")) == p["n_sha256"], "n differs at the end of the prefix"
    assert _sha(f.astype("<u8")) == p["f_sha256"], "f differs at the end of the prefix"
    return True


def _run_case(gold, g, m, run):
    rho, R = run["rho"], gold["n_replicas"]
    grid, pgrid = gold["grid"], gold["prefix_grid"]
    assert grid == ka.log_time_grid(10_000) and pgrid == ka.log_time_grid(100)
    sim = ka.ka_init(g, m, rho, gold["seed"], R)
    assert sim.K == run["K"]
    assert ka.ka_sim_path(sim) == 1
    has_prefix = any(p["rho"] == rho for p in gold["prefix"])
    if has_prefix:
        _say(f"rho={rho}: all {R} replicas for {pgrid[-1]} sweeps")
        d1, o1, p1 = ka.ka_run(sim, pgrid)
        assert _check_prefix(gold, rho, d1, o1, p1, ka.ka_get_state(sim))
        rest = [t for t in grid if t > pgrid[-1]]
        head = [t for t in grid if t <= pgrid[-1]]
        assert head == pgrid
    else:
        d1 = o1 = p1 = np.zeros((0, R), dtype=np.int64)
        rest = grid
    _say(f"rho={rho}: to {grid[-1]} sweeps, sampled replicas {sorted(run['replicas'], key=int)}")
    d2, o2, p2 = ka.ka_run(sim, rest)
    dens, ov, pers = np.vstack([d1, d2]), np.vstack([o1, o2]), np.vstack([p1, p2])
    n, n0, f, t = ka.ka_get_state(sim)
    assert t == grid[-1]
    for b_str, want in run["replicas"].items():
        b = int(b_str)
        for q, tt in enumerate(grid):
            assert [int(dens[q, b]), int(ov[q, b]), int(pers[q, b])] == want["counts"][q], (tt, b)
        assert _sha(_row(n0, b)) == want["n0_sha256"], b
        assert _sha(_row(n, b)) == want["n_sha256"], b
        assert _sha(_row(f, b)) == want["f_sha256"], b
    sim.free()


def _prefix_only(gold, g, m, p):
    R = gold["n_replicas"]
    sim = ka.ka_init(g, m, p["rho"], gold["seed"], R)
    assert sim.K == p["K"] and ka.ka_sim_path(sim) == 1
    _say(f"rho={p['rho']}: all {R} replicas for {gold['prefix_grid'][-1]} sweeps")
    d, o, pe = ka.ka_run(sim, gold["prefix_grid"])
    assert _check_prefix(gold, p["rho"], d, o, pe, ka.ka_get_state(sim))
    sim.free()


@pytest.mark.parametrize("rho", [0.80, 0.85, 0.88])
def test_cubic128_full_length(rho):
    gold = _load("cubic128")
    runs = [r for r in gold["sampled"] if r["rho"] == rho]
    assert runs, rho
    g = ka.ka_graph_lattice(3, 128)
    _run_case(gold, g, gold["m"], runs[0])


@pytest.fixture(scope="module")
def rrg20():
    g = ka.ka_graph_rrg(1 << 20, 4, 1)
    return g


@pytest.mark.parametrize("rho", [0.50, 0.75])
def test_rrg20_full_length(rrg20, rho):
    gold = _load("rrg20")
    runs = [r for r in gold["sampled"] if r["rho"] == rho]
    assert runs, rho
    _run_case(gold, rrg20, gold["m"], runs[0])


def test_golden_prefixes_cover_listed_densities():
    """Every all-replica prefix has a full-length run at the same density (checked there),
    or is checked on its own here."""
    for name in ("cubic128", "rrg20"):
        gold = _load(name)
        sampled = {r["rho"] for r in gold["sampled"]}
        for p in gold["prefix"]:
            if p["rho"] in sampled:
                continue
            g = ka.ka_graph_lattice(3, 128) if name == "cubic128" else ka.ka_graph_rrg(1 << 20, 4, 1)
            _prefix_only(gold, g, gold["m"], p)
