"""The C ABI used from C: tests/c_api_example.c includes include/ka.h alone, is compiled as
strict C11 and linked against the in-tree libka.so; on the GPU its printed counts, state words
and averages must equal the oracle's for the same graphs, seeds and times."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1710_05155_amd import ka

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_api_example.c")
GCC = ["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include")]


def test_example_compiles_as_strict_c11():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    subprocess.run([*GCC, "-fsyntax-only", SRC], check=True)


def _build(tmp_path):
    pkg = os.path.dirname(ka.LIB_PATH)
    exe = str(tmp_path / "c_api_example")
    subprocess.run([*GCC, SRC, "-L", pkg, "-lka", "-Wl,-rpath-link,/opt/rocm/lib",
                    f"-Wl,-rpath,{pkg}", "-o", exe], check=True)
    return exe


def _parse(text):
    rows = {}
    for line in text.splitlines():
        key, *vals = line.split()
        rows.setdefault(key, []).append(vals)
    return rows


@pytest.mark.gpu
def test_c_program_matches_oracle(oracle, tmp_path):
    exe = _build(tmp_path)
    print("[gpu-case] C program through include/ka.h", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = _parse(r.stdout)

    # 1. lattice L = 8, 128 replicas, m = 2, rho = 0.5, seed 3, observed at 0, 1, 3, 6
    og = oracle.lattice(2, 8)
    K = oracle.k_from_rho(og.N, 0.5)
    assert rows["lattice_graph"][0] == [str(og.N), "4", str(og.E), str(og.C)]
    assert int(rows["lattice_K"][0][0]) == K
    orc = oracle.Sim(og, 2, K, 3, range(128))
    ovs, perss = [], []
    for q, t in enumerate((0, 1, 3, 6)):
        orc.sweep(t - orc.t)
        d, o, p = orc.observe()
        got = {k: np.array([int(v) for v in rows[f"lattice_{k}"][q][1:]]) for k in ("density", "overlap", "persistence")}
        assert np.array_equal(got["density"], d) and np.array_equal(got["overlap"], o)
        assert np.array_equal(got["persistence"], p)
        ovs.append(o)
        perss.append(p)
    assert int(rows["lattice_t"][0][0]) == 6
    n = np.array([int(v) for v in rows["lattice_n"][0]], dtype=np.uint64).reshape(2, og.N)
    f = np.array([int(v) for v in rows["lattice_f"][0]], dtype=np.uint64).reshape(2, og.N)
    assert np.array_equal(n, oracle.pack(orc.occ)) and np.array_equal(f, oracle.pack(orc.moved))
    for q, vals in enumerate(rows["lattice_derived"]):
        C, chi4, P = oracle.derived(og.N, K, ovs[q], perss[q])
        assert np.allclose([float(v) for v in vals[1:]], [C, chi4, P], rtol=1e-12, atol=1e-12)

    # 2. random regular graph N = 100, z = 3, graph seed 11, K = 40, m = 1, 64 replicas, seed 5
    adj, _ = oracle.rrg_adjacency(100, 3, 11)
    gg = oracle.graph_from_adjacency(adj)
    orc = oracle.Sim(gg, 1, 40, 5, range(64))
    orc.sweep(5)
    d, o, p = orc.observe()
    assert int(rows["graph_t"][0][0]) == 5
    for key, ref in (("density", d), ("overlap", o), ("persistence", p)):
        assert np.array_equal(np.array([int(v) for v in rows[f"graph_{key}"][0][1:]]), ref), key
    n = np.array([int(v) for v in rows["graph_n"][0]], dtype=np.uint64).reshape(1, 100)
    assert np.array_equal(n, oracle.pack(orc.occ))

    # 3. argument error
    assert rows["error"][0] == [str(ka.KA_EINVAL), "null"]
