"""Pins of the oracle's random numbers and exchange rule against things other than itself.

- Philox4x32-10 against rocRAND's independent host-callable implementation (library).
- The exchange rule against the paper's own Boolean formulation: the Karnaugh subset-OR
  threshold strings s_{k4}, s_{k5} (Sec. 3.2, generalised from m=3 to any m), the move
  permissions s_i = s_{i4} & s_{j5}, s_j = s_{j4} & s_{i5}, and Table 1 (golden fixture),
  exhaustively over every local configuration for z = 3..6 and every m <= z-1.
"""
import itertools
import os
import shutil
import subprocess

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    rows = {}
    with open(os.path.join(GOLDEN, "table1_update.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            ni, nj, si, sj, a, b = (int(v) for v in line.split())
            rows[(ni, nj, si, sj)] = (a, b)
    assert len(rows) == 16
    return rows


def test_table1_matches_closed_forms():
    """The fixture transcribes Table 1; the paper's explicit equations for n_i+ and n_j+
    (Sec. 3.2) must give the same 16 rows."""
    for (ni, nj, si, sj), (a, b) in _table1().items():
        ni_p = (ni & nj) | (nj & sj) | (ni & (1 - si))
        nj_p = (ni & nj) | (ni & si) | (nj & (1 - sj))
        assert (ni_p, nj_p) == (a, b)


def _s_at_most(nbrs, limit):
    """Paper's Karnaugh form: 1 iff NOT (some (limit+1)-subset of the neighbours is all
    occupied), i.e. at most `limit` occupied neighbours.  Empty family -> 1."""
    k = limit + 1
    if k > len(nbrs):
        return 1
    for sub in itertools.combinations(range(len(nbrs)), k):
        if all(nbrs[q] for q in sub):
            return 0
    return 1


@pytest.mark.parametrize("z", [3, 4, 5, 6])
def test_exchange_rule_equals_paper_boolean_form(oracle, z):
    table = _table1()
    for m in range(z):
        for ni, nj in itertools.product((0, 1), repeat=2):
            for oi in itertools.product((0, 1), repeat=z - 1):
                for oj in itertools.product((0, 1), repeat=z - 1):
                    full_i = list(oi) + [nj]     # all z neighbours of i (partner j included)
                    full_j = list(oj) + [ni]
                    s_i4 = _s_at_most(full_i, m)
                    s_i5 = _s_at_most(full_i, m + 1)
                    s_j4 = _s_at_most(full_j, m)
                    s_j5 = _s_at_most(full_j, m + 1)
                    si = s_i4 & s_j5
                    sj = s_j4 & s_i5
                    want = table[(ni, nj, si, sj)]
                    got = oracle.exchange(z, m, ni, nj, oi, oj, 1)
                    assert got == want, (z, m, ni, nj, oi, oj)
                    assert oracle.exchange(z, m, ni, nj, oi, oj, 0) == (ni, nj)


def test_philox_matches_rocrand_library(oracle, tmp_path):
    """Independent implementation: rocRAND's Philox4x32-10 block function (host code)."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers / hipcc not available")
    exe = tmp_path / "probe"
    subprocess.run([hipcc, "-O1", "-o", str(exe), os.path.join(GOLDEN, "rocrand_philox_probe.cpp")],
                   check=True, capture_output=True, cwd=str(tmp_path))
    rng = np.random.default_rng(20240611)
    n = 4000
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    keys = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # include the all-zero and all-ones corners
    ctr[0] = 0
    keys[0] = 0
    ctr[1] = 0xFFFFFFFF
    keys[1] = 0xFFFFFFFF
    text = "".join(" ".join(f"{v:x}" for v in list(ctr[q]) + list(keys[q])) + "\n" for q in range(n))
    res = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True)
    lib_out = np.array([[int(v, 16) for v in line.split()] for line in res.stdout.strip().splitlines()],
                       dtype=np.uint64)
    ours = np.stack([oracle.philox(ctr[q], keys[q])[0] for q in range(n)]).astype(np.uint64)
    assert lib_out.shape == (n, 4)
    assert np.array_equal(lib_out, ours)
