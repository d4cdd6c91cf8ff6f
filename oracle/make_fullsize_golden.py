"""Write the stored expected values for the full-length parity tests (tests/golden/).

TEST INFRASTRUCTURE ONLY.  Calls nothing but the oracle (oracle/oracle.py, liboracle.so) and
runs on the CPU; the files it writes are compared with the library by
tests/test_gpu_fullsize_golden.py.

Workloads (all seeds 1, the observation grid is 0 and the distinct floor(10^(k/10)) up to
10^4, 38 points):
  cubic128  3D periodic lattice L=128 (Sec. 2.1, z=6), m=3, 256 replicas;
            replicas {0, 63, 64, 255} at rho = 0.80, 0.85, 0.88 for the full 10^4 sweeps;
            all 256 replicas at rho = 0.85 for the first 100 sweeps.
  rrg20     random regular graph N=2^20, z=4 (Sec. 2.1, configuration model, graph seed 1),
            m=2, 64 replicas; replicas {0, 63} at rho = 0.50 and 0.75 for the full 10^4
            sweeps; all 64 replicas at rho = 0.50 and 0.75 for the first 100 sweeps.

Recorded per run: the per-replica counts of Sec. 2.2 / Sec. 3.3 (density, overlap,
persistence) at every grid point, and sha256 digests of the final state:
  - a sampled replica's row: sha256 of its N occupation bytes (0/1, canonical site order)
    for n(t), n(0) and the moved-ever mask f;
  - an all-replica run: sha256 of the canonical export layout (uint64 [W][N], bit b & 63 of
    word b >> 6 is replica b, little-endian) of n, n(0) and f, and per grid point the sha256
    of the int64 [3][R] counts (rows density, overlap, persistence; little-endian).

Every replica is an independent chain (its trajectory does not depend on which other
replicas run beside it), so the work is split into one task per replica (long runs) or per
16 replicas (prefixes), each in its own single-threaded process.

    python -m oracle.make_fullsize_golden [--jobs 8] [--only cubic128|rrg20]

takes about two hours on 8 cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed
import multiprocessing as mp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GOLDEN = os.path.join(ROOT, "tests", "golden")
T_MAX = 10_000
PREFIX = 100
SEED = 1


def log_grid(t_max: int) -> list[int]:
    """0 and the distinct floor(10^(k/10)) <= t_max."""
    out = {0}
    k = 0
    while True:
        v = int(math.floor(10.0 ** (k / 10)))
        if v > t_max:
            break
        out.add(v)
        k += 1
    return sorted(out)


def _sha(a) -> str:
    import numpy as np
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


_graphs: dict = {}


def _graph(name: str):
    from oracle import oracle as o
    if name not in _graphs:
        if name == "cubic128":
            _graphs[name] = o.lattice(3, 128)
        else:
            _graphs[name] = o.rrg(1 << 20, 4, 1)
    return _graphs[name]


def _m(name: str) -> int:
    return 3 if name == "cubic128" else 2


def run_task(name: str, rho: float, replicas: list[int], t_max: int) -> dict:
    """Run the listed replicas from t=0 to t_max, observing at every grid point."""
    import numpy as np
    from oracle import oracle as o
    t0 = time.time()
    g = _graph(name)
    K = o.k_from_rho(g.N, rho)
    sim = o.Sim(g, _m(name), K, SEED, replicas)
    counts = []
    for t in log_grid(t_max):
        sim.sweep(t - sim.t)
        d, ov, p = sim.observe()
        counts.append(np.stack([d, ov, p]).astype(np.int64))   # [3][r]
    return dict(name=name, rho=rho, replicas=replicas, K=K, t_max=t_max,
                counts=np.stack(counts),                         # [grid][3][r]
                occ=sim.occ, occ0=sim.occ0, moved=sim.moved,
                seconds=time.time() - t0)


def _tasks(only: str | None, t_max: int, prefix: int):
    tasks = []
    if only in (None, "cubic128"):
        for rho in (0.80, 0.85, 0.88):
            for b in (0, 63, 64, 255):
                tasks.append(("cubic128", rho, [b], t_max))
        for q in range(16):
            tasks.append(("cubic128", 0.85, list(range(16 * q, 16 * q + 16)), prefix))
    if only in (None, "rrg20"):
        for rho in (0.50, 0.75):
            for b in (0, 63):
                tasks.append(("rrg20", rho, [b], t_max))
        for rho in (0.50, 0.75):
            for q in range(4):
                tasks.append(("rrg20", rho, list(range(16 * q, 16 * q + 16)), prefix))
    # longest first: full-length runs, then prefixes
    tasks.sort(key=lambda a: -a[3] * len(a[2]))
    return tasks


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", choices=["cubic128", "rrg20"], default=None)
    ap.add_argument("--t-max", type=int, default=T_MAX, help="shorter runs, for a dry run")
    ap.add_argument("--prefix", type=int, default=PREFIX, help="shorter prefix, for a dry run")
    ap.add_argument("--out", default=GOLDEN, help="output directory")
    args = ap.parse_args()
    import numpy as np
    from oracle import oracle as o

    os.environ["OMP_NUM_THREADS"] = "1"     # one replica chain per process
    tasks = _tasks(args.only, args.t_max, args.prefix)
    results: dict = {}
    ctx = mp.get_context("spawn")
    t_start = time.time()
    with ProcessPoolExecutor(max_workers=args.jobs, mp_context=ctx) as ex:
        futs = {ex.submit(run_task, *a): a for a in tasks}
        for k, fut in enumerate(as_completed(futs)):
            r = fut.result()
            a = futs[fut]
            results[(a[0], a[1], tuple(a[2]), a[3])] = r
            print(f"[{time.time() - t_start:7.0f} s] {k + 1}/{len(tasks)} {a[0]} rho={a[1]} "
                  f"replicas {a[2][0]}..{a[2][-1]} to t={a[3]} ({r['seconds']:.0f} s)", flush=True)

    names = ["cubic128", "rrg20"] if args.only is None else [args.only]
    for name in names:
        N = 128 ** 3 if name == "cubic128" else 1 << 20
        desc = dict(
            cubic128="3D periodic lattice L=128, z=6, m=3, seed 1, 256 replicas",
            rrg20="random regular graph N=2^20, z=4, graph seed 1, m=2, seed 1, 64 replicas",
        )[name]
        R = 256 if name == "cubic128" else 64
        out = dict(workload=desc, N=N, m=_m(name), seed=SEED, n_replicas=R,
                   generated_by="oracle/make_fullsize_golden.py (oracle only, CPU)",
                   grid=log_grid(args.t_max), prefix_grid=log_grid(args.prefix), sampled=[],
                   prefix=[])
        # sampled replicas, full length
        by_rho: dict = {}
        for (nm, rho, reps, tm), r in results.items():
            if nm != name or tm != args.t_max:
                continue
            e = by_rho.setdefault(rho, dict(rho=rho, K=r["K"], replicas={}))
            b = reps[0]
            e["replicas"][str(b)] = dict(
                counts=r["counts"][:, :, 0].tolist(),            # [grid][density, overlap, persistence]
                n_sha256=_sha(r["occ"][0]), n0_sha256=_sha(r["occ0"][0]),
                f_sha256=_sha(r["moved"][0]))
        out["sampled"] = [by_rho[k] for k in sorted(by_rho)]
        # all replicas, prefix
        pre: dict = {}
        for (nm, rho, reps, tm), r in results.items():
            if nm != name or tm != args.prefix:
                continue
            pre.setdefault(rho, []).append(r)
        for rho in sorted(pre):
            parts = sorted(pre[rho], key=lambda r: r["replicas"][0])
            reps = [b for r in parts for b in r["replicas"]]
            assert reps == list(range(R)), (name, rho, reps[:5])
            counts = np.concatenate([r["counts"] for r in parts], axis=2)   # [grid][3][R]
            occ = np.concatenate([r["occ"] for r in parts])
            occ0 = np.concatenate([r["occ0"] for r in parts])
            moved = np.concatenate([r["moved"] for r in parts])
            out["prefix"].append(dict(
                rho=rho, K=parts[0]["K"],
                counts_sha256=[_sha(counts[q].astype("<i8")) for q in range(counts.shape[0])],
                density_total=counts[:, 0, :].sum(axis=1).tolist(),
                overlap_total=counts[:, 1, :].sum(axis=1).tolist(),
                persistence_total=counts[:, 2, :].sum(axis=1).tolist(),
                n_sha256=_sha(o.pack(occ).astype("<u8")),
                n0_sha256=_sha(o.pack(occ0).astype("<u8")),
                f_sha256=_sha(o.pack(moved).astype("<u8"))))
        path = os.path.join(args.out, f"fullsize_{name}.json")
        text = json.dumps(out, indent=1)
        # one line per list of numbers
        text = re.sub(r"\[[\s\d,.\-]*\]", lambda mt: re.sub(r"\s+", "", mt.group(0)), text)
        text = text.replace(",", ", ").replace(",  ", ", ")
        with open(path, "w") as fh:
            fh.write(text + "\n")
        print("wrote", path, flush=True)


if __name__ == "__main__":
    main()
