"""Seeded synthetic workload recipes (inputs only; none of the method's arithmetic).

- log_time_grid: the log-spaced observation grid, 0 and the distinct floor(10^(k/10)).
- batch_manifest: 256 uneven instances: geometry uniform over {2D lattice, 3D lattice,
  random regular graph}; 2D L in {32, 64, 128, 256, 512}, 3D L in {16, 32, 64, 128}, RRG
  N in {2^12 .. 2^18} with z in {3, 4, 5}; m uniform in {1 .. z-1} (m = 0 freezes every
  particle with an occupied neighbour); rho uniform in [0.5, 0.9]; 64 replicas; instance k
  has seed 1+k and graph seed 1000+k; numpy default_rng(4).
- serving_trace: Poisson arrivals (mean rate per second given) of jobs drawn from the same
  instance mix, sweeps log-uniform in [10^2, 10^4]; numpy default_rng(5).
"""
from __future__ import annotations

import math

import numpy as np


def log_time_grid(t_max: int, per_decade: int = 10) -> list[int]:
    out = {0}
    k = 0
    while True:
        v = int(math.floor(10.0 ** (k / per_decade)))
        if v > t_max:
            break
        out.add(v)
        k += 1
    return sorted(out)


def _instance(rng, k: int) -> dict:
    kind = int(rng.integers(0, 3))
    if kind == 0:
        L = int(rng.choice([32, 64, 128, 256, 512]))
        z = 4
        inst = dict(kind="lattice", d=2, L=L, N=L * L, z=z)
    elif kind == 1:
        L = int(rng.choice([16, 32, 64, 128]))
        z = 6
        inst = dict(kind="lattice", d=3, L=L, N=L ** 3, z=z)
    else:
        N = 1 << int(rng.integers(12, 19))
        z = int(rng.choice([3, 4, 5]))
        inst = dict(kind="rrg", N=N, z=z, graph_seed=1000 + k)
    inst["m"] = int(rng.integers(1, inst["z"]))
    inst["rho"] = float(rng.uniform(0.5, 0.9))
    inst["R"] = 64
    inst["seed"] = 1 + k
    return inst


def batch_manifest(n: int = 256, sweeps: int = 1000, seed: int = 4) -> list[dict]:
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        inst = _instance(rng, k)
        inst["sweeps"] = sweeps
        out.append(inst)
    return out


def serving_trace(n_jobs: int, rate_per_s: float, seed: int = 5,
                  sweeps_range=(100, 10_000)) -> list[dict]:
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    lo, hi = math.log(sweeps_range[0]), math.log(sweeps_range[1])
    for k in range(n_jobs):
        t += float(rng.exponential(1.0 / rate_per_s))
        inst = _instance(rng, k)
        inst["sweeps"] = int(round(math.exp(rng.uniform(lo, hi))))
        inst["arrival_s"] = t
        out.append(inst)
    return out
