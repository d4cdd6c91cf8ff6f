"""Randomised GPU parity: 40 configurations drawn with a fixed seed over every axis at once
(geometry and size, degree, activation number, density, replica count, noise mode, kernel
path, sweep chunking), each compared with the oracle bit for bit after every chunk."""
import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _configs(n=40, seed=2024):
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n):
        kind = ["lattice2", "lattice3", "rrg", "layered"][k % 4]
        if kind == "lattice2":
            geo = (2, int(rng.choice([4, 8, 12, 16, 20, 28, 36])))
        elif kind == "lattice3":
            geo = (3, int(rng.choice([4, 8, 12])))
        elif kind == "rrg":
            z = int(rng.integers(3, 7))
            N = int(rng.integers(z + 1, 500))
            N += (N * z) % 2
            geo = (N, z)
        else:
            geo = (int(rng.integers(2, 4)), int(rng.choice([4, 5, 6, 8])), int(rng.integers(1, 5)))
        R = 64 * int(rng.integers(1, 6))
        out.append(dict(kind=kind, geo=geo, R=R, rho=float(rng.uniform(0.05, 0.95)),
                        mfrac=float(rng.random()), noise=int(rng.integers(0, 2)),
                        path=int(rng.integers(1, 3)), seed=int(rng.integers(1, 1 << 40)),
                        chunks=[int(c) for c in rng.integers(0, 5, size=3)]))
    return out


@pytest.mark.parametrize("cfg", _configs(), ids=lambda c: f"{c['kind']}{c['geo']}R{c['R']}")
def test_random_config_parity(oracle, cfg):
    kind, geo = cfg["kind"], cfg["geo"]
    if kind.startswith("lattice"):
        g, og = ka.ka_graph_lattice(*geo), oracle.lattice(*geo)
    elif kind == "rrg":
        g = ka.ka_graph_rrg(geo[0], geo[1], cfg["seed"] & 0xFFFF)
        og = oracle.graph_from_adjacency(oracle.rrg_adjacency(geo[0], geo[1], cfg["seed"] & 0xFFFF)[0])
    else:
        g, og = ka.ka_graph_layered(*geo, 7), oracle.layered(*geo, 7)
    m = min(int(cfg["mfrac"] * og.z), og.z - 1)
    K = oracle.k_from_rho(og.N, cfg["rho"])
    print(f"[gpu-case] random config {cfg} m={m} K={K}", flush=True)
    sim = ka.ka_init_k(g, m, K, cfg["seed"], cfg["R"])
    path = cfg["path"]
    try:
        ka.ka_set_option(sim, ka.KA_OPT_PATH, path)
    except ka.KaError:
        ka.ka_set_option(sim, ka.KA_OPT_PATH, 1)
    ka.ka_set_option(sim, ka.KA_OPT_NOISE, cfg["noise"])
    orc = oracle.Sim(og, m, K, cfg["seed"], range(cfg["R"]), shared=bool(cfg["noise"]))
    for n in cfg["chunks"]:
        ka.ka_sweep(sim, n)
        orc.sweep(n)
        nn, n0, f, t = ka.ka_get_state(sim)
        assert t == orc.t
        assert np.array_equal(n0, oracle.pack(orc.occ0))
        assert np.array_equal(nn, oracle.pack(orc.occ))
        assert np.array_equal(f, oracle.pack(orc.moved))
    _, dens, ov, pers = ka.ka_observe(sim)
    od, oo, op = orc.observe()
    assert np.array_equal(dens, od) and np.array_equal(ov, oo) and np.array_equal(pers, op)
    sim.free()
