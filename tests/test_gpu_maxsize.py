"""GPU checks at the largest lattices the library accepts (N = 2^30 sites, 64 replicas:
3D L = 1024 and 2D L = 32768; 24 GiB of device state per sim).

The oracle cannot run these sizes whole, so they are checked on sampled outputs it computes
one by one, and on properties that hold at any size:

- Initial state: for replicas 0 and 63 and 20,000 sampled sites, every occupied site's
  Philox key (u_i, i), computed by the oracle's own Philox, is below every empty site's key;
  with the exact count K this is the K-smallest-keys rule of the initial state.
- Dynamics: particle number conserved per replica; persistence <= overlap <= K; and split
  invariance: two sims with the same seed, one run 2 sweeps in one call and the other in
  two calls of 1 sweep, end with identical per-replica counts.
"""
import numpy as np
import pytest

from paper_1710_05155_amd import ka

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


@pytest.mark.parametrize("d,L", [(3, 1024), (2, 32768)])
def test_largest_lattice(oracle, d, L):
    g = ka.ka_graph_lattice(d, L)
    assert g.N == 1 << 30
    m, rho, seed, R = d, 0.85, 11, 64
    K = ka.ka_particles(g.N, rho)
    _say(f"max size: d={d} L={L} N=2^30 R={R} K={K}")
    a = ka.ka_init(g, m, rho, seed, R)
    t, dens, ov, pers = ka.ka_observe(a)
    assert t == 0 and (dens == K).all() and (ov == K).all() and (pers == K).all()
    n, _, _, _ = ka.ka_get_state(a, n0=False, f=False)
    rng = np.random.default_rng(d)
    sites = np.sort(rng.choice(g.N, size=20_000, replace=False)).astype(np.int64)
    for b in (0, 63):
        occ = ((n[0, sites] >> np.uint64(b)) & np.uint64(1)).astype(bool)
        assert occ.any() and (~occ).any()
        ctr = np.zeros((sites.size, 4), dtype=np.uint32)
        ctr[:, 1] = 0xFFFFFFFF
        ctr[:, 2] = sites.astype(np.uint32)
        ctr[:, 3] = b >> 1
        out = oracle.philox(ctr, [seed & 0xFFFFFFFF, seed >> 32]).astype(np.uint64)
        if b & 1:
            u = out[:, 2] | (out[:, 3] << np.uint64(32))
        else:
            u = out[:, 0] | (out[:, 1] << np.uint64(32))
        keys = list(zip(u.tolist(), sites.tolist()))
        top_occ = max(k for k, o in zip(keys, occ) if o)
        low_empty = min(k for k, o in zip(keys, occ) if not o)
        assert top_occ < low_empty, (b, top_occ, low_empty)
    del n
    bsim = ka.ka_init(g, m, rho, seed, R)
    ka.ka_sweep(a, 2)
    ka.ka_sweep(bsim, 1)
    ka.ka_sweep(bsim, 1)
    ta, da, oa, pa = ka.ka_observe(a)
    tb, db, ob, pb = ka.ka_observe(bsim)
    assert ta == tb == 2
    assert (da == K).all() and (pa <= oa).all() and (oa <= K).all()
    assert (oa < K).any(), "nothing moved in 2 sweeps"
    assert np.array_equal(da, db) and np.array_equal(oa, ob) and np.array_equal(pa, pb)
    a.free()
    bsim.free()
