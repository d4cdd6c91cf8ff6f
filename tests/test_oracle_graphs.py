"""Pins of the oracle's graphs and edge classes by brute force.

- Lattice classes (mod-4 coordinate residues): every class holds N/4 edges and any two
  edges of one class are at graph distance >= 2 (no endpoint of one is an endpoint of, or
  a neighbour of an endpoint of, the other), checked pairwise on small lattices.
- Random regular graphs (Sec. 2.1): simple, z-regular, deterministic in the seed, and
  uniform over labelled simple cubic graphs on 6 vertices (chi-square over seeds): the
  configuration model with whole-pairing rejection is exactly uniform.
- Greedy distance-2 colouring: valid (same check as above) and greedy-minimal (each
  edge's colour is the smallest one not held by a conflicting earlier edge), with the
  conflict sets recomputed here from BFS distances.
- Layered random graphs (Sec. 5.2): simple, 2d-regular, every link projects onto a lattice
  bond, one copy is the plain lattice, each bond's links are a uniform permutation of the
  copies (chi-square), and the projected classes pass the same distance check.
"""
import itertools
from collections import Counter

import numpy as np
import pytest


def _bfs_dist_le1(adj, sources):
    """Set of vertices at distance <= 1 from the source set."""
    out = set(int(s) for s in sources)
    for s in sources:
        out.update(int(v) for v in adj[s])
    return out


def _check_classes_distance2(g):
    by_class = {}
    for e in range(g.E):
        by_class.setdefault(int(g.ecls[e]), []).append(e)
    for c, edges in by_class.items():
        for e1, e2 in itertools.combinations(edges, 2):
            near = _bfs_dist_le1(g.adj, [g.eu[e1], g.ev[e1]])
            assert g.eu[e2] not in near and g.ev[e2] not in near, (c, e1, e2)
    return by_class


@pytest.mark.parametrize("d,L", [(2, 4), (2, 8), (2, 12), (3, 4), (3, 8)])
def test_lattice_classes_independent(oracle, d, L):
    g = oracle.lattice(d, L)
    assert g.N == L ** d and g.z == 2 * d and g.E == d * g.N and g.C == 4 * d
    # adjacency: symmetric, simple
    for i in range(g.N):
        row = list(g.adj[i])
        assert len(set(row)) == g.z and i not in row
        for j in row:
            assert i in g.adj[j]
    # every edge appears once, endpoints adjacent
    pairs = {tuple(sorted((int(a), int(b)))) for a, b in zip(g.eu, g.ev)}
    assert len(pairs) == g.E
    for a, b in zip(g.eu, g.ev):
        assert b in g.adj[a]
    by_class = _check_classes_distance2(g)
    assert sorted(by_class) == list(range(g.C))
    assert all(len(v) == g.N // 4 for v in by_class.values())


def test_lattice_rejects_bad_sizes(oracle):
    for d, L in [(2, 6), (3, 2), (2, 0)]:
        with pytest.raises(ValueError):
            oracle.lattice(d, L)


@pytest.mark.parametrize("N,z,seed", [(64, 3, 1), (64, 4, 2), (100, 5, 3), (50, 6, 4), (1 << 10, 4, 1)])
def test_rrg_simple_regular_and_colouring(oracle, N, z, seed):
    adj, attempts = oracle.rrg_adjacency(N, z, seed)
    assert attempts >= 1
    assert adj.shape == (N, z)
    for i in range(N):
        row = list(adj[i])
        assert row == sorted(row) and len(set(row)) == z and i not in row
        for j in row:
            assert i in adj[j]
    adj2, attempts2 = oracle.rrg_adjacency(N, z, seed)
    assert np.array_equal(adj, adj2) and attempts == attempts2
    g = oracle.graph_from_adjacency(adj)
    assert g.E == N * z // 2
    # canonical order: u < v, lexicographic
    keys = list(zip(g.eu.tolist(), g.ev.tolist()))
    assert all(u < v for u, v in keys) and keys == sorted(keys)
    if N <= 128:
        _check_classes_distance2(g)
    # greedy minimality: colour(e) = mex of colours of earlier conflicting edges
    inc = {}
    for e in range(g.E):
        inc.setdefault(int(g.eu[e]), []).append(e)
        inc.setdefault(int(g.ev[e]), []).append(e)
    for e in range(g.E):
        near = _bfs_dist_le1(adj, [g.eu[e], g.ev[e]])
        used = {int(g.ecls[f]) for x in near for f in inc[x] if f < e}
        mex = 0
        while mex in used:
            mex += 1
        assert g.ecls[e] == mex


def test_rrg_uniform_over_labelled_cubic_graphs_on_6_vertices(oracle):
    """There are 70 labelled 3-regular simple graphs on 6 vertices; the configuration
    model with rejection hits each with probability 1/70."""
    n_seeds = 7000
    counts = Counter()
    for s in range(n_seeds):
        adj, _ = oracle.rrg_adjacency(6, 3, 1000 + s)
        key = tuple(sorted((i, int(j)) for i in range(6) for j in adj[i] if i < j))
        counts[key] += 1
    assert len(counts) == 70
    obs = np.array(list(counts.values()), dtype=float)
    exp = n_seeds / 70.0
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    # 69 degrees of freedom: mean 69, sd ~11.7; 140 is beyond p ~ 1e-7
    assert chi2 < 140.0, chi2


def test_rrg_rejects_bad_arguments(oracle):
    for N, z in [(5, 3), (3, 3), (1, 1)]:
        with pytest.raises(ValueError):
            oracle.rrg_adjacency(N, z, 1)


def test_graph_from_adjacency_rejects_non_simple(oracle):
    adj = np.array([[1, 1], [0, 0], [3, 3], [2, 2]], dtype=np.int32)  # multi-edges
    with pytest.raises(ValueError):
        oracle.graph_from_adjacency(adj)


# ------------------------------------------------------------------------ layered graphs (Sec. 5.2)
@pytest.mark.parametrize("d,L,M", [(2, 4, 3), (2, 8, 2), (3, 4, 2), (2, 6, 3)])
def test_layered_graph_structure_and_classes(oracle, d, L, M):
    g = oracle.layered(d, L, M, 11)
    Nb = L ** d
    assert g.N == Nb * M and g.z == 2 * d
    base = oracle.lattice(d, L) if L % 4 == 0 else None
    for v in range(g.N):
        row = [int(u) for u in g.adj[v]]
        assert len(set(row)) == g.z and v not in row
        for u in row:
            assert v in g.adj[u]
        # every link projects onto a lattice bond
        i = v % Nb
        proj = sorted(u % Nb for u in row)
        xs = np.unravel_index(i, (L,) * d, order="F")
        nbrs = []
        for mu in range(d):
            for s in (1, -1):
                y = list(xs)
                y[mu] = (y[mu] + s) % L
                nbrs.append(int(np.ravel_multi_index(y, (L,) * d, order="F")))
        assert proj == sorted(nbrs)
    _check_classes_distance2(g)
    if base is not None:
        assert g.C == 4 * d


def test_layered_single_copy_is_the_lattice(oracle):
    g = oracle.layered(3, 4, 1, 5)
    b = oracle.lattice(3, 4)
    assert np.array_equal(g.adj, np.sort(b.adj, axis=1))


def test_layered_permutations_uniform(oracle):
    """Each bond's links are a uniform random permutation of the copies (M = 3: six
    permutations, chi-square over all bonds of a 2D L=32 base lattice)."""
    d, L, M = 2, 32, 3
    adj = oracle.layered_adjacency(d, L, M, 123)
    Nb = L * L
    counts = {}
    for i in range(Nb):
        x, y = i % L, i // L
        j = ((x + 1) % L) + L * y                    # bond (i, i + e_0)
        perm = []
        for a in range(M):
            u = a * Nb + i
            partner = [int(v) for v in adj[u] if int(v) % Nb == j]
            assert len(partner) == 1
            perm.append(partner[0] // Nb)
        assert sorted(perm) == list(range(M))
        counts[tuple(perm)] = counts.get(tuple(perm), 0) + 1
    obs = np.array(list(counts.values()), dtype=float)
    assert len(obs) == 6
    exp = Nb / 6
    chi2 = float(((obs - exp) ** 2 / exp).sum())
    assert chi2 < 30.0, chi2
