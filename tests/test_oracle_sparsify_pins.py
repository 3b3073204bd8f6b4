"""Pins of the oracle's spectral sparsification (Sec. 3.2, Alg. 2 and
Alg. 6: effective resistances, maximum spanning tree by resistance, then
edges in decreasing resistance up to n log n).

The resistance estimate is Spielman and Srivastava's random projection:
on a tree it is exact (the flow of each sign vector through a tree edge is
its sign), its conjugate-gradient solves are checked against the
pseudo-inverse, and its mean over many projections against exact
resistances (whose sum is n - 1 by Foster's theorem).  The choice of edges
is checked against networkx's maximum spanning tree.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O


def _exact_R(g):
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    A = np.zeros((g.n, g.n))
    A[u, v] = 1
    A[v, u] = 1
    L = np.diag(A.sum(1)) - A
    P = np.linalg.pinv(L)
    return P[u, u] + P[v, v] - 2 * P[u, v], L


def test_foster_theorem_exact_resistances():
    for g in (G.ba(60, 3, 1), G.grid_2d(6, 7), G.complete(9)):
        R, _ = _exact_R(g)
        assert np.isclose(R.sum(), g.n - 1)


@pytest.mark.parametrize("g", [G.path(40), G.star(30), G.ba(200, 1, 4)], ids=["path", "star", "tree"])
def test_tree_estimate_is_exact(g):
    R, its = O.effective_resistance(g.n, g.row_ptr, g.col_idx, q=8, seed=3)
    assert np.allclose(R, 1.0, atol=1e-8)


def test_cg_solves_against_pseudo_inverse():
    g = G.ba(150, 4, 9)
    R, its, X, B = O.effective_resistance(g.n, g.row_ptr, g.col_idx, q=6, seed=11, return_x=True)
    _, L = _exact_R(g)
    P = np.linalg.pinv(L)
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    ref = P @ B
    # potential differences (the constant offset of x does not matter)
    assert np.allclose(X[u] - X[v], ref[u] - ref[v], atol=1e-8)
    assert np.allclose(L @ X, B, atol=1e-8)


def test_estimate_is_unbiased():
    g = G.er(40, 0.2, 5)
    Rex, _ = _exact_R(g)
    R, _ = O.effective_resistance(g.n, g.row_ptr, g.col_idx, q=3000, seed=1)
    assert abs((R / Rex).mean() - 1) < 0.01
    assert np.max(np.abs(R / Rex - 1)) < 0.15
    assert abs(R.sum() - (g.n - 1)) < 0.02 * (g.n - 1)


def test_signs_are_the_generator_bits():
    s = O.jl_signs(77, 3, 5)
    for k in range(3):
        for e in range(5):
            assert s[k, e] == (-1.0 if O.splitmix64(77, k * 5 + e + 1) >= 2**63 else 1.0)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_selection_is_max_spanning_tree_plus_top_edges(seed):
    import networkx as nx
    g = G.er(120, 0.25, seed)
    rng = np.random.default_rng(seed)
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    m = len(u)
    R = rng.uniform(0, 1, m)
    target = int(np.ceil(g.n * np.log(g.n)))
    keep = O.sparsify_select(g.n, g.row_ptr, g.col_idx, R)
    assert keep.sum() == min(m, target)
    H = nx.Graph()
    H.add_nodes_from(range(g.n))
    for e in range(m):
        H.add_edge(int(u[e]), int(v[e]), weight=R[e], idx=e)
    T = nx.maximum_spanning_tree(H)
    tree = np.zeros(m, bool)
    for a, b, d in T.edges(data=True):
        tree[d["idx"]] = True
    assert np.all(keep[tree])
    rest = np.flatnonzero(~tree)
    top = rest[np.argsort(-R[rest], kind="stable")][:keep.sum() - tree.sum()]
    assert np.array_equal(np.sort(np.flatnonzero(keep & ~tree)), np.sort(top))


def test_selection_keeps_components_and_small_graphs():
    g = G.disjoint_union([G.complete(12), G.cycle(7), G.empty(2)])
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    R = np.linspace(0.1, 0.9, len(u))
    keep = O.sparsify_select(g.n, g.row_ptr, g.col_idx, R, target=20)
    assert keep.sum() == 20
    import networkx as nx
    H = nx.Graph()
    H.add_nodes_from(range(g.n))
    H.add_edges_from(zip(u[keep], v[keep]))
    assert nx.number_connected_components(H) == 4       # K12, C7 and two isolated vertices
    keep = O.sparsify_select(g.n, g.row_ptr, g.col_idx, R, target=3)
    assert keep.sum() == 11 + 6                           # the forest alone exceeds the target
