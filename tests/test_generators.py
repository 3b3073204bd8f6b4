"""Input generators: seeded, canonical, shaped as requested."""
import numpy as np

import graphgen as G


def canonical(g):
    rp, ci = g.row_ptr, g.col_idx
    assert rp[0] == 0 and rp[-1] == len(ci) and np.all(np.diff(rp) >= 0)
    for v in range(g.n):
        row = ci[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0) and not np.any(row == v)
        assert np.all((row >= 0) & (row < g.n))
    src = np.repeat(np.arange(g.n), g.degrees())
    fwd = set(zip(src.tolist(), ci.tolist()))
    assert all((w, v) in fwd for v, w in fwd)


def test_seeds_reproduce():
    for f in (lambda s: G.ba(2000, 4, s), lambda s: G.er(1000, 0.01, s),
              lambda s: G.rgg(2000, 8, s), lambda s: G.sbm(2000, 8, s)):
        a, b, c = f(7), f(7), f(8)
        assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col_idx, b.col_idx)
        assert not (a.nnz == c.nnz and np.array_equal(a.col_idx, c.col_idx))


def test_canonical_and_shapes():
    g = G.ba(5000, 4, 1)
    canonical(g)
    assert g.m == 10 + (5000 - 5) * 4
    canonical(G.rgg(3000, 10, 2))
    canonical(G.sbm(3000, 10, 3))
    canonical(G.er(800, 0.05, 4))
    canonical(G.grid_2d(7, 9))
    canonical(G.hypercube(5))
    canonical(G.complete_bipartite(3, 4))
    assert abs(G.rgg(20000, 12, 5).degrees().mean() - 12) < 1.0
    assert abs(G.sbm(20000, 12, 6).degrees().mean() - 12) < 0.5
    assert abs(G.er(4000, 0.01, 7).degrees().mean() - 0.01 * 3999) < 1.0


def test_dirty_keeps_edge_set():
    g = G.ba(300, 3, 9)
    d = G.dirty(g, 10)
    assert d.nnz > g.nnz
    clean = G.from_edges(d.n, np.stack([np.repeat(np.arange(d.n), d.degrees()), d.col_idx], 1))
    assert np.array_equal(clean.row_ptr, g.row_ptr) and np.array_equal(clean.col_idx, g.col_idx)


def test_workload_recipes():
    g = G.config_grid()
    assert g.n == 1024 and g.m == 1984
    src = G.config_ba_sources(64)
    assert len(set(src.tolist())) == 64 and src.min() >= 0 and src.max() < 100_000
    params = G.config_batch_params(300)
    ns = np.array([p[1] for p in params])
    assert ns.min() >= 256 and ns.max() <= 16384
    assert [p[0] for p in params[:6]] == [0, 1, 2, 0, 1, 2]
    jobs = G.config_stream_jobs(50)
    assert all(j["k"] in (10, 15, 30) for j in jobs)
    assert all(jobs[i]["t"] < jobs[i + 1]["t"] for i in range(49))
