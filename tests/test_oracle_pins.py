"""Pins of the CPU oracle against what the paper and mathematics fix.

Every check here is independent of the oracle's own code path: Floyd-Warshall
and networkx for hop distances, closed forms for structured graphs, the BFS
certificate, the k nearest hops from networkx distances for the truncated search, the
companion-matrix roots of the membership polynomial, closed-form bandwidths,
and a hand-worked example under tests/golden/.
"""
import math
import os

import networkx as nx
import numpy as np
import pytest

import graphgen as G
import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ helpers

def floyd_warshall(g):
    n = g.n
    INF = 10**9
    d = np.full((n, n), INF, dtype=np.int64)
    np.fill_diagonal(d, 0)
    for v in range(n):
        for w in g.neighbors(v):
            if w != v:
                d[v, w] = 1
    for m in range(n):
        d = np.minimum(d, d[:, m:m + 1] + d[m:m + 1, :])
    return np.where(d >= INF, 255, d).astype(np.int64)


def to_nx(g):
    h = nx.Graph()
    h.add_nodes_from(range(g.n))
    for v in range(g.n):
        for w in g.neighbors(v):
            if w != v:
                h.add_edge(v, int(w))
    return h


def knn_from_dist(dist_row, s, k):
    """k smallest (hop, id), v != s, reachable; padded -- from a distance row
    obtained independently of the oracle."""
    cand = [(int(dist_row[v]), v) for v in range(len(dist_row)) if v != s and 0 <= dist_row[v] < 255]
    cand.sort()
    ids = [v for _, v in cand[:k]] + [-1] * max(0, k - len(cand))
    hops = [h for h, _ in cand[:k]] + [255] * max(0, k - len(cand))
    return np.array(ids, dtype=np.int32), np.array(hops, dtype=np.uint8)


def small_graph_family(count, seed0=11):
    """Seeded small graphs: sparse/dense/disconnected/isolated, n <= 40."""
    out = []
    for i in range(count):
        u = G.uniform(G.mix_seed(seed0, i), 2)
        n = 1 + int(u[0] * 40)
        p = [0.02, 0.05, 0.1, 0.2, 0.5, 0.9][i % 6]
        out.append(G.tiny_random(n, p, G.mix_seed(seed0 + 1, i)))
    return out


# ------------------------------------------------------------ P-APSP pins

def test_apsp_matches_floyd_warshall_and_networkx():
    graphs = small_graph_family(1000)
    graphs += [G.path(1), G.empty(5), G.star(7), G.cycle(9), G.complete(6)]
    checked_nx = 0
    for g in graphs:
        ids, hops, hm = O.knn_build(g, 3, hop_matrix=True, threads=1)
        fw = floyd_warshall(g)
        assert np.array_equal(hm.astype(np.int64), fw), g.name
        if checked_nx < 150:
            ref = dict(nx.all_pairs_shortest_path_length(to_nx(g)))
            for s in range(g.n):
                row = np.full(g.n, 255)
                for t, d in ref[s].items():
                    row[t] = d
                assert np.array_equal(hm[s].astype(np.int64), row)
            checked_nx += 1


def test_apsp_symmetric_on_random_graphs():
    for i in range(20):
        g = G.er(60, 0.05, 900 + i)
        _, _, hm = O.knn_build(g, 5, hop_matrix=True)
        assert np.array_equal(hm, hm.T)


# ---------------------------------------------------------- P-closed pins

def test_closed_forms_hops():
    g = G.grid_2d(32, 32)
    _, _, hm = O.knn_build(g, 15, hop_matrix=True)
    r, c = np.divmod(np.arange(1024), 32)
    expect = np.abs(r[:, None] - r[None, :]) + np.abs(c[:, None] - c[None, :])
    assert np.array_equal(hm.astype(np.int64), expect)

    g = G.complete(20)
    _, _, hm = O.knn_build(g, 5, hop_matrix=True)
    assert np.array_equal(hm.astype(np.int64), 1 - np.eye(20, dtype=np.int64))

    n = 200
    _, _, hm = O.knn_build(G.path(n), 5, hop_matrix=True)
    i = np.arange(n)
    assert np.array_equal(hm.astype(np.int64), np.abs(i[:, None] - i[None, :]))

    n = 101
    _, _, hm = O.knn_build(G.cycle(n), 5, hop_matrix=True)
    dd = np.abs(i[:n, None] - i[None, :n])
    assert np.array_equal(hm.astype(np.int64), np.minimum(dd, n - dd))

    _, _, hm = O.knn_build(G.star(30), 5, hop_matrix=True)
    expect = np.full((31, 31), 2)
    expect[0, :] = 1
    expect[:, 0] = 1
    np.fill_diagonal(expect, 0)
    assert np.array_equal(hm.astype(np.int64), expect)

    d = 7
    _, _, hm = O.knn_build(G.hypercube(d), 5, hop_matrix=True)
    v = np.arange(1 << d)
    x = v[:, None] ^ v[None, :]
    pc = np.zeros_like(x)
    for b in range(d):
        pc += (x >> b) & 1
    assert np.array_equal(hm.astype(np.int64), pc)

    a, b = 6, 9
    _, _, hm = O.knn_build(G.complete_bipartite(a, b), 4, hop_matrix=True)
    side = np.arange(a + b) >= a
    expect = np.where(side[:, None] == side[None, :], 2, 1)
    np.fill_diagonal(expect, 0)
    assert np.array_equal(hm.astype(np.int64), expect)


def test_hop_range_limit():
    """A finite hop above 254 cannot be stored in the uint8 hop matrix."""
    _, _, hm = O.knn_build(G.path(255), 3, hop_matrix=True)
    assert hm.max() == 254
    with pytest.raises(O.OracleError) as e:
        O.knn_build(G.path(256), 3, hop_matrix=True)
    assert e.value.status == O.ERANGE
    ids, hops, _ = O.knn_build(G.path(400), 3)          # kNN alone is fine
    assert hops.max() <= 3


# ------------------------------------------------------------ P-cert pins

def bfs_certificate(g, s, dist):
    """Graph500-style check that ``dist`` are BFS hop distances from s."""
    assert dist[s] == 0
    src = np.repeat(np.arange(g.n), g.degrees())
    dst = g.col_idx
    ds, dd = dist[src], dist[dst]
    reached_s, reached_d = ds >= 0, dd >= 0
    assert np.all(reached_s == reached_d), "edge joins reached and unreached"
    both = reached_s & reached_d
    assert np.all(np.abs(ds[both] - dd[both]) <= 1)
    # every reached v != s has a neighbour one hop closer
    has_parent = np.zeros(g.n, dtype=bool)
    has_parent[src[both & (dd == ds - 1)]] = True
    reached = dist >= 0
    reached[s] = False
    assert np.all(has_parent[reached])


def test_bfs_certificate_on_generated_families():
    gs = [G.ba(3000, 4, 5), G.rgg(3000, 8, 6), G.sbm(3000, 10, 7), G.er(2000, 0.004, 8),
          G.grid_2d(20, 50)]
    for g in gs:
        for s in [0, g.n // 3, g.n - 1]:
            bfs_certificate(g, s, O.bfs_dist(g, s))


# ------------------------------------------------------------- P-knn pins

def test_knn_grid_closed_form():
    g = G.grid_2d(32, 32)
    ids, hops, _ = O.knn_build(g, 15)
    pids, phops = O.knn_partial(g, 15)
    for r in range(32):
        for c in range(32):
            s = 32 * r + c
            rr, cc = np.divmod(np.arange(1024), 32)
            dist = np.abs(rr - r) + np.abs(cc - c)
            e_ids, e_hops = knn_from_dist(dist, s, 15)
            assert np.array_equal(ids[s], e_ids) and np.array_equal(hops[s], e_hops)
            assert np.array_equal(pids[s], e_ids) and np.array_equal(phops[s], e_hops)
    # interior row: 4 at hop 1, 8 at hop 2, then the three smallest hop-3 ids
    r, c = 10, 17
    s = 32 * r + c
    assert list(hops[s]) == [1] * 4 + [2] * 8 + [3] * 3
    assert list(ids[s][12:]) == [32 * (r - 3) + c, 32 * (r - 2) + c - 1, 32 * (r - 2) + c + 1]
    # boundary row (0, c): the radius-3 ball has exactly 15 other vertices
    s = 9
    assert list(hops[s]) == [1] * 3 + [2] * 5 + [3] * 7


def test_knn_star_complete_dense():
    g = G.star(40)
    ids, hops, _ = O.knn_build(g, 15)
    assert list(ids[0]) == list(range(1, 16)) and list(hops[0]) == [1] * 15
    assert list(ids[7]) == [0] + [1, 2, 3, 4, 5, 6] + list(range(8, 16)) and list(hops[7]) == [1] + [2] * 14
    ids, hops, _ = O.knn_build(G.complete(30), 15)
    for v in (0, 13, 29):
        assert list(ids[v]) == [u for u in range(30) if u != v][:15]
    g = G.er(2048, 1.0 / 8.0, 77)         # diameter 2: kNN = 15 smallest neighbours
    ids, hops, _ = O.knn_build(g, 15, sources=np.arange(0, 2048, 97))
    for r, s in enumerate(range(0, 2048, 97)):
        assert list(ids[r]) == list(g.neighbors(s)[:15]) and list(hops[r]) == [1] * 15


def test_knn_invariants_against_networkx():
    """Sorted, distinct, not self, hops are true distances, complete below the
    last level, minimal ids at the last level -- distances from networkx."""
    for i in range(40):
        g = G.tiny_random(30 + i, [0.04, 0.08, 0.15][i % 3], 3000 + i)
        k = [1, 2, 5, 15, 40][i % 5]
        ids, hops, _ = O.knn_build(g, k)
        pids, phops = O.knn_partial(g, k)
        assert np.array_equal(ids, pids) and np.array_equal(hops, phops)
        ref = dict(nx.all_pairs_shortest_path_length(to_nx(g)))
        for s in range(g.n):
            row = np.full(g.n, 255)
            for t, d in ref[s].items():
                row[t] = d
            e_ids, e_hops = knn_from_dist(row, s, k)
            assert np.array_equal(ids[s], e_ids) and np.array_equal(hops[s], e_hops)
            valid = ids[s] >= 0
            vi = ids[s][valid]
            assert s not in vi and len(set(vi)) == len(vi)
            assert all(row[v] == h for v, h in zip(vi, hops[s][valid]))
            if valid.all():
                hl = hops[s][-1]
                inside = set(np.nonzero((row < hl) & (np.arange(g.n) != s))[0])
                assert inside <= set(vi)
                chosen_last = [v for v, h in zip(vi, hops[s]) if h == hl]
                others = [v for v in np.nonzero(row == hl)[0] if v not in chosen_last]
                assert not others or min(others) > max(chosen_last)


# ------------------------------------------ P-eq and the k-nearest definition

def k_nearest_hops(g, k, v):
    """The hops of the k nearest other vertices of v (Sec. 3.3.1: the search
    stops once k other vertices are reached), from the definition: the k
    smallest shortest-path distances from v to the other vertices it reaches,
    whatever the tie order.  Distances come from networkx, not from the
    oracle's BFS."""
    nxg = nx.Graph()
    nxg.add_nodes_from(range(g.n))
    for u in range(g.n):
        for w in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
            if int(w) != u:
                nxg.add_edge(u, int(w))
    dist = nx.single_source_shortest_path_length(nxg, v)
    return sorted(d for u, d in dist.items() if u != v)[:k]


def test_partial_equals_build_and_definition_multisets():
    gs = [G.ba(800, 3, 21), G.rgg(800, 6, 22), G.sbm(800, 6, 23), G.grid_2d(15, 20),
          G.star(25), G.disjoint_union([G.path(4), G.cycle(7), G.complete(3), G.empty(2)])]
    for g in gs:
        for k in (1, 4, 15, 30):
            ids, hops, _ = O.knn_build(g, k)
            pids, phops = O.knn_partial(g, k)
            assert np.array_equal(ids, pids) and np.array_equal(hops, phops)
            for v in range(0, g.n, max(1, g.n // 60)):
                ms = k_nearest_hops(g, k, v)
                got = sorted(int(h) for h in phops[v] if h != 255)
                assert got == ms, (g.name, k, v)


def test_partial_on_dirty_input_equals_clean():
    g = G.ba(500, 3, 41)
    d = G.dirty(g, 42)
    for k in (3, 15):
        a = O.knn_partial(g, k)
        b = O.knn_partial(d, k)
        c = O.knn_build(d, k)[:2]
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert np.array_equal(a[0], c[0]) and np.array_equal(a[1], c[1])


def test_padding_small_components_and_isolated():
    g = G.disjoint_union([G.path(3), G.empty(1), G.complete(5)])
    ids, hops, _ = O.knn_build(g, 6)
    assert list(ids[0]) == [1, 2, -1, -1, -1, -1] and list(hops[0]) == [1, 2, 255, 255, 255, 255]
    assert list(ids[3]) == [-1] * 6 and list(hops[3]) == [255] * 6
    assert list(ids[4]) == [5, 6, 7, 8, -1, -1]
    pids, phops = O.knn_partial(g, 6)
    assert np.array_equal(ids, pids) and np.array_equal(hops, phops)
    ids, hops, _ = O.knn_build(G.path(1), 4)
    assert list(ids[0]) == [-1] * 4


# ------------------------------------------------------- membership pins

def _poly_root(row, k):
    """Root in (0, 1) of sum_h c_h x^h = log2 k (companion-matrix eigenvalues)."""
    h = np.array([x for x in row if x != 255], dtype=np.int64)
    d = h - h[0]
    c = np.bincount(d).astype(np.float64)
    coeffs = c[::-1].copy()
    coeffs[-1] -= math.log2(k)
    roots = np.roots(coeffs)
    real = [r.real for r in roots if abs(r.imag) < 1e-9 and 0 < r.real < 1]
    assert len(real) == 1
    return real[0]


def test_membership_matches_polynomial_roots():
    rng = np.random.default_rng(5)
    rows = []
    for k in (5, 10, 15, 30, 100, 254):
        for _ in range(60):
            K = int(rng.integers(1, k + 1))
            inc = rng.integers(0, 3, size=K)
            inc[0] = rng.integers(1, 3)
            h = np.minimum(np.cumsum(inc), 250).astype(np.uint8)
            rows.append((k, np.concatenate([h, np.full(k - K, 255, np.uint8)])))
    checked = 0
    for k, row in rows:
        w, rho, sigma = O.membership(row[None, :], k)
        K = int((row != 255).sum())
        T = math.log2(k)
        c0 = int((row[:K] == row[0]).sum())
        assert rho[0] == float(row[0])
        if c0 >= T:
            assert sigma[0] == 0.0
            assert list(w[0][:K]) == [1.0 if x == row[0] else 0.0 for x in row[:K]]
        elif K <= T:
            assert math.isinf(sigma[0]) and np.all(w[0][:K] == 1.0)
        else:
            x = _poly_root(row, k)
            assert abs(math.exp(-1.0 / float(sigma[0])) - x) <= 1e-6 * x + 1e-12
            d = row[:K].astype(np.float64) - row[0]
            ref = x ** d
            assert np.all(np.abs(w[0][:K] - ref) <= 1e-6 * ref + 1e-30)
            assert w[0][0] == 1.0
            # sum equals log2 k to double precision before the float cast
            sig64 = -1.0 / math.log(x)
            assert abs(np.exp(-d / sig64).sum() - T) < 1e-12
            checked += 1
        assert np.all(w[0][K:] == 0.0)
    assert checked > 50


def test_membership_closed_form_bandwidths():
    T = math.log2(15)
    g = G.grid_2d(32, 32)
    ids, hops, _ = O.knn_build(g, 15)
    w, rho, sigma = O.membership(hops)
    xb = (-5 + math.sqrt(25 + 28 * (T - 3))) / 14          # 3 + 5x + 7x^2 = log2 15
    s = 9                                                 # boundary row (0, 9)
    assert abs(sigma[s] - (-1 / math.log(xb))) < 1e-6
    assert np.allclose(w[s], [1] * 3 + [xb] * 5 + [xb * xb] * 7, rtol=1e-6)
    corner = np.roots([1, 5, 4, 3, 2 - T])              # 2 + 3x + 4x^2 + 5x^3 + x^4
    xc = [r.real for r in corner if abs(r.imag) < 1e-12 and 0 < r.real < 1][0]
    assert abs(xc - 0.367225) < 1e-6
    assert abs(math.exp(-1 / sigma[0]) - xc) < 1e-6
    interior = 32 * 10 + 17                              # 4 at hop 1 >= log2 15: degenerate
    assert sigma[interior] == 0 and list(w[interior]) == [1.0] * 4 + [0.0] * 11
    ids, hops, _ = O.knn_build(G.star(40), 15)           # leaf: 1 + 14x = log2 15
    w, rho, sigma = O.membership(hops)
    xs = (T - 1) / 14
    assert abs(sigma[5] - (-1 / math.log(xs))) < 1e-6
    assert sigma[0] == 0 and np.all(w[0] == 1.0)           # hub: 15 at hop 1
    # path endpoint: geometric series (1 - x^15)/(1 - x) = log2 15
    ids, hops, _ = O.knn_build(G.path(40), 15)
    w, rho, sigma = O.membership(hops)
    x = math.exp(-1 / float(sigma[0]))
    assert abs((1 - x**15) / (1 - x) - T) < 1e-5


def test_membership_degenerate_and_empty_rows():
    rows = np.array([[255] * 4, [1, 1, 2, 2], [1, 2, 255, 255], [3, 3, 3, 3]], dtype=np.uint8)
    w, rho, sigma = O.membership(rows)
    assert list(w[0]) == [0] * 4 and rho[0] == 0 and sigma[0] == 0
    assert list(w[1]) == [1, 1, 0, 0] and sigma[1] == 0              # c0 = 2 >= log2 4
    assert list(w[2]) == [1, 1, 0, 0] and math.isinf(sigma[2])        # K = 2 <= 2
    assert list(w[3]) == [1, 1, 1, 1] and rho[3] == 3 and sigma[3] == 0


# ------------------------------------------------------------ golden pin

def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = [float(x) for x in rest]
    return vals


def test_hand_worked_example():
    gv = _golden("hand_worked_7v.txt")
    e = np.array(gv["edges"], dtype=np.int64).reshape(-1, 2)
    g = G.from_edges(7, e)
    s = int(gv["source"][0])
    for k in (3, 4, 5, 8):
        ids, hops, _ = O.knn_build(g, k, sources=[s])
        pids, phops = O.knn_partial(g, k, sources=[s])
        assert list(ids[0]) == [int(x) for x in gv["k%d_ids" % k]]
        assert list(hops[0]) == [int(x) for x in gv["k%d_hops" % k]]
        assert np.array_equal(ids, pids) and np.array_equal(hops, phops)
        if "k%d_sigma" % k in gv:
            w, rho, sigma = O.membership(hops, k)
            assert rho[0] == 1.0
            assert abs(sigma[0] - gv["k%d_sigma" % k][0]) <= 1e-6 * max(1.0, gv["k%d_sigma" % k][0])
            assert np.allclose(w[0], gv["k%d_weights" % k], rtol=1e-6, atol=0)


# ----------------------------------------------------- stress (Sec. 4.1.3) --

def _line_layout(n, scale=1.0):
    return np.stack([scale * np.arange(n), np.zeros(n)], 1).astype(np.float32)


@pytest.mark.parametrize("c", [1.0, 2.0, 0.5, 0.25])
def test_stress_scaled_path_closed_form(c):
    """A path drawn on a line with spacing c: every pair contributes
    ((d - c d) / d)^2 = (1 - c)^2, over all n(n-1) ordered pairs."""
    n = 37
    s, pairs = O.stress(G.path(n), _line_layout(n, c))
    assert pairs == n * (n - 1)
    assert s == pytest.approx((1 - c) ** 2 * pairs, rel=1e-12, abs=1e-12)


def test_stress_collapsed_complete_graph():
    """Every vertex at one point: each pair at hop 1 contributes 1."""
    n = 12
    s, pairs = O.stress(G.complete(n), np.zeros((n, 2), dtype=np.float32))
    assert pairs == n * (n - 1) and s == pytest.approx(pairs, rel=1e-15)


def test_stress_grid_in_its_own_coordinates():
    """Grid drawn at its lattice points: hop distance |dx| + |dy| against the
    Euclidean sqrt(dx^2 + dy^2), summed over the (w - |dx|)(h - |dy|) ordered
    pairs with each offset."""
    w, h = 9, 6
    g = G.grid_2d(h, w)   # h rows of w columns, id = row * w + column
    xy = np.array([[v % w, v // w] for v in range(g.n)], dtype=np.float32)
    expect = 0.0
    for dx in range(-(w - 1), w):
        for dy in range(-(h - 1), h):
            if dx == 0 and dy == 0:
                continue
            d = abs(dx) + abs(dy)
            e = math.hypot(dx, dy)
            expect += (w - abs(dx)) * (h - abs(dy)) * ((d - e) / d) ** 2
    s, pairs = O.stress(g, xy)
    assert pairs == g.n * (g.n - 1)
    assert s == pytest.approx(expect, rel=1e-12)


def test_stress_disconnected_pairs_and_sources():
    """Only connected pairs count; a source subset sums its own rows."""
    a, b = G.path(7), G.cycle(5)
    g = G.disjoint_union([a, b])
    rng = np.random.default_rng(3)
    xy = rng.normal(size=(g.n, 2)).astype(np.float32)
    s, pairs = O.stress(g, xy)
    sa, pa = O.stress(a, xy[:7])
    sb, pb = O.stress(b, xy[7:])
    assert pairs == 7 * 6 + 5 * 4 == pa + pb
    assert s == pytest.approx(sa + sb, rel=1e-12)
    rows, rpairs = O.stress_rows(g, xy)
    src = np.array([0, 3, 9, 3], dtype=np.int32)
    s2, p2 = O.stress(g, xy, sources=src)
    assert p2 == int(rpairs[src].sum()) and s2 == pytest.approx(float(rows[src].sum()), rel=1e-12)


def test_stress_brute_force_tiny_graphs():
    """Floyd-Warshall distances and the metric written out pair by pair."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import shortest_path
    for seed in range(5):
        g = G.tiny_random(14, 0.25, seed)
        rng = np.random.default_rng(100 + seed)
        xy = (rng.random((g.n, 2)) * 5).astype(np.float32)
        adj = csr_matrix((np.ones(len(g.col_idx)), g.col_idx, g.row_ptr), shape=(g.n, g.n))
        d = shortest_path(adj, unweighted=True, directed=False)
        tot, cnt = 0.0, 0
        for i in range(g.n):
            for j in range(g.n):
                if i != j and np.isfinite(d[i, j]):
                    e = math.dist(xy[i].astype(np.float64), xy[j].astype(np.float64))
                    tot += ((d[i, j] - e) / d[i, j]) ** 2
                    cnt += 1
        s, pairs = O.stress(g, xy)
        assert pairs == cnt and s == pytest.approx(tot, rel=1e-12, abs=1e-12)


# ---------------------------------------- neighbourhood preservation (Sec. 4.1.3) --

def test_neighborhood_line_and_lattice_drawings_score_one():
    """A path on a line and a grid at its lattice points keep every graph ball
    (r = 1, 2) as the nearest points of the drawing, ties included whole."""
    n = 23
    s, c = O.neighborhood_preservation(G.path(n), np.stack([np.arange(n), np.zeros(n)], 1))
    assert (s, c) == (float(n), n)
    g = G.grid_2d(7, 11)
    xy = np.array([[v % 11, v // 11] for v in range(g.n)], dtype=np.float32)
    for r in (1, 2):
        score, ball = O.neighborhood_scores(g, xy, r)
        assert np.all(score == 1.0)
        assert ball.max() == (4 if r == 1 else 12)


def test_neighborhood_collapsed_cycle_tie_rule():
    """Every vertex of C_n at one point: all distances tie, so N_D(v) is the K
    smallest ids other than v; the score follows from the two sets."""
    n = 12
    score, ball = O.neighborhood_scores(G.cycle(n), np.zeros((n, 2), dtype=np.float32), 2)
    for v in range(n):
        ng = {(v + d) % n for d in (-2, -1, 1, 2)}
        nd = set([u for u in range(n) if u != v][:4])
        assert ball[v] == 4
        assert score[v] == len(ng & nd) / len(ng | nd)


def test_neighborhood_isolated_vertices_undefined():
    g = G.disjoint_union([G.path(4), G.empty(3)])
    xy = np.random.default_rng(0).random((g.n, 2)).astype(np.float32)
    score, ball = O.neighborhood_scores(g, xy)
    assert np.all(np.isnan(score[4:])) and np.all(ball[4:] == 0)
    s, c = O.neighborhood_preservation(g, xy)
    assert c == 4 and s == pytest.approx(float(score[:4].sum()))
    sub, subball = O.neighborhood_scores(g, xy, vertices=[2, 5, 2])
    assert np.array_equal(subball, ball[[2, 5, 2]]) and sub[0] == score[2] and sub[2] == score[2]


def test_neighborhood_brute_force_tiny_graphs():
    """networkx balls and a lexicographic sort of (squared distance, id)."""
    for seed in range(6):
        g = G.tiny_random(25, 0.12, 300 + seed)
        rng = np.random.default_rng(400 + seed)
        xy = np.round(rng.random((g.n, 2)) * 4).astype(np.float32)   # many exact ties
        nxg = to_nx(g)
        score, ball = O.neighborhood_scores(g, xy, 2)
        for v in range(g.n):
            ng = set(nx.single_source_shortest_path_length(nxg, v, cutoff=2)) - {v}
            assert ball[v] == len(ng)
            if not ng:
                assert np.isnan(score[v])
                continue
            others = np.array([u for u in range(g.n) if u != v])
            d2 = ((xy[others].astype(np.float64) - xy[v].astype(np.float64)) ** 2).sum(1)
            order = np.lexsort((others, d2))
            nd = set(others[order[:len(ng)]].tolist())
            assert score[v] == len(ng & nd) / len(ng | nd)
