"""GPU parity: the HIP path (through the C-ABI) against the CPU oracle.

Bit-exact on neighbour ids, hops and hop matrices; weights within 1e-5
relative (2^-126 absolute floor), rho bit-exact, sigma within 1e-5.
"""
import os
import sys

import numpy as np
import pytest

import graphgen as G
import oracle as O

sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import assert_weights_close, first_mismatch, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _graphs_small():
    return [
        ("grid32", G.grid_2d(32, 32)),
        ("ba2000", G.ba(2000, 4, 11)),
        ("rgg2000", G.rgg(2000, 8, 12)),
        ("sbm2000", G.sbm(2000, 12, 13)),
        ("er600", G.er(600, 0.1, 14)),
        ("star300", G.star(300)),
        ("complete40", G.complete(40)),
        ("path200", G.path(200)),
        ("union", G.disjoint_union([G.path(5), G.complete(4), G.empty(3), G.cycle(9), G.star(20)])),
        ("hypercube8", G.hypercube(8)),
        ("single", G.empty(1)),
    ]


def _check_build(gm, g, k, sources=None, hop_matrix=True, flags=0, dirty=False):
    import torch
    gi = G.dirty(g, 99) if dirty else g
    rp, ci = to_dev(gi)
    src_t = None if sources is None else torch.from_numpy(np.asarray(sources, np.int32)).cuda()
    print("build n=%d k=%d rows=%s hm=%s flags=%d" % (g.n, k, "all" if sources is None else len(sources),
                                                       hop_matrix, flags), flush=True)
    ids, hops, hm = gm.knn_build(rp, ci, k, sources=src_t, hop_matrix=hop_matrix,
                                 flags=flags | (0 if dirty else gm.CSR_SORTED))
    oi, oh, ohm = O.knn_build(g, k, sources=sources, hop_matrix=hop_matrix)
    assert np.array_equal(ids.cpu().numpy(), oi), first_mismatch(ids.cpu().numpy(), oi)
    assert np.array_equal(hops.cpu().numpy(), oh), first_mismatch(hops.cpu().numpy(), oh)
    if hop_matrix:
        assert np.array_equal(hm.cpu().numpy(), ohm), first_mismatch(hm.cpu().numpy(), ohm)
    return oi, oh


@pytest.mark.parametrize("name,g", _graphs_small(), ids=[n for n, _ in _graphs_small()])
def test_build_all_sources_small(gumap, name, g):
    _check_build(gumap, g, 15)


@pytest.mark.parametrize("name,g", _graphs_small(), ids=[n for n, _ in _graphs_small()])
def test_partial_and_membership_small(gumap, name, g):
    rp, ci = to_dev(g)
    for k in (1, 15, 30):
        print("partial", name, k, flush=True)
        ids, hops = gumap.knn_partial(rp, ci, k, flags=gumap.CSR_SORTED)
        oi, oh = O.knn_partial(g, k)
        assert np.array_equal(ids.cpu().numpy(), oi), first_mismatch(ids.cpu().numpy(), oi)
        assert np.array_equal(hops.cpu().numpy(), oh)
        w, rho, sigma = gumap.membership(hops)
        ow, orho, osig = O.membership(oh)
        assert_weights_close(w.cpu().numpy(), ow, rho.cpu().numpy(), orho, sigma.cpu().numpy(), osig)


@pytest.mark.parametrize("k", [1, 2, 7, 16, 17, 30, 63, 64, 100, 254])
def test_k_range(gumap, k):
    g = G.ba(1500, 3, 21)
    _check_build(gumap, g, k, hop_matrix=False)
    rp, ci = to_dev(g)
    ids, hops = gumap.knn_partial(rp, ci, k, flags=gumap.CSR_SORTED)
    oi, oh = O.knn_partial(g, k)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)
    w, rho, sigma = gumap.membership(hops)
    ow, orho, osig = O.membership(oh)
    assert_weights_close(w.cpu().numpy(), ow, rho.cpu().numpy(), orho, sigma.cpu().numpy(), osig)


@pytest.mark.parametrize("words", [1, 2, 4, 8])
def test_bitset_width_invariance(gumap, words, monkeypatch):
    monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
    for g in (G.rgg(3000, 6, 31), G.grid_2d(20, 37)):
        _check_build(gumap, g, 15, hop_matrix=True)
        src = G.sample_sources(g.n, 700, 32)
        _check_build(gumap, g, 10, sources=src, hop_matrix=False)


@pytest.mark.parametrize("verts,first", [(1, "1"), (2, "1"), (4, "1"), (8, "1"), (1, "0"), (4, "0")])
def test_level_items_per_thread_invariance(gumap, verts, first, monkeypatch):
    """The per-level BFS gives the oracle's rows whether a thread of its
    level kernel takes 1, 2, 4 or 8 (vertex, word) items, and whether level 1
    runs as a fill plus a scatter from the sources or as a range scan in the
    level kernel: ragged vertex counts, hub vertices searched by whole waves,
    every bitset width."""
    monkeypatch.setenv("GUMAP_FUSED", "0")
    monkeypatch.setenv("GUMAP_LEVEL_VERTS", str(verts))
    monkeypatch.setenv("GUMAP_FIRST_LEVEL", first)
    print("level items per thread %d, first level split %s" % (verts, first), flush=True)
    for g, words in ((G.ba(4099, 4, 33), 8), (G.ba(2051, 6, 34), 2), (G.rgg(1777, 6, 35), 1), (G.star(1025), 4)):
        monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
        _check_build(gumap, g, 15, hop_matrix=True)
        src = G.sample_sources(g.n, 333, 36)
        _check_build(gumap, g, 7, sources=src, hop_matrix=False)


@pytest.mark.parametrize("hist", ["0", "1", "3", "15"])
def test_frontier_history_depth_invariance(gumap, hist, monkeypatch):
    """The hop rows are the oracle's whether hops 1..H are rebuilt from the
    kept frontiers (H = 1, 3, 15) or every hop goes to the bit-planes
    (H = 0): graphs whose depth is below, at and far above H (a path of
    depth 249, a grid of depth 55), truncated searches that end at k, and
    the stress terms that read the same hop rows."""
    import torch
    monkeypatch.setenv("GUMAP_FUSED", "0")
    monkeypatch.setenv("GUMAP_HIST_LEVELS", hist)
    print("frontier history levels %s" % hist, flush=True)
    for g, words in ((G.path(250), 1), (G.grid_2d(20, 37), 2), (G.ba(3001, 3, 61), 8), (G.star(700), 4)):
        monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
        _check_build(gumap, g, 15, hop_matrix=True)
        src = G.sample_sources(g.n, 257, 62)
        _check_build(gumap, g, 3, sources=src, hop_matrix=False)
        _check_build(gumap, g, 17, sources=src, hop_matrix=True)
    g = G.grid_2d(24, 29)
    xy = np.random.default_rng(63).standard_normal((g.n, 2)).astype(np.float32)
    rp, ci = to_dev(g)
    gs, gp = gumap.stress(rp, ci, torch.from_numpy(xy).cuda(), flags=gumap.CSR_SORTED)
    os_, op = O.stress(g, xy)
    assert gp == op
    assert abs(gs - os_) <= 1e-9 * max(1.0, abs(os_))


@pytest.mark.parametrize("push_levels,ratio,hist,first", [
    ("0", "4", "15", "1"), ("0", "4", "0", "0"), ("2", "4", "15", "0"),
    ("2", "0", "15", "1"), ("3", "0", "15", "1"), ("2", "0", "0", "1"),
    ("3", "4", "15", "1"), ("2", "4", "0", "1")])
def test_direction_invariance(gumap, push_levels, ratio, hist, first, monkeypatch):
    """The hop rows are the oracle's whether levels 2..3 run top-down (every
    group forced with ratio 0, or picked by the frontier edge count) or
    bottom-up, in history and plane mode, with level 1 as a scatter or a
    range scan (which turns the top-down levels off): hub vertices pushed
    in chunks and gathered by whole waves (star, BA), deep graphs, repeated
    sources, truncated searches and every bitset width."""
    monkeypatch.setenv("GUMAP_FUSED", "0")
    monkeypatch.setenv("GUMAP_FIRST_LEVEL", first)
    monkeypatch.setenv("GUMAP_PUSH_LEVELS", push_levels)
    monkeypatch.setenv("GUMAP_PUSH_RATIO", ratio)
    monkeypatch.setenv("GUMAP_HIST_LEVELS", hist)
    print("push levels %s ratio %s history %s first %s" % (push_levels, ratio, hist, first), flush=True)
    for g, words in ((G.ba(3001, 3, 71), 8), (G.star(1500), 4), (G.grid_2d(23, 31), 2), (G.rgg(2500, 7, 72), 1),
                     (G.sbm(2000, 10, 73), 8)):
        monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
        _check_build(gumap, g, 15, hop_matrix=True)
        src = np.concatenate([G.sample_sources(g.n, 300, 74), [0, 0, 7]]).astype(np.int32)
        _check_build(gumap, g, 2, sources=src, hop_matrix=False)
        _check_build(gumap, g, 9, sources=src, hop_matrix=True)


def test_sources_with_repeats_and_order(gumap):
    g = G.sbm(2500, 10, 41)
    src = np.concatenate([G.sample_sources(g.n, 300, 42), [5, 5, 17, 2499, 0, 17]]).astype(np.int32)
    _check_build(gumap, g, 15, sources=src, hop_matrix=True)
    _check_build(gumap, g, 15, sources=src[::-1].copy(), hop_matrix=False)


def test_dirty_input_canonicalised(gumap):
    for g in (G.ba(3000, 5, 51), G.grid_2d(16, 16), G.star(1500), G.complete(70)):
        _check_build(gumap, g, 15, dirty=True, hop_matrix=True)
        d = G.dirty(g, 52)
        rp, ci = to_dev(d)
        ids, hops = gumap.knn_partial(rp, ci, 15)
        oi, oh = O.knn_partial(g, 15)
        assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)


def test_long_rows_canonicalised(gumap):
    # rows above 1,024 and above 32,768 entries go through the workgroup and bitmap paths
    g = G.disjoint_union([G.star(40000), G.star(5000), G.complete(30)])
    d = G.dirty(g, 61)
    rp, ci = to_dev(d)
    ids, hops = gumap.knn_partial(rp, ci, 15, flags=gumap.VALIDATE)
    oi, oh = O.knn_partial(g, 15)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)


def _rows_of_lengths(n, special, seed):
    """CSR input with row v of length special[v] where given (else 0..12),
    entries drawn uniformly from [0, n) with repeats and about one in ten
    replaced by the row's own id (a self-loop).  Symmetry is not needed to
    canonicalise."""
    rng = np.random.default_rng(seed)
    lengths = rng.integers(0, 13, n).astype(np.int64)
    for v, d in special.items():
        lengths[v] = d
    rp = np.zeros(n + 1, np.int64)
    np.cumsum(lengths, out=rp[1:])
    src = np.repeat(np.arange(n, dtype=np.int64), lengths)
    col = rng.integers(0, n, int(rp[-1]))
    loop = rng.random(len(col)) < 0.1
    col[loop] = src[loop]
    return rp.astype(np.int32), col.astype(np.int32)


def _canonical_by_definition(n, rp, col):
    """Rows sorted ascending, repeats and the row's own vertex removed."""
    src = np.repeat(np.arange(n, dtype=np.int64), np.diff(rp))
    dst = col.astype(np.int64)
    key = np.unique(src[src != dst] * n + dst[src != dst])
    out_rp = np.zeros(n + 1, np.int64)
    np.cumsum(np.bincount(key // n, minlength=n), out=out_rp[1:])
    return out_rp.astype(np.int32), (key % n).astype(np.int32)


@pytest.mark.parametrize("n", [5000, 300000])
def test_canonicalize_row_lengths(gumap, n):
    """gumap_csr_canonicalize against the definition, with input rows on
    each side of every bound between sorting paths (thread 16/32, wave
    64/256, workgroup 4,096, big-row LDS 32,768), at the lowest ids (where a
    preferential-attachment graph puts its hubs), among them, and at the
    last ids; n = 5,000 sorts every long row through the n-bit set of the
    row kernel, n = 300,000 through the LDS bitonic sort and the big-row
    kernel.  The last tile of rows is ragged in both."""
    import torch
    lengths = (0, 1, 15, 16, 17, 31, 32, 33, 63, 64, 65, 255, 256, 257, 4095, 4096, 4097, 32768, 32769, 50000)
    special = {}
    for i, d in enumerate(lengths):
        special[i] = d                    # lowest ids
        special[n // 2 + 37 * i] = d      # spread
        special[n - 1 - i] = d            # last ids
    rp, col = _rows_of_lengths(n, special, 71 + n)
    print("canonicalize n=%d nnz=%d" % (n, len(col)), flush=True)
    out_rp, out_col = gumap.csr_canonicalize(torch.from_numpy(rp).cuda(), torch.from_numpy(col).cuda())
    want_rp, want_col = _canonical_by_definition(n, rp, col)
    assert np.array_equal(out_rp.cpu().numpy(), want_rp), first_mismatch(out_rp.cpu().numpy(), want_rp)
    assert np.array_equal(out_col.cpu().numpy(), want_col), first_mismatch(out_col.cpu().numpy(), want_col)


def test_canonicalize_degenerate(gumap):
    """Edgeless rows, a graph of self-loops only, and an already canonical
    graph (nothing moves) against the definition."""
    import torch
    cases = [(7, np.zeros(8, np.int32), np.zeros(0, np.int32)),
             (5, np.arange(6, dtype=np.int32), np.arange(5, dtype=np.int32)),
             (G.ba(3000, 4, 72).n, G.ba(3000, 4, 72).row_ptr, G.ba(3000, 4, 72).col_idx)]
    for n, rp, col in cases:
        out_rp, out_col = gumap.csr_canonicalize(torch.from_numpy(np.ascontiguousarray(rp)).cuda(),
                                                 torch.from_numpy(np.ascontiguousarray(col)).cuda())
        want_rp, want_col = _canonical_by_definition(n, rp, col)
        assert np.array_equal(out_rp.cpu().numpy(), want_rp)
        assert np.array_equal(out_col.cpu().numpy(), want_col)


def test_build_in_rounds(gumap, monkeypatch):
    """A BFS memory budget below one source group's state makes every group a
    round of its own: each round reuses the search state, the level counters
    (copied back beside the transpose) and the hop-count buffers.  Rows, hops
    and hop matrices equal the oracle's for all and for listed sources, at
    several bitset widths and depths."""
    monkeypatch.setenv("GUMAP_BFS_BUDGET_MB", "1")
    monkeypatch.setenv("GUMAP_FUSED", "0")
    for g, words in ((G.ba(3001, 4, 31), 8), (G.rgg(2000, 8, 32), 2), (G.path(200), 1)):
        monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
        print("rounds", g.n, words, flush=True)
        _check_build(gumap, g, 15, hop_matrix=True)
        _check_build(gumap, g, 6, sources=G.sample_sources(g.n, 700, 33), hop_matrix=False)


def test_hop_range_error(gumap):
    import torch
    g = G.path(300)
    rp, ci = to_dev(g)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_build(rp, ci, 5, hop_matrix=True, flags=gumap.CSR_SORTED)
    assert e.value.status == gumap.ERANGE
    _check_build(gumap, g, 5, hop_matrix=False)
    _check_build(gumap, G.path(255), 5, hop_matrix=True)
    torch.cuda.synchronize()


def test_validation_errors(gumap):
    import torch
    dev = "cuda"
    # asymmetric: 0 -> 1 only
    rp = torch.tensor([0, 1, 1], dtype=torch.int32, device=dev)
    ci = torch.tensor([1], dtype=torch.int32, device=dev)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_partial(rp, ci, 3, flags=gumap.VALIDATE)
    assert e.value.status == gumap.EGRAPH
    # id out of range
    rp = torch.tensor([0, 1, 2], dtype=torch.int32, device=dev)
    ci = torch.tensor([1, 7], dtype=torch.int32, device=dev)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_build(rp, ci, 3, flags=gumap.VALIDATE)
    assert e.value.status == gumap.EGRAPH
    # row_ptr not monotone
    rp = torch.tensor([0, 2, 1, 2], dtype=torch.int32, device=dev)
    ci = torch.tensor([1, 2], dtype=torch.int32, device=dev)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_partial(rp, ci, 3, flags=gumap.VALIDATE)
    assert e.value.status == gumap.EGRAPH
    # claims sorted but is not
    g = G.dirty(G.grid_2d(5, 5), 3)
    rp, ci = to_dev(g)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_partial(rp, ci, 3, flags=gumap.VALIDATE | gumap.CSR_SORTED)
    assert e.value.status == gumap.EGRAPH
    # bad source id
    g = G.grid_2d(5, 5)
    rp, ci = to_dev(g)
    with pytest.raises(gumap.GumapError) as e:
        gumap.knn_build(rp, ci, 3, sources=torch.tensor([0, 25], dtype=torch.int32, device=dev))
    assert e.value.status == gumap.EINVAL
    # the library keeps working after errors
    _check_build(gumap, g, 4)


def test_ba100k_full_partial_and_sampled_build(gumap):
    """The BA workload at full size: partial BFS from all 100,000 vertices and
    the all-source BFS from the 4,096 sampled sources, against the oracle."""
    g = G.config_ba()
    src = G.config_ba_sources()
    rp, ci = to_dev(g)
    import torch
    print("ba100k partial", flush=True)
    ids, hops = gumap.knn_partial(rp, ci, 15, flags=gumap.CSR_SORTED)
    oi, oh = O.knn_partial(g, 15)
    assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)
    w, rho, sigma = gumap.membership(hops)
    ow, orho, osig = O.membership(oh)
    assert_weights_close(w.cpu().numpy(), ow, rho.cpu().numpy(), orho, sigma.cpu().numpy(), osig)
    print("ba100k build", flush=True)
    src_t = torch.from_numpy(src).cuda()
    bids, bhops, hm = gumap.knn_build(rp, ci, 15, sources=src_t, hop_matrix=True, flags=gumap.CSR_SORTED)
    assert np.array_equal(bids.cpu().numpy(), oi[src]) and np.array_equal(bhops.cpu().numpy(), oh[src])
    pick = np.arange(0, len(src), 64)
    _, _, ohm = O.knn_build(g, 15, sources=src[pick], hop_matrix=True)
    assert np.array_equal(hm[torch.from_numpy(pick).cuda()].cpu().numpy(), ohm)


def test_er16k_all_sources_closed_form(gumap):
    """Dense ER workload at full size: diameter 2, so every hop row is 1 on the
    adjacency and 2 elsewhere, and the kNN row is the first 15 neighbours."""
    import torch
    g = G.config_er()
    rp, ci = to_dev(g)
    print("er16k build", flush=True)
    ids, hops, hm = gumap.knn_build(rp, ci, 15, hop_matrix=True, flags=gumap.CSR_SORTED)
    n = g.n
    deg = g.degrees()
    # closed form per row, checked on the device to keep host memory small
    adj = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
    src = torch.from_numpy(np.repeat(np.arange(n), deg)).cuda().long()
    dst = torch.from_numpy(g.col_idx).cuda().long()
    adj[src, dst] = 1
    expect = 2 - adj
    expect.fill_diagonal_(0)
    assert torch.equal(hm, expect)
    first15 = np.stack([g.neighbors(v)[:15] for v in range(n)])
    assert np.array_equal(ids.cpu().numpy(), first15)
    assert np.all(hops.cpu().numpy() == 1)
    pick = G.sample_sources(n, 32, 71)
    oi, oh, ohm = O.knn_build(g, 15, sources=pick, hop_matrix=True)
    assert np.array_equal(hm[torch.from_numpy(pick).cuda().long()].cpu().numpy(), ohm)
    w, rho, sigma = gumap.membership(hops)
    assert torch.all(w == 1.0) and torch.all(sigma == 0.0)


def test_build_equals_partial(gumap):
    for g in (G.ba(4000, 4, 81), G.rgg(4000, 10, 82), G.grid_2d(40, 40)):
        rp, ci = to_dev(g)
        for k in (5, 15, 40):
            ids, hops, _ = gumap.knn_build(rp, ci, k, flags=gumap.CSR_SORTED)
            pids, phops = gumap.knn_partial(rp, ci, k, flags=gumap.CSR_SORTED)
            assert np.array_equal(ids.cpu().numpy(), pids.cpu().numpy())
            assert np.array_equal(hops.cpu().numpy(), phops.cpu().numpy())


@pytest.mark.parametrize("lanes", ["0", "16", "32", "64"])
def test_partial_lane_width_invariance(gumap, lanes, monkeypatch):
    """The register-resident search (16/32/64 lanes per source) and the
    one-wave LDS form give identical rows."""
    monkeypatch.setenv("GUMAP_PARTIAL_LANES", lanes)
    for g in (G.ba(3000, 4, 91), G.rgg(3000, 7, 92), G.star(600),
              G.disjoint_union([G.path(3), G.empty(2), G.complete(20)])):
        rp, ci = to_dev(g)
        for k in (1, 5, 15, 31, 63):
            ids, hops = gumap.knn_partial(rp, ci, k, flags=gumap.CSR_SORTED)
            oi, oh = O.knn_partial(g, k)
            assert np.array_equal(ids.cpu().numpy(), oi), (lanes, k, first_mismatch(ids.cpu().numpy(), oi))
            assert np.array_equal(hops.cpu().numpy(), oh)


def _synthetic_hop_rows(rows, k, seed):
    """Sorted hop rows with 255 padding: the valid count K, rho and the spread
    of levels above rho vary per row (spreads past 16 levels included)."""
    rng = np.random.default_rng(seed)
    out = np.full((rows, k), 255, dtype=np.uint8)
    for r in range(rows):
        K = int(rng.integers(0, k + 1)) if r % 4 else k
        rho = int(rng.integers(1, 4))
        p_step = (0.05, 0.2, 0.5, 0.9)[r % 4]
        if K == 0:
            continue
        steps = rng.random(K) < p_step
        steps[0] = False
        h = rho + np.cumsum(steps)
        out[r, :K] = np.minimum(h, 254)
    return out


@pytest.mark.parametrize("k", [2, 3, 10, 15, 16, 30, 64, 100, 254])
def test_membership_synthetic_rows(gumap, k):
    """Membership of rows of every shape (degenerate low and high, narrow and
    wide level spreads, padding) against the oracle's bisection."""
    import torch
    oh = _synthetic_hop_rows(3000, k, 900 + k)
    hops = torch.from_numpy(oh).cuda()
    w, rho, sigma = gumap.membership(hops)
    ow, orho, osig = O.membership(oh)
    assert_weights_close(w.cpu().numpy(), ow, rho.cpu().numpy(), orho, sigma.cpu().numpy(), osig)


@pytest.mark.parametrize("name,g", [("grid", G.grid_2d(40, 37)), ("ba", G.ba(3000, 3, 95)),
                                    ("union", G.disjoint_union([G.path(90), G.star(30), G.empty(4)]))])
def test_fused_small_graph_path_equals_per_level(gumap, monkeypatch, name, g):
    """The one-launch small-graph BFS and the per-level launches give the
    same rows and hop matrices (with and without the hop cap of k)."""
    import torch
    rp, ci = to_dev(g)
    src = torch.from_numpy(G.sample_sources(g.n, min(g.n, 700), 96)).cuda()
    out = {}
    for fused in ("1", "0"):
        monkeypatch.setenv("GUMAP_FUSED", fused)
        a = gumap.knn_build(rp, ci, 15, hop_matrix=True, flags=gumap.CSR_SORTED)
        b = gumap.knn_build(rp, ci, 6, sources=src, hop_matrix=False, flags=gumap.CSR_SORTED)
        out[fused] = [t.cpu().numpy() for t in a if t is not None] + [t.cpu().numpy() for t in b[:2]]
    for x, y in zip(out["1"], out["0"]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("n,fused", [(300, "1"), (300, "0"), (7000, "1")])
def test_hop_range_error_both_paths(gumap, monkeypatch, n, fused):
    """A hop above 254 in a requested hop matrix is ERANGE on the one-launch
    path (n = 300), the per-level path (forced off, and n = 7000 above the
    one-launch LDS limit)."""
    import torch
    monkeypatch.setenv("GUMAP_FUSED", fused)
    g = G.path(n)
    rp, ci = to_dev(g)
    src = None if n < 1000 else torch.arange(8, dtype=torch.int32).cuda()
    print("range n=%d fused=%s" % (n, fused), flush=True)
    with pytest.raises(gumap.GumapError) as ei:
        gumap.knn_build(rp, ci, 3, sources=src, hop_matrix=True, flags=gumap.CSR_SORTED)
    assert ei.value.status == gumap.ERANGE


@pytest.mark.parametrize("rows", [1, 2, 1023, 1024, 1025, 4096, 4097, 9000])
def test_listed_sources_ranking_both_paths(gumap, rows):
    """Listed sources with repeats in any order: up to 4,096 rows are ranked
    by one workgroup, more by the scan path; both give the oracle's rows
    (repeated sources copy their first row)."""
    g = G.ba(3000, 3, 401)
    rng = np.random.default_rng(rows)
    src = rng.integers(0, g.n, rows).astype(np.int32)
    if rows > 4:
        src[rows // 2] = src[0]
        src[-1] = src[1]
    print("ranking rows=%d" % rows, flush=True)
    _check_build(gumap, g, 7, sources=src, hop_matrix=rows <= 1025)


@pytest.mark.parametrize("rows", [3, 4096, 5000])
def test_stress_listed_sources_multiplicity_both_paths(gumap, rows):
    """Stress over listed sources counts a repeated source once per listing,
    on both ranking paths."""
    import torch
    g = G.ba(2500, 3, 402)
    rng = np.random.default_rng(7 + rows)
    src = rng.integers(0, g.n, rows).astype(np.int32)
    src[-1] = src[0]
    xy = rng.uniform(0, 50, (g.n, 2)).astype(np.float32)
    rp, ci = to_dev(g)
    gs, gp = gumap.stress(rp, ci, torch.from_numpy(xy).cuda(), torch.from_numpy(src).cuda(),
                          flags=gumap.CSR_SORTED)
    os_, op = O.stress(g, xy, sources=src)
    assert gp == op and abs(gs - os_) <= 1e-9 * abs(os_)


def test_listed_sources_ranking_large_graph(gumap):
    """More than 131,072 vertices: listed sources take the scan path."""
    g = G.ba(140000, 2, 403)
    src = np.concatenate([G.sample_sources(g.n, 60, 404), [7, 7, 139999]]).astype(np.int32)
    _check_build(gumap, g, 9, sources=src, hop_matrix=False)


def test_profile_only_records_listed_kernels(gumap):
    """gumap_profile_only restricts the launch profiler to the named kernels
    and NULL records all of them again; the rows are unaffected."""
    import torch
    g = G.ba(9000, 4, 61)
    rp, ci = to_dev(g)
    src = torch.from_numpy(G.sample_sources(g.n, 300, 62)).cuda()
    oi, oh, _ = O.knn_build(g, 9, sources=G.sample_sources(g.n, 300, 62), hop_matrix=False)
    try:
        for only, want in ((["knn_select", "msbfs_level"], {"knn_select", "msbfs_level"}), (None, None)):
            gumap.profile_reset()
            gumap.profile_only(only)
            gumap.profile_enable(True)
            ids, hops, _ = gumap.knn_build(rp, ci, 9, sources=src, hop_matrix=False, flags=gumap.CSR_SORTED)
            gumap.profile_enable(False)
            got = set(gumap.profile_entries())
            assert np.array_equal(ids.cpu().numpy(), oi) and np.array_equal(hops.cpu().numpy(), oh)
            if want is not None:
                assert got == want
            else:
                assert {"knn_select", "msbfs_level", "msbfs_hops"} <= got
    finally:
        gumap.profile_enable(False)
        gumap.profile_only(None)
        gumap.profile_reset()
