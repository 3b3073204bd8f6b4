"""GPU parity of the layout step C2 (fuzzy union, edge shuffle, GradSample
of Alg. 5 in Sec. 3.3.2) through the C-ABI, against the CPU oracle on the
same inputs.

Union and shuffle are bit-exact (integer work plus one FP64 expression
evaluated in the same order on both sides).

GradSample is checked two ways.  Against the paper's serial order
(``O.grad_sample``): exactly (up to the 2^-32 grid) on windows whose entries
touch disjoint vertices, where the device's synchronous parts and the serial
order are the same computation; and, at full size (BA n = 100,000, 200
iterations), by the end-of-run cross-entropy cost and neighbourhood
preservation, within tolerances stated at that test.  Against the oracle of
the device's own form (``O.grad_sample_window``, synchronous parts in fixed
point), to check the kernels' arithmetic: both sides evaluate the same FP64
expressions in the same order, so the only source of difference is the last
bit of the power function (the device's and the host's pow may round
differently); such a difference moves a fixed-point step by at most one unit
(2^-32) and a float coordinate by at most one ulp per window, which the
tests allow while requiring nearly all coordinates to agree exactly.
"""
import os
import sys

import numpy as np
import pytest

import graphgen as G
import oracle as O

sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import random_knn, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _knn_inputs(name):
    if name.startswith("rand"):
        k = int(name[4:])
        return random_knn(700, k, k + 40)
    g = {"grid": G.grid_2d(31, 29), "ba": G.ba(3000, 4, 71), "sbm": G.sbm(2500, 10, 72),
         "union": G.disjoint_union([G.path(40), G.star(25), G.empty(5), G.complete(9)])}[name]
    ids, hops = O.knn_partial(g, 15)
    w, _, _ = O.membership(hops)
    return ids, w


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("name", ["grid", "ba", "sbm", "union", "rand7", "rand30", "rand1"])
def test_fuzzy_union_parity(gumap, name):
    ids, w = _knn_inputs(name)
    print("union", name, ids.shape, flush=True)
    rp, col, val = gumap.fuzzy_union(_dev(ids), _dev(w))
    orp, ocol, oval = O.fuzzy_union(ids, w)
    assert np.array_equal(rp.cpu().numpy(), orp)
    assert np.array_equal(col.cpu().numpy(), ocol)
    assert np.array_equal(val.cpu().numpy().view(np.uint32), oval.view(np.uint32))


def test_fuzzy_union_edge_cases(gumap):
    import torch
    # every slot empty: no entries, all row pointers zero
    ids = np.full((50, 4), -1, np.int32)
    rp, col, val = gumap.fuzzy_union(_dev(ids), _dev(np.ones((50, 4), np.float32)))
    assert col.numel() == 0 and int(rp.abs().sum()) == 0
    # all weights zero: nothing kept
    ids, w = random_knn(60, 5, 3)
    rp, col, _ = gumap.fuzzy_union(_dev(ids), _dev(np.zeros_like(w)))
    assert col.numel() == 0
    # capacity too small: ERANGE with the needed count
    ids, w = random_knn(80, 6, 4, zero_frac=0.0)
    need = len(O.fuzzy_union(ids, w)[1])
    rpd = torch.empty(81, dtype=torch.int32, device="cuda")
    cd = torch.empty(need, dtype=torch.int32, device="cuda")
    vd = torch.empty(need, dtype=torch.float32, device="cuda")
    assert gumap.gumap_fuzzy_union(80, 6, _dev(ids), _dev(w), rpd, cd, vd, need) == need
    with pytest.raises(gumap.GumapError) as e:
        gumap.gumap_fuzzy_union(80, 6, _dev(ids), _dev(w), rpd, cd, vd, need - 1)
    assert e.value.status == gumap.ERANGE
    # an id equal to its row, or out of range
    bad = ids.copy()
    bad[3, 0] = 3
    with pytest.raises(gumap.GumapError) as e:
        gumap.fuzzy_union(_dev(bad), _dev(w))
    assert e.value.status == gumap.EINVAL
    bad = ids.copy()
    bad[5, 1] = 80
    with pytest.raises(gumap.GumapError) as e:
        gumap.fuzzy_union(_dev(bad), _dev(w))
    assert e.value.status == gumap.EINVAL


@pytest.mark.parametrize("name,seed", [("grid", 1), ("ba", 2), ("ba", 0xFFFFFFFFFFFFFFFF), ("rand30", 99)])
def test_edge_shuffle_parity(gumap, name, seed):
    ids, w = _knn_inputs(name)
    orp, ocol, oval = O.fuzzy_union(ids, w)
    print("shuffle", name, len(ocol), flush=True)
    head, tail, ws = gumap.edge_shuffle(_dev(orp), _dev(ocol), _dev(oval), seed)
    oh, ot, ow = O.edge_shuffle(orp, ocol, oval, seed)
    assert np.array_equal(head.cpu().numpy(), oh)
    assert np.array_equal(tail.cpu().numpy(), ot)
    assert np.array_equal(ws.cpu().numpy(), ow)


def test_edge_shuffle_checks_count(gumap):
    ids, w = _knn_inputs("grid")
    orp, ocol, oval = O.fuzzy_union(ids, w)
    import torch
    m = len(ocol)
    h = torch.empty(m + 1, dtype=torch.int32, device="cuda")
    with pytest.raises(gumap.GumapError) as e:
        gumap.gumap_edge_shuffle(len(orp) - 1, _dev(orp), _dev(ocol), _dev(oval), m - 1, 1, h, h, h.float())
    assert e.value.status == gumap.EINVAL
    empty = np.zeros(6, np.int32)
    gumap.gumap_edge_shuffle(5, _dev(empty), None, None, 0, 1, None, None, None)


def _layout_case(name, seed=5):
    ids, w = _knn_inputs(name)
    rp, col, val = O.fuzzy_union(ids, w)
    head, tail, ws = O.edge_shuffle(rp, col, val, seed)
    n = ids.shape[0]
    rng = np.random.default_rng(seed)
    xy = rng.uniform(-10, 10, (n, 2)).astype(np.float32)
    return n, head, tail, ws, xy


def _window(n, head, tail, ws, xy, parts=None, **kw):
    """The oracle of the device's form with the library's default parts."""
    import paper_2509_19703_amd as gm
    return O.grad_sample_window(n, head, tail, ws, xy, parts=parts or gm.LAYOUT_DEFAULT_PARTS, **kw)


def _compare_xy(got, ref, windows, what):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    diff = np.abs(got - ref)
    exact = float(np.mean(diff == 0))
    print("%s: exact %.6f max diff %.3g (max ulps %.1f)" % (what, exact, diff.max(), (diff / ulp).max()),
          flush=True)
    assert np.all(diff <= windows * (ulp + 2.0**-26)), what
    assert exact >= 0.99, what


@pytest.mark.parametrize("name", ["grid", "ba", "sbm", "union", "rand7"])
@pytest.mark.parametrize("neg", [0, 5])
def test_grad_sample_one_window(gumap, name, neg):
    n, head, tail, ws, xy = _layout_case(name)
    m = len(head)
    s = int(m ** 0.9)
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, gamma=1.0, alpha0=1.0, window=s, neg=neg, t=50, seed=123)
    for it in (0, 17):
        ref = _window(n, head, tail, ws, xy, it_begin=it, it_end=it + 1, **kw)
        got = _dev(xy.copy())
        gumap.grad_sample(got, _dev(head), _dev(tail), _dev(ws), it_begin=it, it_end=it + 1, **kw)
        _compare_xy(got.cpu().numpy(), ref, 1, "%s neg=%d it=%d" % (name, neg, it))


@pytest.mark.parametrize("parts", [1, 3, 64, 1000000])
def test_grad_sample_parts(gumap, parts):
    """Windows in 1, 3 or 64 synchronous parts, or one entry per part (the
    serial order, parts clamped to the window)."""
    n, head, tail, ws, xy = _layout_case("ba", 6)
    m = len(head)
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, window=int(m ** 0.9), neg=5, t=40, seed=77, it_begin=5, it_end=7)
    ref = _window(n, head, tail, ws, xy, parts=min(parts, kw["window"]), **kw)
    got = _dev(xy.copy())
    gumap.grad_sample(got, _dev(head), _dev(tail), _dev(ws), parts=parts, **kw)
    _compare_xy(got.cpu().numpy(), ref, 2, "parts=%d" % parts)


def _disjoint_case(n, pairs, neg, seed, it):
    """Entries whose vertices no other entry of the window touches, negative
    samples included (the draws of iteration it are computed first)."""
    base = it * pairs
    drawn = {O.splitmix64(seed, (base + l) * neg + q + 1) % n for l in range(pairs) for q in range(neg)}
    free = np.array(sorted(set(range(n)) - drawn))
    rng = np.random.default_rng(seed)
    perm = rng.permutation(free)
    head, tail = perm[:pairs].astype(np.int32), perm[pairs:2 * pairs].astype(np.int32)
    w = rng.uniform(0.2, 1.0, pairs).astype(np.float32)
    xy = rng.uniform(-10, 10, (n, 2)).astype(np.float32)
    return head, tail, w, xy


@pytest.mark.parametrize("neg", [0, 5])
@pytest.mark.parametrize("parts", [1, 4])
def test_grad_sample_disjoint_window_is_serial(gumap, neg, parts):
    """Where no two entries of a window share a vertex, the device computes
    Alg. 5's serial order itself: it agrees with the serial oracle up to the
    fixed-point rounding of the start positions and each move (2^-33 each),
    then the float rounding of the result."""
    n, pairs, seed, it = 200000, 3000, 99, 3
    head, tail, w, xy = _disjoint_case(n, pairs, neg, seed, it)
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, alpha0=1.0, window=pairs, neg=neg, t=10, seed=seed,
              it_begin=it, it_end=it + 1)
    ref = O.grad_sample(n, head, tail, w, xy, **kw).astype(np.float64)
    got = _dev(xy.copy())
    gumap.grad_sample(got, _dev(head), _dev(tail), _dev(w), parts=parts, **kw)
    got = got.cpu().numpy().astype(np.float64)
    ulp = np.spacing(np.abs(ref).astype(np.float32)).astype(np.float64)
    diff = np.abs(got - ref)
    moved = np.zeros(n, bool)
    moved[head] = moved[tail] = True
    print("disjoint neg=%d parts=%d: exact %.6f max diff %.3g" % (neg, parts, np.mean(diff == 0), diff.max()),
          flush=True)
    assert np.all(diff <= ulp + (neg + 2) * 2.0**-33)
    # untouched vertices come back unchanged where the 2^-32 grid holds their
    # float value exactly (magnitude at least 2^-9)
    big = np.abs(xy) >= 2.0**-9
    assert np.array_equal(got[~moved][big[~moved]], xy[~moved][big[~moved]].astype(np.float64))
    assert np.mean(diff[moved] == 0) >= 0.98


@pytest.mark.parametrize("name", ["grid", "ba", "rand30"])
def test_grad_sample_many_windows(gumap, name):
    """A whole t-iteration run in one call (and split over three calls)."""
    n, head, tail, ws, xy = _layout_case(name, 8)
    m = len(head)
    t = 30
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, gamma=1.0, alpha0=1.0, window=int(m ** 0.9), neg=5, t=t, seed=7)
    ref = _window(n, head, tail, ws, xy, **kw)
    got = _dev(xy.copy())
    dh, dt, dw = _dev(head), _dev(tail), _dev(ws)
    gumap.grad_sample(got, dh, dt, dw, **kw)
    _compare_xy(got.cpu().numpy(), ref, t, "%s t=%d one call" % (name, t))
    again = _dev(xy.copy())
    gumap.grad_sample(again, dh, dt, dw, **kw)
    assert np.array_equal(again.cpu().numpy(), got.cpu().numpy())   # deterministic
    ref3 = xy.copy()
    split = _dev(xy.copy())
    for b, e in ((0, 7), (7, 8), (8, t)):
        ref3 = _window(n, head, tail, ws, ref3, it_begin=b, it_end=e, **kw)
        gumap.grad_sample(split, dh, dt, dw, it_begin=b, it_end=e, **kw)
    _compare_xy(split.cpu().numpy(), ref3, t, "%s t=%d three calls" % (name, t))


def test_grad_sample_window_edge_cases(gumap):
    """Window of one edge, window of all edges, a window that wraps, and an
    empty iteration range (a no-op)."""
    n, head, tail, ws, xy = _layout_case("grid", 3)
    m = len(head)
    dh, dt, dw = _dev(head), _dev(tail), _dev(ws)
    for s, t, it in ((1, 5, 3), (m, 4, 2), (m - 3, 10, 7), (m // 3 + 1, 9, 8)):
        kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, window=s, neg=3, t=t, seed=11)
        ref = _window(n, head, tail, ws, xy, it_begin=it, it_end=it + 1, **kw)
        got = _dev(xy.copy())
        gumap.grad_sample(got, dh, dt, dw, it_begin=it, it_end=it + 1, **kw)
        _compare_xy(got.cpu().numpy(), ref, 1, "s=%d it=%d" % (s, it))
    got = _dev(xy.copy())
    gumap.grad_sample(got, dh, dt, dw, it_begin=4, it_end=4, t=9, window=5)
    assert np.array_equal(got.cpu().numpy(), xy)


def test_grad_sample_errors(gumap):
    n, head, tail, ws, xy = _layout_case("grid", 3)
    dh, dt, dw = _dev(head), _dev(tail), _dev(ws)
    bad = head.copy()
    bad[len(bad) // 2] = n
    with pytest.raises(gumap.GumapError) as e:
        gumap.grad_sample(_dev(xy.copy()), _dev(bad), dt, dw, window=10, t=2)
    assert e.value.status == gumap.EINVAL
    far = xy.copy()
    far[7, 1] = 2.0**21
    with pytest.raises(gumap.GumapError) as e:
        gumap.grad_sample(_dev(far), dh, dt, dw, window=10, t=2)
    assert e.value.status == gumap.EINVAL
    with pytest.raises(gumap.GumapError) as e:
        gumap.grad_sample(_dev(xy.copy()), dh, dt, dw, window=len(head) + 1, t=2)
    assert e.value.status == gumap.EINVAL
    # the library still works after the errors
    got = _dev(xy.copy())
    gumap.grad_sample(got, dh, dt, dw, window=10, t=2, it_end=1)
    ref = _window(n, head, tail, ws, xy, a=gumap.UMAP_A, b=gumap.UMAP_B, window=10, neg=5, t=2, seed=0,
                        it_end=1)
    _compare_xy(got.cpu().numpy(), ref, 1, "after errors")


def test_layout_pipeline_ba100k_sampled(gumap):
    """The full-size pipeline of the layout benchmark (BA n = 100,000, k = 15):
    partial kNN, membership, union and shuffle on the device are bit-exact
    against the oracle; the first windows of the run agree to the window
    bound."""
    g = G.config_ba()
    rp, ci = to_dev(g)
    print("layout ba100k", flush=True)
    ids, hops = gumap.knn_partial(rp, ci, 15, flags=gumap.CSR_SORTED)
    w, _, _ = gumap.membership(hops)
    urp, ucol, uval = gumap.fuzzy_union(ids, w)
    oi, oh = O.knn_partial(g, 15)
    ow, _, _ = O.membership(oh)
    orp, ocol, oval = O.fuzzy_union(oi, ow)
    assert np.array_equal(urp.cpu().numpy(), orp) and np.array_equal(ucol.cpu().numpy(), ocol)
    assert np.array_equal(uval.cpu().numpy(), oval)
    head, tail, ws = gumap.edge_shuffle(urp, ucol, uval, 2509)
    oh_, ot_, ow_ = O.edge_shuffle(orp, ocol, oval, 2509)
    assert np.array_equal(head.cpu().numpy(), oh_) and np.array_equal(tail.cpu().numpy(), ot_)
    rng = np.random.default_rng(250919703)
    xy = rng.uniform(-10, 10, (g.n, 2)).astype(np.float32)
    m = len(ocol)
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, window=int(m ** 0.9), neg=5, t=200, seed=17)
    got = _dev(xy.copy())
    gumap.grad_sample(got, head, tail, ws, it_begin=0, it_end=3, **kw)
    ref = _window(g.n, oh_, ot_, ow_, xy, it_begin=0, it_end=3, **kw)
    _compare_xy(got.cpu().numpy(), ref, 3, "ba100k 3 windows")


def test_layout_degenerate_inputs(gumap):
    """One row (k = 1), a kNN with no entries, and edge arrays holding
    self-loops (attraction 0, only negative samples move the head)."""
    import torch
    ids = np.array([[1], [0]], np.int32)
    w = np.array([[0.5], [0.25]], np.float32)
    rp, col, val = gumap.fuzzy_union(_dev(ids), _dev(w))
    orp, ocol, oval = O.fuzzy_union(ids, w)
    assert np.array_equal(rp.cpu().numpy(), orp) and np.array_equal(col.cpu().numpy(), ocol)
    assert np.array_equal(val.cpu().numpy(), oval)
    head = np.array([0, 1, 2, 2], np.int32)
    tail = np.array([0, 3, 2, 1], np.int32)
    ws = np.array([1.0, 0.5, 1.0, 0.75], np.float32)
    xy = np.random.default_rng(4).uniform(-3, 3, (4, 2)).astype(np.float32)
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, window=3, neg=4, t=6, seed=9)
    ref = _window(4, head, tail, ws, xy, **kw)
    got = _dev(xy.copy())
    gumap.grad_sample(got, _dev(head), _dev(tail), _dev(ws), **kw)
    assert np.array_equal(got.cpu().numpy(), ref)
    one = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    gumap.grad_sample(one, _dev(np.zeros(0, np.int32)), _dev(np.zeros(0, np.int32)), _dev(np.zeros(0, np.float32)),
                      window=1, t=3)
    assert float(one.abs().sum()) == 0.0


def _layout_metrics(g, rows, col, val, xy, pairs, verts):
    """End-of-run quality of a drawing: the cross-entropy C of Sec. 2.1 with
    w = 1 / (1 + a d^(2b)), its edge part summed over the union graph and its
    non-edge part (h = 0: -log(1 - w)) estimated from a fixed sample of
    non-adjacent ordered pairs, plus the mean neighbourhood preservation
    (r = 2, Sec. 4.1.3) of the listed vertices (oracle)."""
    import paper_2509_19703_amd as gm
    x = xy.astype(np.float64)
    d2 = ((x[rows] - x[col]) ** 2).sum(1)
    wl = 1.0 / (1.0 + gm.UMAP_A * d2 ** gm.UMAP_B)
    h = val.astype(np.float64)
    tiny = 1e-300
    att = float(np.sum(h * np.log(h / np.maximum(wl, tiny)) +
                       np.where(h < 1.0, (1 - h) * np.log(np.maximum(1 - h, tiny) / np.maximum(1 - wl, tiny)), 0.0)))
    I, J = pairs
    d2n = ((x[I] - x[J]) ** 2).sum(1)
    wn = 1.0 / (1.0 + gm.UMAP_A * d2n ** gm.UMAP_B)
    n = g.n
    rep = float(np.mean(-np.log(np.maximum(1.0 - wn, tiny)))) * (float(n) * (n - 1) - len(col))
    sc, _ = O.neighborhood_scores(g, xy, r=2, vertices=verts)
    return att, rep, float(np.nanmean(sc))


def test_grad_sample_ba100k_run_matches_serial_order(gumap):
    """The layout benchmark's GradSample run at full size (BA n = 100,000,
    k = 15, |E_k| = 799,980, s = floor(|E_k|^0.9), 5 negative samples,
    t = 200, from a seeded uniform drawing) on the device against the serial
    oracle on the same shuffled array and the same negative-sample draws.
    The two trajectories differ (the device applies each window in
    synchronous parts), so the end-of-run drawings are compared by their
    quality.  Tolerances, relative to the serial run: edge part of C 1.5 %,
    non-edge part of C 1.5 %, mean neighbourhood preservation 4 %.  Measured
    on the CPU for this run: three serial runs with different negative-sample
    seeds spread by 0.13 %, 0.18 % and 1.5 %; the whole window applied at
    once (one part) misses the serial run by +2.4 %, -3.0 % and -7 %, so the
    test fails that form; the device with four parts per window (the
    default) measured +0.50 %, -0.57 % and -2.85 %."""
    g = G.config_ba()
    oi, oh = O.knn_partial(g, 15)
    ow, _, _ = O.membership(oh)
    orp, ocol, oval = O.fuzzy_union(oi, ow)
    head, tail, ws = O.edge_shuffle(orp, ocol, oval, 2509)
    rng = np.random.default_rng(250919703)
    xy = rng.uniform(-10, 10, (g.n, 2)).astype(np.float32)
    m = len(ocol)
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, window=int(m ** 0.9), neg=5, t=200, seed=17)
    print("ba100k layout run: device", flush=True)
    got = _dev(xy.copy())
    gumap.grad_sample(got, _dev(head), _dev(tail), _dev(ws), **kw)
    got = got.cpu().numpy()
    print("ba100k layout run: serial oracle", flush=True)
    ref = O.grad_sample(g.n, head, tail, ws, xy, **kw)
    rows = np.repeat(np.arange(g.n), np.diff(orp))
    prng = np.random.default_rng(250919703 + 404)
    I = prng.integers(0, g.n, 2_000_000)
    J = prng.integers(0, g.n, 2_000_000)
    keep = I != J
    I, J = I[keep], J[keep]
    ekey = np.sort(rows.astype(np.int64) * g.n + ocol)
    pk = I.astype(np.int64) * g.n + J
    pos = np.minimum(np.searchsorted(ekey, pk), len(ekey) - 1)
    nonedge = ekey[pos] != pk
    pairs = (I[nonedge], J[nonedge])
    verts = np.sort(np.random.default_rng(250919803).choice(g.n, 4096, replace=False))
    mg = _layout_metrics(g, rows, ocol, oval, got, pairs, verts)
    ms = _layout_metrics(g, rows, ocol, oval, ref, pairs, verts)
    m0 = _layout_metrics(g, rows, ocol, oval, xy, pairs, verts)
    rel = [abs(a - b) / abs(b) for a, b in zip(mg, ms)]
    print("start  C_edges %.6e C_nonedges %.6e NP %.6f" % m0, flush=True)
    print("serial C_edges %.6e C_nonedges %.6e NP %.6f" % ms, flush=True)
    print("device C_edges %.6e C_nonedges %.6e NP %.6f" % mg, flush=True)
    print("relative differences %.4f %.4f %.4f" % tuple(rel), flush=True)
    assert rel[0] <= 0.015 and rel[1] <= 0.015 and rel[2] <= 0.04
    # both runs improve on the start by far more than they differ
    assert ms[0] < 0.5 * m0[0] and mg[0] < 0.5 * m0[0] and ms[2] > 1.8 * m0[2] and mg[2] > 1.8 * m0[2]
