"""GPU parity of the layout step C2 (fuzzy union, edge shuffle, GradSample
of Alg. 5) through the C-ABI, against the CPU oracle on the same inputs.

Union and shuffle are bit-exact (integer work plus one FP64 expression
evaluated in the same order on both sides).  GradSample runs in FP64 with
positions in 2^-32 fixed point; both sides evaluate the same expressions in
the same order, so the only source of difference is the last bit of the
FP64 power function (the device's and the host's pow may round differently).
Such a difference moves a fixed-point step by at most one unit (2^-32) and
a float coordinate by at most one ulp after one window; the tests allow
that per window and check that nearly all coordinates agree exactly.
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
        ref = O.grad_sample(n, head, tail, ws, xy, it_begin=it, it_end=it + 1, **kw)
        got = _dev(xy.copy())
        gumap.grad_sample(got, _dev(head), _dev(tail), _dev(ws), it_begin=it, it_end=it + 1, **kw)
        _compare_xy(got.cpu().numpy(), ref, 1, "%s neg=%d it=%d" % (name, neg, it))


@pytest.mark.parametrize("name", ["grid", "ba", "rand30"])
def test_grad_sample_many_windows(gumap, name):
    """A whole t-iteration run in one call (and split over three calls)."""
    n, head, tail, ws, xy = _layout_case(name, 8)
    m = len(head)
    t = 30
    kw = dict(a=gumap.UMAP_A, b=gumap.UMAP_B, gamma=1.0, alpha0=1.0, window=int(m ** 0.9), neg=5, t=t, seed=7)
    ref = O.grad_sample(n, head, tail, ws, xy, **kw)
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
        ref3 = O.grad_sample(n, head, tail, ws, ref3, it_begin=b, it_end=e, **kw)
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
        ref = O.grad_sample(n, head, tail, ws, xy, it_begin=it, it_end=it + 1, **kw)
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
    ref = O.grad_sample(n, head, tail, ws, xy, a=gumap.UMAP_A, b=gumap.UMAP_B, window=10, neg=5, t=2, seed=0,
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
    ref = O.grad_sample(g.n, oh_, ot_, ow_, xy, it_begin=0, it_end=3, **kw)
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
    ref = O.grad_sample(4, head, tail, ws, xy, **kw)
    got = _dev(xy.copy())
    gumap.grad_sample(got, _dev(head), _dev(tail), _dev(ws), **kw)
    assert np.array_equal(got.cpu().numpy(), ref)
    one = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
    gumap.grad_sample(one, _dev(np.zeros(0, np.int32)), _dev(np.zeros(0, np.int32)), _dev(np.zeros(0, np.float32)),
                      window=1, t=3)
    assert float(one.abs().sum()) == 0.0
