"""Pins of the oracle's layout step (C2 of Sec. 2.1, GradSample of Alg. 5 in
Sec. 3.3.2).

Each check compares the oracle with something other than itself: the
generator's published reference outputs, the fuzzy union written as a
probability (1 - (1 - a)(1 - b)) on dense matrices, finite differences of
the UMAP cross-entropy terms, the closed-form window schedule, windows worked
by hand in which the serial order of Alg. 5 changes the result, the serial
window as a composition of one-entry windows, and, for the synchronous
fixed-point form the device runs, the independence of a window from the
order of its edges and its agreement with the serial order when no two
entries share a vertex.
"""
import os

import numpy as np
import pytest

import graphgen as G
import oracle as O

import sys
sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import random_knn  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
A_UMAP, B_UMAP = 1.5769434603113077, 0.8950608781227859


def test_splitmix64_reference_outputs():
    lines = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
             if l.strip() and not l.startswith("#")]
    seed = int(lines[0][1])
    for i, v in lines[1:]:
        assert O.splitmix64(seed, int(i)) == int(v)


def test_umap_default_curve_parameters():
    """alpha, beta are UMAP's least-squares fit of 1 / (1 + a x^(2b)) to the
    target curve of min_dist 0.1, spread 1 (1 below min_dist, exp decay
    above)."""
    from scipy.optimize import curve_fit
    x = np.linspace(0, 3.0, 300)
    y = np.where(x < 0.1, 1.0, np.exp(-(x - 0.1) / 1.0))
    (a, b), _ = curve_fit(lambda x, a, b: 1.0 / (1.0 + a * x ** (2 * b)), x, y)
    assert abs(a - A_UMAP) < 1e-3 and abs(b - B_UMAP) < 1e-3


def _random_knn(n, k, seed, binary=False, zero_frac=0.2):
    return random_knn(n, k, seed, binary=binary, zero_frac=zero_frac)


def _dense(rp, col, val, n):
    d = np.zeros((n, n))
    for i in range(n):
        d[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return d


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fuzzy_union_is_probabilistic_or(seed):
    n, k = 60, 7
    ids, w = _random_knn(n, k, seed)
    A = np.zeros((n, n))
    for i in range(n):
        for q in range(k):
            if ids[i, q] >= 0:
                A[i, ids[i, q]] = w[i, q]
    U = 1.0 - (1.0 - A) * (1.0 - A.T)
    rp, col, val = O.fuzzy_union(ids, w)
    assert rp[0] == 0 and rp[-1] == len(col)
    for i in range(n):
        c = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(c) > 0)
        assert np.array_equal(c, np.nonzero(U[i] > 0)[0])
    D = _dense(rp, col, val, n)
    assert np.allclose(D, U.astype(np.float32), rtol=2e-7, atol=0)
    assert np.array_equal(D, D.T)
    assert np.all(D >= np.maximum(A, A.T).astype(np.float32) - 1e-7)


def test_fuzzy_union_binary_weights_is_or_of_patterns():
    ids, w = _random_knn(50, 5, 9, binary=True, zero_frac=0.0)
    rp, col, val = O.fuzzy_union(ids, w)
    pat = np.zeros((50, 50), bool)
    for i in range(50):
        pat[i, ids[i][ids[i] >= 0]] = True
    pat |= pat.T
    assert np.array_equal(_dense(rp, col, val, 50) > 0, pat) and np.all(val == 1.0)


def test_fuzzy_union_rejects_self_and_out_of_range():
    ids = np.array([[1, 0], [0, -1]], np.int32)
    with pytest.raises(O.OracleError):
        O.fuzzy_union(ids, np.ones((2, 2), np.float32))
    with pytest.raises(O.OracleError):
        O.fuzzy_union(np.array([[2]], np.int32), np.ones((1, 1), np.float32))


def test_edge_shuffle_is_the_keyed_permutation():
    ids, w = _random_knn(80, 6, 4)
    rp, col, val = O.fuzzy_union(ids, w)
    seed = 0xC0FFEE
    head, tail, ws = O.edge_shuffle(rp, col, val, seed)
    m = len(col)
    rows = np.repeat(np.arange(80), np.diff(rp))
    keys = np.array([O.splitmix64(seed, e + 1) for e in range(m)], dtype=np.uint64)
    order = np.lexsort((np.arange(m), keys))
    assert np.array_equal(head, rows[order]) and np.array_equal(tail, col[order]) and np.array_equal(ws, val[order])


def _two(xa, xb, h=1.0):
    return np.array([0], np.int32), np.array([1], np.int32), np.array([h], np.float32), \
        np.array([xa, xb], np.float32)


def _attr_cost(xa, xb):
    d2 = (xa[0] - xb[0]) ** 2 + (xa[1] - xb[1]) ** 2
    return np.log1p(A_UMAP * d2 ** B_UMAP)


def _rep_cost(xa, xb):
    d2 = (xa[0] - xb[0]) ** 2 + (xa[1] - xb[1]) ** 2
    return -np.log1p(-1.0 / (1.0 + A_UMAP * d2 ** B_UMAP))


def _num_grad(f, xa, xb, eps=1e-6):
    g = np.zeros(2)
    for d in range(2):
        p, q = np.array(xa, float), np.array(xa, float)
        p[d] += eps
        q[d] -= eps
        g[d] = (f(p, xb) - f(q, xb)) / (2 * eps)
    return g


@pytest.mark.parametrize("xa,xb", [((0.5, 0.25), (-0.3, 0.1)), ((1.0, -2.0), (0.25, 0.5)),
                                   ((0.0, 0.0), (3.0, 4.0))])
def test_attraction_is_the_cross_entropy_gradient(xa, xb):
    """With no negative samples one window moves a by -lr h grad_a of
    h log(1 + a d^(2b)) and b by the opposite amount."""
    h, lr = 0.7, 0.01
    head, tail, w, xy = _two(xa, xb, h)
    out = O.grad_sample(2, head, tail, w, xy, a=A_UMAP, b=B_UMAP, alpha0=lr, window=1, neg=0, t=1, seed=1)
    g = _num_grad(_attr_cost, np.array(xy[0], float), np.array(xy[1], float))
    da = out[0].astype(float) - xy[0]
    db = out[1].astype(float) - xy[1]
    assert np.allclose(da, -lr * h * g, rtol=2e-4, atol=2e-8)
    assert np.allclose(db, lr * h * g, rtol=2e-4, atol=2e-8)


def _seed_drawing(n, neg, want, start=1):
    """The first seed whose neg draws splitmix64(seed, q + 1) mod n equal want."""
    for seed in range(start, start + 100000):
        if [O.splitmix64(seed, q + 1) % n for q in range(neg)] == list(want):
            return seed
    raise AssertionError("no seed")


def test_repulsion_is_the_cross_entropy_gradient():
    """A negative sample that hits b pushes a along -grad_a of
    gamma * (-log(1 - w)) (up to UMAP's 0.001 regulariser of d^2), taken at
    a's position after the entry's attraction; a sample hitting a is skipped."""
    h, lr, gamma = 0.6, 0.1, 1.3
    xa, xb = (0.5, 1.0), (2.5, 3.0)
    head, tail, w, xy = _two(xa, xb, h)
    kw = dict(a=A_UMAP, b=B_UMAP, gamma=gamma, alpha0=lr, window=1, t=1)
    seed = _seed_drawing(2, 1, [1])
    base = O.grad_sample(2, head, tail, w, xy, neg=0, seed=seed, **kw)
    out = O.grad_sample(2, head, tail, w, xy, neg=1, seed=seed, **kw)
    g = _num_grad(_rep_cost, np.array(base[0], float), np.array(base[1], float))
    rep = out[0].astype(float) - base[0]
    assert np.allclose(rep, -lr * h * gamma * g, rtol=3e-4)
    assert np.array_equal(out[1], base[1])
    skip = _seed_drawing(2, 2, [0, 1])
    assert np.array_equal(O.grad_sample(2, head, tail, w, xy, neg=2, seed=skip, **kw), out)


def test_repulsion_clip_and_coincident_points():
    h, lr = 1.0, 0.01
    seed = _seed_drawing(2, 1, [1])
    head, tail, w, xy = _two((0.25, 0.5), (0.25, 0.5), h)      # coincident: +4 per coordinate
    out = O.grad_sample(2, head, tail, w, xy, a=A_UMAP, b=B_UMAP, alpha0=lr, window=1, neg=1, t=1, seed=seed)
    assert np.allclose(out[0].astype(float) - xy[0], lr * h * 4.0, rtol=1e-6)
    head, tail, w, xy = _two((0.26, 0.5), (0.25, 0.49), h)     # close: clipped at 4
    out = O.grad_sample(2, head, tail, w, xy, a=A_UMAP, b=B_UMAP, alpha0=lr, window=1, neg=1, t=1, seed=seed)
    base = O.grad_sample(2, head, tail, w, xy, a=A_UMAP, b=B_UMAP, alpha0=lr, window=1, neg=0, t=1, seed=seed)
    assert np.allclose(out[0].astype(float) - base[0], lr * h * 4.0, rtol=1e-5)


def _golden_cases():
    cases, cur = [], None
    for line in open(os.path.join(GOLDEN, "gradsample_hand_3v.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        key, *rest = line.split()
        if key == "case":
            cur = {"name": rest[0]}
        elif key == "params":
            cur["params"] = {k: float(v) for k, v in (r.split("=") for r in rest)}
        elif key == "end":
            cases.append(cur)
        else:
            cur[key] = [float(x) for x in rest]
    return cases


@pytest.mark.parametrize("case", _golden_cases(), ids=lambda c: c["name"])
def test_grad_sample_hand_worked_windows(case):
    """Windows worked by hand: the serial order (each entry reads the moved
    coordinates) and the synchronous form differ on a chain of entries, and
    a negative sample reads its head after the entry's attraction."""
    p = case["params"]
    n = int(p["n"])
    e = np.array(case["edges"]).reshape(-1, 3)
    head, tail, w = e[:, 0].astype(np.int32), e[:, 1].astype(np.int32), e[:, 2].astype(np.float32)
    xy = np.array(case["xy"], np.float32).reshape(n, 2)
    if "drawn" in p:
        assert O.splitmix64(int(p["seed"]), 1) % n == int(p["drawn"])
    kw = dict(a=p["a"], b=p["b"], gamma=p["gamma"], alpha0=p["alpha0"], window=int(p["window"]),
              neg=int(p["neg"]), t=int(p["t"]), seed=int(p["seed"]))
    ser = O.grad_sample(n, head, tail, w, xy, **kw)
    win = O.grad_sample_window(n, head, tail, w, xy, **kw)
    exp_s = np.array(case["serial"], np.float64).reshape(n, 2)
    exp_w = np.array(case["window"], np.float64).reshape(n, 2)
    assert np.allclose(ser, exp_s, rtol=2e-7, atol=1e-7), ser
    assert np.allclose(win, exp_w, rtol=2e-7, atol=1e-7), win


def test_serial_window_is_a_composition_of_single_entries():
    """A window of s entries (no negative samples) equals s one-entry windows
    applied in the same order at the same rate, and depends on the order."""
    g = G.grid_2d(5, 6)
    rng = np.random.default_rng(12)
    head = np.repeat(np.arange(g.n), np.diff(g.row_ptr)).astype(np.int32)
    tail = g.col_idx.astype(np.int32)
    w = rng.uniform(0.2, 1.0, len(tail)).astype(np.float32)
    xy = rng.uniform(-3, 3, (g.n, 2)).astype(np.float32)
    m = len(tail)
    kw = dict(a=A_UMAP, b=B_UMAP, alpha0=0.3, neg=0, t=1, seed=1)
    whole = O.grad_sample(g.n, head, tail, w, xy, window=m, **kw)
    step = xy.copy()
    for e in range(m):
        step = O.grad_sample(g.n, head[e:e + 1], tail[e:e + 1], w[e:e + 1], step, window=1, **kw)
    # one-entry calls round the drawing to float after every entry
    assert np.allclose(whole, step, rtol=0, atol=5e-6)
    p = rng.permutation(m)
    other = O.grad_sample(g.n, head[p], tail[p], w[p], xy, window=m, **kw)
    assert np.abs(other.astype(float) - whole).max() > 1e-3


def test_window_form_equals_serial_on_disjoint_entries():
    """When no two entries of a window share a vertex (negative samples
    included), the synchronous fixed-point form and the serial order agree up
    to the 2^-33 rounding of each move."""
    n, pairs, neg, seed = 4000, 40, 5, 4242
    drawn = {O.splitmix64(seed, l * neg + q + 1) % n for l in range(pairs) for q in range(neg)}
    free = np.array(sorted(set(range(n)) - drawn))
    rng = np.random.default_rng(5)
    perm = rng.permutation(free)
    head, tail = perm[:pairs].astype(np.int32), perm[pairs:2 * pairs].astype(np.int32)
    w = rng.uniform(0.3, 1.0, pairs).astype(np.float32)
    xy = rng.uniform(-10, 10, (n, 2)).astype(np.float32)
    kw = dict(a=A_UMAP, b=B_UMAP, alpha0=1.0, window=pairs, neg=neg, t=3, seed=seed, it_begin=0, it_end=1)
    ser = O.grad_sample(n, head, tail, w, xy, **kw).astype(np.float64)
    win = O.grad_sample_window(n, head, tail, w, xy, **kw).astype(np.float64)
    # grid rounding: the start position and each of at most neg + 1 moves
    # by 2^-33, then both sides round to float once
    ulp = np.spacing(np.abs(ser).astype(np.float32)).astype(np.float64)
    assert np.all(np.abs(ser - win) <= ulp + (neg + 2) * 2.0**-33)
    assert np.mean(ser == win) > 0.98


@pytest.mark.parametrize("m,s,t", [(37, 5, 20), (10, 10, 3), (11, 1, 25), (64, 63, 7)])
def test_window_schedule_closed_form(m, s, t):
    rng = np.random.default_rng(m)
    head = rng.integers(0, 20, m).astype(np.int32)
    tail = ((head + 1 + rng.integers(0, 18, m)) % 20).astype(np.int32)
    xy = rng.uniform(-5, 5, (20, 2)).astype(np.float32)
    _, vis = O.grad_sample(20, head, tail, np.ones(m, np.float32), xy, a=A_UMAP, b=B_UMAP, window=s, neg=2, t=t,
                           seed=3, visits=True)
    x = np.arange(t * s) % m
    assert np.array_equal(vis, np.bincount(x, minlength=m))


def test_learning_rate_decays_linearly():
    """Per-iteration move of a far-apart pair (attraction nearly constant) is
    alpha0 (1 - it / t) times the first."""
    head, tail, w, xy = _two((0.0, 0.0), (30.0, 40.0))
    t = 8
    moves = []
    for it in range(t):
        out = O.grad_sample(2, head, tail, w, xy, a=A_UMAP, b=B_UMAP, alpha0=1.0, window=1, neg=0, t=t, seed=1,
                            it_begin=it, it_end=it + 1)
        moves.append(float(out[0, 0]) - float(xy[0, 0]))
    assert np.allclose(np.array(moves) / moves[0], 1.0 - np.arange(t) / t, rtol=1e-4)


def test_synchronous_window_ignores_edge_order():
    """The device's synchronous form: one window over all edges (s = m, no
    negatives): permuting the edge array leaves the result bit-identical, and
    each window equals the sum of the single-edge moves."""
    g = G.grid_2d(6, 7)
    rng = np.random.default_rng(2)
    head = np.repeat(np.arange(g.n), np.diff(g.row_ptr)).astype(np.int32)
    tail = g.col_idx.astype(np.int32)
    w = rng.uniform(0.2, 1.0, len(tail)).astype(np.float32)
    xy = rng.uniform(-3, 3, (g.n, 2)).astype(np.float32)
    m = len(tail)
    kw = dict(a=A_UMAP, b=B_UMAP, alpha0=0.3, window=m, neg=0, t=4, seed=1)
    r1 = O.grad_sample_window(g.n, head, tail, w, xy, **kw)
    p = rng.permutation(m)
    r2 = O.grad_sample_window(g.n, head[p], tail[p], w[p], xy, **kw)
    assert np.array_equal(r1, r2)
    one = O.grad_sample_window(g.n, head, tail, w, xy, **dict(kw, t=1))
    acc = np.zeros((g.n, 2))
    for e in range(m):
        single = O.grad_sample_window(g.n, head[e:e + 1], tail[e:e + 1], w[e:e + 1], xy, **dict(kw, window=1, t=1))
        acc += single.astype(float) - xy
    assert np.allclose(one.astype(float) - xy, acc, atol=1e-6)


def test_attraction_lowers_the_cost():
    """Without negative samples and with a small rate the attractive cost
    sum_e h log(1 + a d^(2b)) falls at every window."""
    g = G.grid_2d(8, 8)
    ids, hops = O.knn_partial(g, 15)
    w, _, _ = O.membership(hops)
    rp, col, val = O.fuzzy_union(ids, w)
    head, tail, ws = O.edge_shuffle(rp, col, val, 11)
    rng = np.random.default_rng(3)
    xy = rng.uniform(-4, 4, (g.n, 2)).astype(np.float32)

    def cost(x):
        d2 = ((x[head].astype(float) - x[tail]) ** 2).sum(1)
        return float((ws * np.log1p(A_UMAP * d2 ** B_UMAP)).sum())

    s = int(len(head) ** 0.9)
    prev = cost(xy)
    for it in range(10):
        xy = O.grad_sample(g.n, head, tail, ws, xy, a=A_UMAP, b=B_UMAP, alpha0=0.02, window=s, neg=0, t=10, seed=1,
                           it_begin=it, it_end=it + 1)
        c = cost(xy)
        assert c < prev
        prev = c


def test_grad_sample_argument_errors():
    head, tail, w, xy = _two((0, 0), (1, 1))
    with pytest.raises(O.OracleError):
        O.grad_sample(2, head, tail, w, xy, a=1, b=1, window=2, t=1, seed=0)
    with pytest.raises(O.OracleError):
        O.grad_sample(2, head, np.array([2], np.int32), w, xy, a=1, b=1, window=1, t=1, seed=0)
    out = O.grad_sample(2, head, tail, w, xy, a=1, b=1, window=1, t=3, seed=0, it_begin=2, it_end=2)
    assert np.array_equal(out, xy)


def test_window_form_with_one_entry_per_part_is_serial():
    """With as many parts as entries, every part is one entry and the
    synchronous form takes the entries one after the other: it then follows
    the serial order up to the 2^-32 grid (on a grid graph, where the
    entries of a window share vertices everywhere)."""
    g = G.grid_2d(7, 6)
    rng = np.random.default_rng(21)
    head = np.repeat(np.arange(g.n), np.diff(g.row_ptr)).astype(np.int32)
    tail = g.col_idx.astype(np.int32)
    w = rng.uniform(0.2, 1.0, len(tail)).astype(np.float32)
    xy = rng.uniform(-3, 3, (g.n, 2)).astype(np.float32)
    m = len(tail)
    s = m - 7
    kw = dict(a=A_UMAP, b=B_UMAP, alpha0=0.5, window=s, neg=4, t=5, seed=31, it_begin=2, it_end=4)
    ser = O.grad_sample(g.n, head, tail, w, xy, **kw)
    one = O.grad_sample_window(g.n, head, tail, w, xy, parts=s, **kw)
    whole = O.grad_sample_window(g.n, head, tail, w, xy, parts=1, **kw)
    assert np.abs(one.astype(float) - ser).max() < 1e-5
    assert np.abs(whole.astype(float) - ser).max() > 1e-2
