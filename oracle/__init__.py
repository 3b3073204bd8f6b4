"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct CPU statement of the BFS kNN construction of
arXiv 2509.19703 (GUMAP steps C0/C1 of Alg. 1, PartialBFS of Alg. 4 in
Sec. 3.3.1, and the UMAP fuzzy membership of Sec. 2.1), of the drawing
quality metrics of Sec. 4.1.3 computed on the same BFS, of the layout step C2
that follows (fuzzy union of the kNN weights, edge shuffle and the sliding
window GradSample of Alg. 5, Sec. 3.3.2), of its spectral initial drawing and
of the spectral sparsification front end (Sec. 3.2, Alg. 2).  Only
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use it.  It shares no code with the GPU library and the GPU
library never calls it.

Where the arithmetic lives: ``oracle.c`` (plain C, gcc) holds the BFS, kNN,
partial BFS, membership, stress, neighbourhood preservation, SplitMix64,
fuzzy union, edge shuffle and GradSample; this module only moves numpy arrays
in and out of those.  Three oracles are numpy code in this module:
``spectral_layout`` (a dense eigendecomposition), ``effective_resistance``
(random projection with preconditioned conjugate gradients) and
``sparsify_select`` (maximum spanning forest and the top remaining edges).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

OK, EINVAL, EGRAPH, ERANGE, ENOMEM = 0, -1, -2, -3, -4


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc."""
    src = os.path.join(_HERE, "oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", src, "-o", tmp,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        i32, i64 = ctypes.c_int32, ctypes.c_int64
        lib.oracle_bfs_dist.argtypes = [i32, vp, vp, i32, vp]
        lib.oracle_knn_build.argtypes = [i32, vp, vp, i32, vp, i32, vp, vp, vp, ctypes.c_int]
        lib.oracle_knn_partial.argtypes = [i32, vp, vp, i32, vp, i32, vp, vp, ctypes.c_int]
        lib.oracle_membership.argtypes = [i64, i32, vp, vp, vp, vp, ctypes.c_int]
        lib.oracle_stress.argtypes = [i32, vp, vp, vp, vp, i64, vp, vp, ctypes.c_int]
        lib.oracle_neighborhood.argtypes = [i32, vp, vp, vp, i32, vp, i64, vp, vp, ctypes.c_int]
        lib.oracle_splitmix64.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.oracle_splitmix64.restype = ctypes.c_uint64
        lib.oracle_fuzzy_union.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64, vp]
        lib.oracle_edge_shuffle.argtypes = [i32, vp, vp, vp, ctypes.c_uint64, vp, vp, vp]
        d = ctypes.c_double
        lib.oracle_grad_sample.argtypes = [i32, i64, vp, vp, vp, vp, d, d, d, d, i64, i32, i32, ctypes.c_uint64,
                                           i32, i32, vp]
        lib.oracle_grad_sample_window.argtypes = lib.oracle_grad_sample.argtypes + [i32]
        for f in (lib.oracle_fuzzy_union, lib.oracle_edge_shuffle, lib.oracle_grad_sample,
                  lib.oracle_grad_sample_window):
            f.restype = ctypes.c_int
        for f in (lib.oracle_bfs_dist, lib.oracle_knn_build, lib.oracle_knn_partial, lib.oracle_membership,
                  lib.oracle_stress, lib.oracle_neighborhood):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


def default_threads() -> int:
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)


def _ptr(a):
    return None if a is None else a.ctypes.data


def _csr(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    return rp, ci


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__("oracle status %d" % status)
        self.status = status


def bfs_dist(g, s: int) -> np.ndarray:
    """Hop distance from ``s`` to every vertex (-1 = unreachable)."""
    rp, ci = _csr(g)
    dist = np.empty(g.n, dtype=np.int32)
    st = _load().oracle_bfs_dist(g.n, _ptr(rp), _ptr(ci), int(s), _ptr(dist))
    if st:
        raise OracleError(st)
    return dist


def knn_build(g, k: int, sources=None, hop_matrix: bool = False, threads: int | None = None):
    """All-source (or listed-source) BFS + (hop, id) kNN.

    Returns ``(ids int32[rows,k], hops uint8[rows,k], hop_matrix uint8[rows,n] or None)``.
    """
    rp, ci = _csr(g)
    src = None if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    rows = g.n if src is None else int(src.shape[0])
    ids = np.empty((rows, k), dtype=np.int32)
    hops = np.empty((rows, k), dtype=np.uint8)
    hm = np.empty((rows, g.n), dtype=np.uint8) if hop_matrix else None
    st = _load().oracle_knn_build(g.n, _ptr(rp), _ptr(ci), int(k), _ptr(src), rows,
                                  _ptr(ids), _ptr(hops), _ptr(hm), int(threads or default_threads()))
    if st:
        raise OracleError(st)
    return ids, hops, hm


def knn_partial(g, k: int, sources=None, threads: int | None = None):
    """Truncated BFS kNN (PartialBFS).  Returns ``(ids, hops)``."""
    rp, ci = _csr(g)
    src = None if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    rows = g.n if src is None else int(src.shape[0])
    ids = np.empty((rows, k), dtype=np.int32)
    hops = np.empty((rows, k), dtype=np.uint8)
    st = _load().oracle_knn_partial(g.n, _ptr(rp), _ptr(ci), int(k), _ptr(src), rows,
                                    _ptr(ids), _ptr(hops), int(threads or default_threads()))
    if st:
        raise OracleError(st)
    return ids, hops


def membership(hops: np.ndarray, k: int | None = None, threads: int | None = None):
    """FP64 rho/sigma bisection.  Returns ``(weights f32[rows,k], rho f32[rows], sigma f32[rows])``."""
    hops = np.ascontiguousarray(hops, dtype=np.uint8)
    rows, kk = hops.shape
    k = kk if k is None else k
    assert k == kk
    w = np.empty((rows, k), dtype=np.float32)
    rho = np.empty(rows, dtype=np.float32)
    sigma = np.empty(rows, dtype=np.float32)
    st = _load().oracle_membership(rows, int(k), _ptr(hops), _ptr(w), _ptr(rho), _ptr(sigma),
                                   int(threads or default_threads()))
    if st:
        raise OracleError(st)
    return w, rho, sigma


def stress_rows(g, xy: np.ndarray, sources=None, threads: int | None = None):
    """Per-source stress sums and pair counts (Sec. 4.1.3 aggregated stress).

    ``xy`` is float32 [n, 2].  Returns ``(row_sum float64[rows], row_pairs int64[rows])``."""
    rp, ci = _csr(g)
    xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(g.n, 2)
    src = None if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    rows = g.n if src is None else int(src.shape[0])
    row_sum = np.empty(rows, dtype=np.float64)
    row_pairs = np.empty(rows, dtype=np.int64)
    st = _load().oracle_stress(g.n, _ptr(rp), _ptr(ci), _ptr(xy), _ptr(src), rows, _ptr(row_sum),
                               _ptr(row_pairs), int(threads or default_threads()))
    if st:
        raise OracleError(st)
    return row_sum, row_pairs


def stress(g, xy: np.ndarray, sources=None, threads: int | None = None):
    """Aggregated stress: ``(sum, pairs)``; the metric is ``sum / pairs``."""
    row_sum, row_pairs = stress_rows(g, xy, sources, threads)
    return float(row_sum.sum()), int(row_pairs.sum())


def neighborhood_scores(g, xy: np.ndarray, r: int = 2, vertices=None, threads: int | None = None):
    """Per-vertex neighbourhood preservation (Sec. 4.1.3) of the listed vertices
    (all when None): ``(score float64[rows] (NaN where the graph ball is
    empty), ball int32[rows])``."""
    rp, ci = _csr(g)
    xy = np.ascontiguousarray(xy, dtype=np.float32).reshape(g.n, 2)
    vt = None if vertices is None else np.ascontiguousarray(vertices, dtype=np.int32)
    rows = g.n if vt is None else int(vt.shape[0])
    score = np.empty(rows, dtype=np.float64)
    ball = np.empty(rows, dtype=np.int32)
    st = _load().oracle_neighborhood(g.n, _ptr(rp), _ptr(ci), _ptr(xy), int(r), _ptr(vt), rows, _ptr(score),
                                     _ptr(ball), int(threads or default_threads()))
    if st:
        raise OracleError(st)
    return score, ball


def neighborhood_preservation(g, xy: np.ndarray, r: int = 2, threads: int | None = None):
    """``(sum of defined scores, number of defined scores)``."""
    score, _ = neighborhood_scores(g, xy, r, threads=threads)
    ok = ~np.isnan(score)
    return float(score[ok].sum()), int(ok.sum())


# ---------------------------------------------------------------- layout C2 --
def splitmix64(seed: int, i: int) -> int:
    """The i-th output (i >= 1) of SplitMix64 seeded with ``seed``."""
    return int(_load().oracle_splitmix64(ctypes.c_uint64(seed & (2**64 - 1)), ctypes.c_uint64(i & (2**64 - 1))))


def fuzzy_union(ids: np.ndarray, weights: np.ndarray):
    """Symmetric fuzzy union of directed kNN weights.

    ``ids`` int32[n, k], ``weights`` float32[n, k] -> ``(row_ptr int32[n+1],
    col int32[nnz], val float32[nnz])`` with ascending columns per row."""
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    w = np.ascontiguousarray(weights, dtype=np.float32)
    n, k = ids.shape
    cap = max(1, 2 * n * k)
    rp = np.empty(n + 1, dtype=np.int32)
    col = np.empty(cap, dtype=np.int32)
    val = np.empty(cap, dtype=np.float32)
    nnz = np.zeros(1, dtype=np.int64)
    st = _load().oracle_fuzzy_union(n, k, _ptr(ids), _ptr(w), _ptr(rp), _ptr(col), _ptr(val), cap, _ptr(nnz))
    if st:
        raise OracleError(st)
    m = int(nnz[0])
    return rp, col[:m].copy(), val[:m].copy()


def edge_shuffle(row_ptr: np.ndarray, col: np.ndarray, val: np.ndarray, seed: int):
    """E_k in shuffled order: ``(head int32[m], tail int32[m], w float32[m])``."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float32)
    n = rp.shape[0] - 1
    m = int(rp[-1])
    head = np.empty(max(m, 1), dtype=np.int32)
    tail = np.empty(max(m, 1), dtype=np.int32)
    w = np.empty(max(m, 1), dtype=np.float32)
    st = _load().oracle_edge_shuffle(n, _ptr(rp), _ptr(col), _ptr(val), ctypes.c_uint64(seed & (2**64 - 1)),
                                     _ptr(head), _ptr(tail), _ptr(w))
    if st:
        raise OracleError(st)
    return head[:m], tail[:m], w[:m]


def _grad_call(fn, n, head, tail, w, xy, a, b, gamma, alpha0, window, neg, t, seed, it_begin, it_end, visits,
               *extra):
    head = np.ascontiguousarray(head, dtype=np.int32)
    tail = np.ascontiguousarray(tail, dtype=np.int32)
    w = np.ascontiguousarray(w, dtype=np.float32)
    out = np.ascontiguousarray(np.array(xy, dtype=np.float32).reshape(n, 2))
    m = int(head.shape[0])
    vis = np.zeros(max(m, 1), dtype=np.int32) if visits else None
    it_end = t if it_end is None else it_end
    st = fn(int(n), m, _ptr(head), _ptr(tail), _ptr(w), _ptr(out), float(a), float(b), float(gamma), float(alpha0),
            int(window), int(neg), int(t), ctypes.c_uint64(seed & (2**64 - 1)), int(it_begin), int(it_end),
            _ptr(vis), *extra)
    if st:
        raise OracleError(st)
    return (out, vis[:m]) if visits else out


def grad_sample(n: int, head, tail, w, xy: np.ndarray, *, a: float, b: float, gamma: float = 1.0,
                alpha0: float = 1.0, window: int, neg: int = 5, t: int, seed: int, it_begin: int = 0,
                it_end: int | None = None, visits: bool = False):
    """GradSample (Alg. 5, Sec. 3.3.2) iterations [it_begin, it_end) of a run
    of ``t``, entries moved one after the other in the paper's order (FP64
    coordinates during the call).

    Returns the new float32[n, 2] drawing (and the per-position visit counts
    when ``visits``)."""
    return _grad_call(_load().oracle_grad_sample, n, head, tail, w, xy, a, b, gamma, alpha0, window, neg, t, seed,
                      it_begin, it_end, visits)


def grad_sample_window(n: int, head, tail, w, xy: np.ndarray, *, a: float, b: float, gamma: float = 1.0,
                       alpha0: float = 1.0, window: int, neg: int = 5, t: int, seed: int, it_begin: int = 0,
                       it_end: int | None = None, visits: bool = False, parts: int = 1):
    """The same iterations with every window cut into ``parts`` consecutive
    parts, each applied synchronously in 2^-32 fixed point (each entry from
    its part's start positions, its own steps in Alg. 5's order): the
    device's form, used to check the kernels' arithmetic; ``grad_sample`` is
    the paper's serial order."""
    return _grad_call(_load().oracle_grad_sample_window, n, head, tail, w, xy, a, b, gamma, alpha0, window, neg, t,
                      seed, it_begin, it_end, visits, int(parts))


def spectral_layout(n: int, row_ptr, col, val, dim: int = 2):
    """Spectral initial drawing (Sec. 3.2: the layout starts from a spectral
    layout, as in UMAP): the eigenvectors of the 2nd .. (dim+1)-th smallest
    eigenvalues of the normalised Laplacian L = I - D^-1/2 W D^-1/2 of the
    symmetric weighted graph W (FP64, dense numpy.linalg.eigh).  Each vector
    has unit norm and the sign that makes positive its first entry (in index
    order) of magnitude above half its largest (a rule that rounding cannot
    flip, unlike "the largest entry" on symmetric graphs); the drawing is the
    vectors
    scaled by 10 / (largest magnitude over all coordinates), rounded to
    float.  Returns (xy float32 [n, dim], eigenvalues float64 [dim]).
    Raises OracleError(EGRAPH) for a vertex of zero degree or a disconnected
    graph (second eigenvalue below 1e-10), EINVAL for n < dim + 1."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    w = np.asarray(val, dtype=np.float64)
    if n < dim + 1:
        raise OracleError(EINVAL)
    W = np.zeros((n, n))
    for i in range(n):
        W[i, c[rp[i]:rp[i + 1]]] += w[rp[i]:rp[i + 1]]
    d = W.sum(axis=1)
    if np.any(d <= 0):
        raise OracleError(EGRAPH)
    s = 1.0 / np.sqrt(d)
    L = np.eye(n) - (s[:, None] * W) * s[None, :]
    evals, evecs = np.linalg.eigh(L)
    if evals[1] < 1e-10:
        raise OracleError(EGRAPH)
    V = evecs[:, 1:dim + 1].copy()
    for j in range(dim):
        a = np.abs(V[:, j])
        p = int(np.argmax(a > 0.5 * a.max()))
        if V[p, j] < 0:
            V[:, j] = -V[:, j]
    scale = 10.0 / np.abs(V).max()
    return (V * scale).astype(np.float32), evals[1:dim + 1].copy()


# ------------------------------------------------- spectral sparsification ---
def undirected_edges(row_ptr, col):
    """The edges (u, v), u < v, of a symmetric CSR in CSR order: (u, v) arrays."""
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
    up = c > rows
    return rows[up], c[up]


def jl_signs(seed: int, q: int, m: int) -> np.ndarray:
    """s[k, e] = +1 when bit 63 of SplitMix64(seed, k m + e + 1) is 0, else -1."""
    s = np.empty((q, m), dtype=np.float64)
    for k in range(q):
        for e in range(m):
            s[k, e] = -1.0 if (splitmix64(seed, k * m + e + 1) >> 63) else 1.0
    return s


def effective_resistance(n: int, row_ptr, col, q: int = 32, seed: int = 0, tol: float = 1e-10,
                         max_iters: int = 2000, return_x: bool = False):
    """Effective resistances of the edges of an unweighted graph (Sec. 3.2,
    Alg. 2: the sparsifier ranks edges by effective resistance), estimated
    as Spielman and Srivastava do: with random signs s_k (q vectors over the
    edges), x_k solves L x_k = B^T s_k (B the edge-vertex incidence, L = D - W)
    by conjugate gradients preconditioned with D, from x = 0, stopping when
    |r| <= tol |b| (or after max_iters), and
    R_e = (1/q) sum_k (x_k(u) - x_k(v))^2 for e = (u, v).
    FP64, plain loops over the steps.  Returns (R float64[m], iterations)."""
    u, v = undirected_edges(row_ptr, col)
    m = len(u)
    rp = np.asarray(row_ptr, dtype=np.int64)
    c = np.asarray(col, dtype=np.int64)
    deg = np.diff(rp).astype(np.float64)
    rows = np.repeat(np.arange(n), np.diff(rp))

    def lap(x):   # L x for every column of x (n x q)
        y = deg[:, None] * x
        np.subtract.at(y, rows, x[c])
        return y

    S = jl_signs(seed, q, m)
    B = np.zeros((n, q))
    for k in range(q):
        np.add.at(B[:, k], u, S[k])
        np.subtract.at(B[:, k], v, S[k])
    X = np.zeros((n, q))
    its = 0
    dinv = np.where(deg > 0, 1.0 / np.where(deg > 0, deg, 1.0), 0.0)
    for k in range(q):
        b = B[:, k]
        bn = np.sqrt(b @ b)
        x = np.zeros(n)
        r = b.copy()
        z = dinv * r
        p = z.copy()
        rz = r @ z
        it = 0
        while np.sqrt(r @ r) > tol * bn and it < max_iters:
            Ap = lap(p[:, None])[:, 0]
            a = rz / (p @ Ap)
            x += a * p
            r -= a * Ap
            z = dinv * r
            rz_new = r @ z
            p = z + (rz_new / rz) * p
            rz = rz_new
            it += 1
        X[:, k] = x
        its = max(its, it)
    R = ((X[u] - X[v]) ** 2).sum(axis=1) / q
    return (R, its, X, B) if return_x else (R, its)


def sparsify_select(n: int, row_ptr, col, R, target: int | None = None):
    """The sparsifier's edge choice (Sec. 3.2, Alg. 2): a maximum spanning
    forest with the effective resistances as weights, then further edges in
    decreasing resistance until `target` edges (default ceil(n ln n), at most
    m).  Edges are ordered by (R descending, edge index ascending), so the
    forest and the choice are unique.  Returns keep (bool [m])."""
    u, v = undirected_edges(row_ptr, col)
    m = len(u)
    R = np.asarray(R, dtype=np.float64)
    if target is None:
        target = int(np.ceil(n * np.log(n))) if n > 1 else 0
    target = min(target, m)
    order = sorted(range(m), key=lambda e: (-R[e], e))
    parent = list(range(n))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    keep = np.zeros(m, dtype=bool)
    count = 0
    for e in order:
        a, b = find(int(u[e])), find(int(v[e]))
        if a != b:
            parent[a] = b
            keep[e] = True
            count += 1
    for e in order:
        if count >= target:
            break
        if not keep[e]:
            keep[e] = True
            count += 1
    return keep
