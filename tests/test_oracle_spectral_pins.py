"""Pins of the oracle's spectral initial drawing (the layout starts from a
spectral layout, Sec. 3.2; UMAP's spectral initialisation).

Closed forms of the normalised Laplacian: on a path P_n the eigenvectors are
D^1/2 cos(pi k i / (n - 1)) with eigenvalues 1 - cos(pi k / (n - 1)); on a
cycle C_n the second eigenvalue 1 - cos(2 pi / n) is double and the drawing is
a regular n-gon.  On weighted graphs the eigenpairs are checked against the
eigen-equation and against ARPACK (scipy eigsh), a different routine.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O


def _ones(g):
    return np.ones(g.nnz)


@pytest.mark.parametrize("n", [5, 12, 40, 101])
def test_path_closed_form(n):
    g = G.path(n)
    xy, ev = O.spectral_layout(g.n, g.row_ptr, g.col_idx, _ones(g))
    assert np.allclose(ev, 1 - np.cos(np.pi * np.array([1, 2]) / (n - 1)), atol=1e-12)
    d = np.diff(g.row_ptr).astype(float)
    i = np.arange(n)
    for k in (1, 2):
        f = np.sqrt(d) * np.cos(np.pi * k * i / (n - 1))
        v = xy[:, k - 1].astype(float)
        cos = abs(f @ v) / (np.linalg.norm(f) * np.linalg.norm(v))
        assert cos > 1 - 1e-12
    assert np.isclose(np.abs(xy).max(), 10.0)
    for k in range(2):
        a = np.abs(xy[:, k])
        p = int(np.argmax(a > 0.5 * a.max()))
        assert xy[p, k] > 0


@pytest.mark.parametrize("n", [6, 17, 64])
def test_cycle_is_a_regular_polygon(n):
    g = G.cycle(n)
    xy, ev = O.spectral_layout(g.n, g.row_ptr, g.col_idx, _ones(g))
    assert np.allclose(ev, 1 - np.cos(2 * np.pi / n), atol=1e-12)
    r = np.hypot(xy[:, 0].astype(float), xy[:, 1])
    assert np.allclose(r, r[0], rtol=1e-6)
    ang = np.arctan2(xy[:, 1].astype(float), xy[:, 0])
    step = np.angle(np.exp(1j * np.diff(ang)))
    assert np.allclose(np.abs(step), 2 * np.pi / n, atol=1e-5)
    assert np.all(np.sign(step) == np.sign(step[0]))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_weighted_eigenpairs(seed):
    from scipy.sparse import csr_matrix, identity, diags
    from scipy.sparse.linalg import eigsh
    g = G.ba(300, 3, seed)
    rng = np.random.default_rng(seed)
    # symmetric positive weights
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    wu = rng.uniform(0.1, 1.0, g.nnz)
    W = csr_matrix((wu, (rows, g.col_idx)), shape=(g.n, g.n))
    W = (W + W.T) * 0.5
    W.sort_indices()
    xy, ev = O.spectral_layout(g.n, W.indptr, W.indices, W.data)
    d = np.asarray(W.sum(axis=1)).ravel()
    s = diags(1 / np.sqrt(d))
    L = identity(g.n) - s @ W @ s
    ref = np.sort(eigsh(L, k=3, which="SA", tol=1e-12)[0])
    assert np.allclose(ev, ref[1:3], atol=1e-9)
    for k in range(2):
        v = xy[:, k].astype(float)
        v /= np.linalg.norm(v)
        assert np.linalg.norm(L @ v - ev[k] * v) < 1e-5            # float32 rounding of the drawing
        assert abs(v @ np.sqrt(d)) / np.linalg.norm(np.sqrt(d)) < 1e-5


def test_disconnected_and_isolated_are_rejected():
    g = G.disjoint_union([G.path(5), G.path(6)])
    with pytest.raises(O.OracleError) as e:
        O.spectral_layout(g.n, g.row_ptr, g.col_idx, _ones(g))
    assert e.value.status == O.EGRAPH
    g = G.disjoint_union([G.cycle(5), G.empty(1)])
    with pytest.raises(O.OracleError) as e:
        O.spectral_layout(g.n, g.row_ptr, g.col_idx, _ones(g))
    assert e.value.status == O.EGRAPH
    with pytest.raises(O.OracleError) as e:
        O.spectral_layout(2, np.array([0, 1, 2]), np.array([1, 0]), np.ones(2))
    assert e.value.status == O.EINVAL
