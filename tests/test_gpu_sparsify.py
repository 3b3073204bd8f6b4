"""GPU parity of the spectral sparsification front end (effective
resistances by random projection and conjugate gradients; the maximum
spanning forest and top edges) through the C-ABI, against the oracle.

Resistances: both sides run the same projection and the same
preconditioned CG to |r| <= 1e-10 |b|; they differ only by the rounding of
the sums, so the estimates agree to 1e-7 relative.  The selection is exact
for given resistances (a total order), so the sparsified CSR is compared
bit-exact on seeded resistance values, ties included.
"""
import numpy as np
import pytest

import graphgen as G
import oracle as O

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _csr_of_keep(g, keep):
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    rows = np.concatenate([u[keep], v[keep]])
    cols = np.concatenate([v[keep], u[keep]])
    order = np.lexsort((cols, rows))
    rp = np.zeros(g.n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    return np.cumsum(rp).astype(np.int32), cols[order].astype(np.int32)


@pytest.mark.parametrize("name,g", [("ba300", G.ba(300, 3, 21)), ("er500", G.er(500, 0.05, 22)),
                                    ("grid20", G.grid_2d(20, 20)), ("tree", G.ba(400, 1, 23)),
                                    ("union", G.disjoint_union([G.complete(9), G.cycle(30), G.empty(3),
                                                                G.ba(100, 2, 24)]))],
                         ids=lambda x: x if isinstance(x, str) else "")
def test_effective_resistance_parity(gumap, name, g):
    print("resistance", name, g.n, flush=True)
    R, its = gumap.effective_resistance(_dev(g.row_ptr), _dev(g.col_idx), q=32, seed=2509, flags=gumap.CSR_SORTED)
    oR, oits = O.effective_resistance(g.n, g.row_ptr, g.col_idx, q=32, seed=2509)
    R = R.cpu().numpy()
    rel = np.abs(R - oR) / np.maximum(oR, 1e-300)
    print("  iterations %d (oracle %d), max relative difference %.3g" % (its, oits, rel.max()), flush=True)
    assert len(R) == len(oR)
    assert rel.max() < 1e-7
    if name == "tree":
        assert np.allclose(R, 1.0, atol=1e-8)


def _seeded_R(m, seed, ties):
    rng = np.random.default_rng(seed)
    R = rng.uniform(0.0, 1.0, m)
    return np.round(R, 1) if ties else R


@pytest.mark.parametrize("name,g,target,ties", [
    ("er1500", G.er(1500, 0.02, 31), 0, False),
    ("er1500_ties", G.er(1500, 0.02, 31), 0, True),
    ("small_target", G.er(600, 0.05, 32), 50, False),
    ("all_edges", G.ba(500, 2, 33), 10**9, False),
    ("union", G.disjoint_union([G.complete(40), G.cycle(50), G.empty(4), G.er(300, 0.1, 34)]), 0, True),
])
def test_sparsify_select_parity(gumap, name, g, target, ties):
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    R = _seeded_R(len(u), 41, ties)
    print("select", name, g.n, len(u), flush=True)
    rp, col = gumap.sparsify_select(_dev(g.row_ptr), _dev(g.col_idx), _dev(R), target=target, flags=gumap.CSR_SORTED)
    keep = O.sparsify_select(g.n, g.row_ptr, g.col_idx, R, target=target if target > 0 else None)
    orp, ocol = _csr_of_keep(g, keep)
    assert np.array_equal(rp.cpu().numpy(), orp)
    assert np.array_equal(col.cpu().numpy(), ocol)


def test_sparsify_select_mid_size(gumap):
    g = G.er(4000, 0.05, 35)
    u, v = O.undirected_edges(g.row_ptr, g.col_idx)
    R = _seeded_R(len(u), 42, False)
    print("select er4000", len(u), flush=True)
    rp, col = gumap.sparsify_select(_dev(g.row_ptr), _dev(g.col_idx), _dev(R), flags=gumap.CSR_SORTED)
    keep = O.sparsify_select(g.n, g.row_ptr, g.col_idx, R)
    orp, ocol = _csr_of_keep(g, keep)
    assert np.array_equal(rp.cpu().numpy(), orp) and np.array_equal(col.cpu().numpy(), ocol)


def test_sparsify_errors(gumap):
    # an entry without its mirror
    rp = np.array([0, 2, 2, 3], np.int32)      # 0-1 has no mirror
    col = np.array([1, 2, 0], np.int32)
    with pytest.raises(gumap.GumapError) as e:
        gumap.effective_resistance(_dev(rp), _dev(col), flags=gumap.CSR_SORTED)
    assert e.value.status == gumap.EGRAPH
    # a self-loop in input declared canonical
    rp = np.array([0, 2, 3], np.int32)
    col = np.array([0, 1, 0], np.int32)
    with pytest.raises(gumap.GumapError) as e:
        gumap.sparsify_select(_dev(rp), _dev(col), _dev(np.ones(1)), flags=gumap.CSR_SORTED)
    assert e.value.status == gumap.EGRAPH
    # unsorted input without the flag is canonicalised first
    g = G.ba(200, 3, 36)
    d = G.dirty(g, 5)
    R1, _ = gumap.effective_resistance(_dev(d.row_ptr), _dev(d.col_idx), q=8, seed=1)
    R2, _ = gumap.effective_resistance(_dev(g.row_ptr), _dev(g.col_idx), q=8, seed=1, flags=gumap.CSR_SORTED)
    assert np.array_equal(R1.cpu().numpy(), R2.cpu().numpy())


def test_sparsify_pipeline_dense_er(gumap):
    """Full size: the dense ER graph G(16,384, 1/16) (8.4 M edges).  Foster's
    theorem (the resistances sum to n - 1) holds for the estimate to its
    sampling error; the sparsified graph has ceil(n ln n) edges, contains a
    spanning tree (connected) and is reproducible."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    g = G.config_er()
    rp, ci = _dev(g.row_ptr), _dev(g.col_idx)
    R, its = gumap.effective_resistance(rp, ci, q=32, seed=7, tol=1e-8, flags=gumap.CSR_SORTED)
    Rn = R.cpu().numpy()
    print("er16k: m %d, CG iterations %d, sum R %.2f (n - 1 = %d)" % (len(Rn), its, Rn.sum(), g.n - 1), flush=True)
    assert abs(Rn.sum() - (g.n - 1)) < 0.01 * (g.n - 1)
    assert np.all(Rn > 0) and np.all(Rn <= 1.0 + 1e-6 + 5 * np.sqrt(2 / 32))
    srp, scol = gumap.sparsify_select(rp, ci, R, flags=gumap.CSR_SORTED)
    target = int(np.ceil(g.n * np.log(g.n)))
    assert scol.numel() == 2 * target
    A = sp.csr_matrix((np.ones(scol.numel()), scol.cpu().numpy(), srp.cpu().numpy()), shape=(g.n, g.n))
    assert connected_components(A)[0] == 1
    assert (A != A.T).nnz == 0
    srp2, scol2 = gumap.sparsify_select(rp, ci, R, flags=gumap.CSR_SORTED)
    assert np.array_equal(scol.cpu().numpy(), scol2.cpu().numpy())


def test_sparsify_degenerate_inputs(gumap):
    """No edges at all, and a graph whose only edges form a tree (every edge
    kept, resistance exactly 1)."""
    g = G.empty(7)
    R, its = gumap.effective_resistance(_dev(g.row_ptr), _dev(np.zeros(1, np.int32)), flags=gumap.CSR_SORTED)
    assert R.numel() == 0 and its == 0
    rp, col = gumap.sparsify_select(_dev(g.row_ptr), _dev(np.zeros(1, np.int32)), _dev(np.zeros(1)),
                                    flags=gumap.CSR_SORTED)
    assert col.numel() == 0 and int(rp.abs().sum()) == 0
    g = G.star(25)
    R, _ = gumap.effective_resistance(_dev(g.row_ptr), _dev(g.col_idx), q=4, flags=gumap.CSR_SORTED)
    assert np.allclose(R.cpu().numpy(), 1.0, atol=1e-8)
    rp, col = gumap.sparsify_select(_dev(g.row_ptr), _dev(g.col_idx), R, target=3, flags=gumap.CSR_SORTED)
    assert np.array_equal(rp.cpu().numpy(), g.row_ptr) and np.array_equal(col.cpu().numpy(), g.col_idx)
