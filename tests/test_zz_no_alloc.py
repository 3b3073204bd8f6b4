"""gumap_knn_partial_noalloc (the partial-BFS kNN of Sec. 3.3.1, Alg. 4, with
its scratch in a fixed device array) against gumap_knn_partial, both called
through the C-ABI: ids and hops bit-exact, on two calls in a row whose second
input is smaller (the array keeps the first call's contents), plus the
oracle on the same graphs and the error paths."""
import os
import sys

import numpy as np
import pytest

import graphgen as G
import oracle as O

sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _both(gumap, g, k, flags=0):
    import torch
    rp, ci = to_dev(g)
    graph = gumap.make_graph(rp, ci, flags=flags)
    a_ids = torch.empty((g.n, k), dtype=torch.int32, device="cuda")
    a_hops = torch.empty((g.n, k), dtype=torch.uint8, device="cuda")
    b_ids = torch.full((g.n, k), 7, dtype=torch.int32, device="cuda")
    b_hops = torch.full((g.n, k), 7, dtype=torch.uint8, device="cuda")
    gumap.gumap_knn_partial(graph, k, a_ids, a_hops)
    gumap.gumap_knn_partial_noalloc(graph, k, b_ids, b_hops)
    return (a_ids.cpu().numpy(), a_hops.cpu().numpy()), (b_ids.cpu().numpy(), b_hops.cpu().numpy())


@pytest.mark.parametrize("k", [15, 30, 100])
def test_noalloc_matches_partial_two_calls_second_smaller(gumap, k):
    big = G.ba(500000, 4, 11)
    small = G.sbm(3000, 12, 12)
    for name, clean, seed in (("ba500000", big, 3), ("sbm3000", small, 4)):
        print("noalloc", name, "k", k, flush=True)
        g = G.dirty(clean, seed)                  # shuffled rows, repeats, self-loops
        (ai, ah), (bi, bh) = _both(gumap, g, k)
        assert np.array_equal(ai, bi) and np.array_equal(ah, bh), name
        oi, oh = O.knn_partial(clean, k)
        assert np.array_equal(bi, oi) and np.array_equal(bh, oh), name


def test_noalloc_sorted_input_uses_no_scratch(gumap):
    g = G.rgg(200000, 8, 13)                     # generators write canonical CSRs
    print("noalloc sorted rgg200000", flush=True)
    (ai, ah), (bi, bh) = _both(gumap, g, 15, flags=gumap.CSR_SORTED)
    assert np.array_equal(ai, bi) and np.array_equal(ah, bh)


def test_noalloc_errors(gumap):
    import torch
    g = G.grid_2d(20, 20)
    rp, ci = to_dev(g)
    ids = torch.empty((g.n, 15), dtype=torch.int32, device="cuda")
    hops = torch.empty((g.n, 15), dtype=torch.uint8, device="cuda")
    with pytest.raises(gumap.GumapError) as e:
        gumap.gumap_knn_partial_noalloc(gumap.make_graph(rp, ci, flags=gumap.VALIDATE), 15, ids, hops)
    assert e.value.status == gumap.EINVAL
    with pytest.raises(gumap.GumapError) as e:
        gumap.gumap_knn_partial_noalloc(gumap.make_graph(rp, ci), 0, ids, hops)
    assert e.value.status == gumap.EINVAL
    # an input whose canonicalisation needs more than the fixed scratch is
    # rejected before any work is enqueued (the arrays are never read)
    n, nnz = 1_000_000, 16_000_000
    huge = gumap.gumap_graph(n, nnz, rp.data_ptr(), ci.data_ptr(), 0)
    with pytest.raises(gumap.GumapError) as e:
        gumap.gumap_knn_partial_noalloc(huge, 15, ids, hops)
    assert e.value.status == gumap.E2BIG
    assert "scratch" in gumap.last_error()
    # an empty graph is a no-op; the entry still works after the errors
    gumap.gumap_knn_partial_noalloc(gumap.gumap_graph(0, 0, None, None, 0), 15, None, None)
    (ai, ah), (bi, bh) = _both(gumap, g, 15)
    assert np.array_equal(ai, bi) and np.array_equal(ah, bh)
