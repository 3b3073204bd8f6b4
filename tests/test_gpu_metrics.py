"""GPU parity of the drawing quality metrics (Sec. 5.1) against the oracle.

Stress is an FP64 sum of many terms whose order differs between the GPU
(per-block partial sums) and the oracle (per-row loops): the sums agree to
1e-9 relative (observed ~1e-14); pair counts are exact."""
import os
import sys

import numpy as np
import pytest

import graphgen as G
import oracle as O

sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import to_dev  # noqa: E402

pytestmark = pytest.mark.gpu

REL = 1e-9


def _layout(n, seed, scale=10.0):
    rng = np.random.default_rng(seed)
    return (rng.random((n, 2)) * scale).astype(np.float32)


def _check(gumap, g, xy, sources=None, flags=None):
    import torch
    rp, ci = to_dev(g)
    dxy = torch.from_numpy(xy).cuda()
    src = None if sources is None else torch.from_numpy(np.asarray(sources, dtype=np.int32)).cuda()
    s, p = gumap.stress(rp, ci, dxy, sources=src, flags=gumap.CSR_SORTED if flags is None else flags)
    os_, op = O.stress(g, xy, sources=sources)
    assert p == op
    assert s == pytest.approx(os_, rel=REL, abs=1e-12)
    return s, p


def _family():
    return [("ba", G.ba(3000, 3, 11)), ("rgg", G.rgg(2500, 8, 12)), ("sbm", G.sbm(2000, 10, 13)),
            ("grid", G.grid_2d(30, 41)), ("star", G.star(200)), ("complete", G.complete(70)),
            ("union", G.disjoint_union([G.path(40), G.cycle(33), G.empty(3), G.star(9)])),
            ("er", G.er(1500, 0.01, 14))]


@pytest.mark.parametrize("name,g", _family(), ids=[n for n, _ in _family()])
def test_stress_all_sources(gumap, name, g):
    print("stress", name, g.n, flush=True)
    _check(gumap, g, _layout(g.n, 21))


def test_stress_sources_with_repeats(gumap):
    g = G.rgg(4000, 7, 31)
    src = np.concatenate([G.sample_sources(g.n, 500, 32), [5, 5, 17, 3999, 0, 17]]).astype(np.int32)
    _check(gumap, g, _layout(g.n, 33), sources=src)


@pytest.mark.parametrize("c", [1.0, 2.0, 0.5])
def test_stress_scaled_path_closed_form(gumap, c):
    n = 200
    xy = np.stack([c * np.arange(n), np.zeros(n)], 1).astype(np.float32)
    s, p = _check(gumap, G.path(n), xy)
    assert p == n * (n - 1)
    assert s == pytest.approx((1 - c) ** 2 * p, rel=1e-12, abs=1e-9)


@pytest.mark.parametrize("words", [1, 2, 4, 8])
def test_stress_bitset_width_invariance(gumap, monkeypatch, words):
    monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
    g = G.sbm(3000, 9, 41)
    _check(gumap, g, _layout(g.n, 42), sources=G.sample_sources(g.n, 900, 43))


def test_stress_unsorted_input(gumap):
    g = G.dirty(G.ba(2000, 4, 51), 52)
    import torch
    rp, ci = to_dev(g)
    xy = _layout(g.n, 53)
    s, p = gumap.stress(rp, ci, torch.from_numpy(xy).cuda(), flags=0)
    os_, op = O.stress(g, xy)
    assert p == op and s == pytest.approx(os_, rel=REL)


def test_stress_errors(gumap):
    import torch
    g = G.path(300)   # hop 299 does not fit the uint8 hop range
    rp, ci = to_dev(g)
    xy = torch.zeros((g.n, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(gumap.GumapError) as ei:
        gumap.stress(rp, ci, xy, flags=gumap.CSR_SORTED)
    assert ei.value.status == gumap.ERANGE
    g = G.path(10)
    rp, ci = to_dev(g)
    gr = gumap.make_graph(rp, ci, flags=gumap.CSR_SORTED)
    with pytest.raises(gumap.GumapError) as ei:
        gumap.gumap_stress(gr, None, None, 0)
    assert ei.value.status == gumap.EINVAL
    bad = torch.tensor([3, 10], dtype=torch.int32, device="cuda")
    with pytest.raises(gumap.GumapError) as ei:
        gumap.gumap_stress(gr, torch.zeros((10, 2), device="cuda"), bad, 2)
    assert ei.value.status == gumap.EINVAL
    empty = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert gumap.stress(rp, ci, torch.zeros((10, 2), device="cuda"), sources=empty) == (0.0, 0)


def test_stress_ba100k_sampled_sources(gumap):
    """The BA workload at full size from 256 of its sampled sources."""
    g = G.config_ba()
    src = G.config_ba_sources()[::16].copy()
    print("ba100k stress", len(src), flush=True)
    _check(gumap, g, _layout(g.n, 61, scale=100.0), sources=src)
