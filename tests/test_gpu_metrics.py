"""GPU parity of the drawing quality metrics (Sec. 4.1.3) against the oracle.

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


# ------------------------------------------------ neighbourhood preservation --

def _np_check(gumap, g, xy, r=2, vertices=None, flags=None):
    import torch
    rp, ci = to_dev(g)
    dxy = torch.from_numpy(np.ascontiguousarray(xy, dtype=np.float32)).cuda()
    vt = None if vertices is None else torch.from_numpy(np.asarray(vertices, dtype=np.int32)).cuda()
    score, ball = gumap.neighborhood(rp, ci, dxy, r=r, vertices=vt,
                                     flags=gumap.CSR_SORTED if flags is None else flags)
    oscore, oball = O.neighborhood_scores(g, xy, r, vertices=vertices)
    score, ball = score.cpu().numpy(), ball.cpu().numpy()
    assert np.array_equal(ball, oball)
    # integer counts decide every score: equal to the last bit (NaN where undefined)
    assert np.array_equal(np.isnan(score), np.isnan(oscore))
    ok = ~np.isnan(oscore)
    assert np.array_equal(score[ok], oscore[ok]), np.flatnonzero(score[ok] != oscore[ok])[:5]
    return score


@pytest.mark.parametrize("name,g", _family(), ids=[n for n, _ in _family()])
def test_neighborhood_random_drawings(gumap, name, g):
    print("neighborhood", name, g.n, flush=True)
    _np_check(gumap, g, _layout(g.n, 71))
    # coarse integer coordinates: many exact distance ties, decided by id
    _np_check(gumap, g, np.floor(_layout(g.n, 72, scale=6.0)), r=1)


def test_neighborhood_lattice_and_collapsed(gumap):
    g = G.grid_2d(20, 33)
    xy = np.array([[v % 33, v // 33] for v in range(g.n)], dtype=np.float32)
    assert np.all(_np_check(gumap, g, xy) == 1.0)
    c = G.cycle(300)
    _np_check(gumap, c, np.zeros((c.n, 2), dtype=np.float32))
    _np_check(gumap, G.complete(50), _layout(50, 73))


def test_neighborhood_vertices_and_unsorted(gumap):
    g = G.rgg(5000, 9, 81)
    verts = np.concatenate([G.sample_sources(g.n, 400, 82), [7, 7, 4999, 0]]).astype(np.int32)
    _np_check(gumap, g, _layout(g.n, 83), vertices=verts)
    d = G.dirty(G.sbm(2500, 8, 84), 85)
    _np_check(gumap, d, _layout(d.n, 86), flags=0)


def test_neighborhood_errors(gumap):
    import torch
    g = G.path(10)
    rp, ci = to_dev(g)
    gr = gumap.make_graph(rp, ci, flags=gumap.CSR_SORTED)
    xy = torch.zeros((10, 2), dtype=torch.float32, device="cuda")
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    for r, x, verts, nv in ((3, xy, None, 0), (2, None, None, 0),
                            (2, xy, torch.tensor([1, 10], dtype=torch.int32, device="cuda"), 2)):
        with pytest.raises(gumap.GumapError) as ei:
            gumap.gumap_neighborhood(gr, x, r, verts, nv, out)
        assert ei.value.status == gumap.EINVAL


def test_neighborhood_ba100k_sampled(gumap):
    g = G.config_ba()
    verts = G.config_ba_sources()[::16].copy()
    print("ba100k neighborhood", len(verts), flush=True)
    _np_check(gumap, g, _layout(g.n, 91, scale=100.0), vertices=verts)


def test_stress_in_rounds(gumap, monkeypatch):
    """A BFS memory budget below one source group's state makes every group a
    round of its own; the stress sums of all rounds equal the oracle's."""
    monkeypatch.setenv("GUMAP_BFS_BUDGET_MB", "1")
    monkeypatch.setenv("GUMAP_FUSED", "0")
    for g, words, src in ((G.ba(3001, 4, 61), 8, None), (G.rgg(2500, 8, 62), 2, G.sample_sources(2500, 700, 63))):
        monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
        print("stress in rounds", g.n, words, flush=True)
        _check(gumap, g, _layout(g.n, 64), sources=src)
