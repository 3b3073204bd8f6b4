"""The all-source autotuner (gumap_knn_build_tune) and the settings it picks
among, through the C-ABI on the GPU: every candidate of every setting gives
the oracle's rows (ids and hops bit-exact, hop matrices bit-exact), the tuner
writes the oracle's rows, records a valid pick that later plain calls use,
and persists it in the JSON cache."""
import json
import os
import sys

import numpy as np
import pytest

import graphgen as G
import oracle as O

sys.path.insert(0, os.path.dirname(__file__))
from gpu_util import first_mismatch, to_dev  # noqa: E402

pytestmark = pytest.mark.gpu


def _check(gm, g, k, sources, hop_matrix, tune=False):
    import torch
    rp, ci = to_dev(g)
    src_t = None if sources is None else torch.from_numpy(np.asarray(sources, np.int32)).cuda()
    print("n=%d k=%d rows=%s hm=%s tune=%s" % (g.n, k, "all" if sources is None else len(sources), hop_matrix,
                                               tune), flush=True)
    if tune:
        ids, hops, hm, pick = gm.knn_build_tune(rp, ci, k, sources=src_t, hop_matrix=hop_matrix,
                                                flags=gm.CSR_SORTED)
    else:
        ids, hops, hm = gm.knn_build(rp, ci, k, sources=src_t, hop_matrix=hop_matrix, flags=gm.CSR_SORTED)
        pick = None
    oi, oh, ohm = O.knn_build(g, k, sources=sources, hop_matrix=hop_matrix)
    assert np.array_equal(ids.cpu().numpy(), oi), first_mismatch(ids.cpu().numpy(), oi)
    assert np.array_equal(hops.cpu().numpy(), oh), first_mismatch(hops.cpu().numpy(), oh)
    if hop_matrix:
        assert np.array_equal(hm.cpu().numpy(), ohm), first_mismatch(hm.cpu().numpy(), ohm)
    return pick


@pytest.mark.parametrize("heavy", ["32", "128", "512", "9"])
def test_heavy_degree_invariance(gumap, heavy, monkeypatch):
    """Every heavy-degree threshold the tuner tries (and a very low one that
    makes most vertices heavy) gives the oracle's rows: whole-wave searches
    of many vertices, with and without hop rows, several widths."""
    monkeypatch.setenv("GUMAP_FUSED", "0")
    monkeypatch.setenv("GUMAP_HEAVY_DEGREE", heavy)
    for g, words in ((G.ba(3001, 4, 81), 8), (G.star(900), 2), (G.sbm(2200, 20, 82), 4), (G.rgg(1500, 10, 83), 1)):
        monkeypatch.setenv("GUMAP_FORCE_WORDS", str(words))
        _check(gumap, g, 15, None, True)
        _check(gumap, g, 6, G.sample_sources(g.n, 200, 84), False)


def test_tune_picks_valid_setting_and_plain_calls_use_it(gumap, monkeypatch, tmp_path):
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("GUMAP_AUTOTUNE_CACHE", str(cache))
    gumap.gumap_autotune_clear()
    cases = ((G.ba(4000, 4, 91), 15, None, True), (G.rgg(3000, 8, 92), 10, G.sample_sources(3000, 700, 93), False),
             (G.grid_2d(24, 24), 15, None, True))
    for g, k, src, hm in cases:
        pick = _check(gumap, g, k, src, hm, tune=True)
        assert pick["fused"] in (0, 1)
        assert pick["words"] in (1, 2, 4, 8) and pick["level_verts"] in (1, 2, 4, 8)
        assert pick["first_level"] in (0, 1) and pick["heavy_degree"] in (0, 32, 128, 512)
        assert pick["hist_levels"] in (0, 15) and pick["push_levels"] in (0, 2)
        assert pick["candidates"] >= 2 and 0.0 < pick["best_ms"] <= pick["default_ms"]
        rows = g.n if src is None else len(src)
        got = gumap.gumap_build_tuning_lookup(g.n, g.nnz, rows, k, hm)
        assert got is not None and {x: got[x] for x in got if not x.endswith("_ms")} == \
            {x: pick[x] for x in pick if not x.endswith("_ms")}
        # a plain call of the same shape now runs with the pick: same rows
        _check(gumap, g, k, src, hm)
    data = json.loads(cache.read_text())
    assert data["format"] == "gumap-build-tuning" and len(data["entries"]) == len(cases)
    # read back from the file into an empty table
    gumap.gumap_autotune_clear()
    assert gumap.gumap_build_tuning_lookup(4000, cases[0][0].nnz, 4000, 15, True) is None
    gumap.gumap_autotune_cache_load(str(cache))
    assert gumap.gumap_build_tuning_lookup(4000, cases[0][0].nnz, 4000, 15, True) is not None
    gumap.gumap_autotune_clear()


def test_tune_errors(gumap):
    import ctypes
    g = gumap.gumap_graph(4, 0, None, None, 0)
    assert gumap.lib.gumap_knn_build_tune(ctypes.byref(g), 3, None, 0, None, None, None, None, None) == gumap.EINVAL
    out = gumap.gumap_build_tuning()
    assert gumap.lib.gumap_knn_build_tune(None, 3, None, 0, None, None, None, None, ctypes.byref(out)) == gumap.EINVAL
    assert gumap.lib.gumap_knn_build_tune(ctypes.byref(g), 0, None, 0, None, None, None, None,
                                          ctypes.byref(out)) == gumap.EINVAL
