"""The C-ABI library loads, exports every declared symbol, and rejects bad
arguments on the host (no GPU needed: these paths return before any device
call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = "".join(open(os.path.join(ROOT, "include", f)).read()
                   for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h"))
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gumap_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol(gumap):
    names = declared_symbols()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(gumap.lib, n)]
    assert not missing, missing


def test_struct_layouts_match_header(gumap):
    assert ctypes.sizeof(gumap.gumap_graph) == 32
    assert ctypes.sizeof(gumap.gumap_batch) == 64
    assert ctypes.sizeof(gumap.gumap_batch_tuning) == 24
    assert ctypes.sizeof(gumap.gumap_layout_params) == 72
    assert gumap.gumap_layout_params.parts.offset == 64
    assert ctypes.sizeof(gumap.gumap_spectral_params) == 24
    assert ctypes.sizeof(gumap.gumap_build_tuning) == 40
    assert gumap.gumap_build_tuning.best_ms.offset == 32


def test_host_side_argument_errors(gumap):
    lib = gumap.lib
    g = gumap.gumap_graph(4, 0, None, None, 0)
    # NULL graph
    assert lib.gumap_knn_build(None, 5, None, 0, None, None, None, None) == gumap.EINVAL
    assert "NULL" in gumap.last_error()
    # k outside [1, 254]
    for k in (0, -3, 255, 1000):
        assert lib.gumap_knn_partial(ctypes.byref(g), k, None, None, None) == gumap.EINVAL
    # row_ptr missing for n > 0
    assert lib.gumap_knn_partial(ctypes.byref(g), 5, None, None, None) == gumap.EINVAL
    bad = gumap.gumap_graph(-1, 0, None, None, 0)
    assert lib.gumap_knn_partial(ctypes.byref(bad), 5, None, None, None) == gumap.EINVAL
    unknown = gumap.gumap_graph(0, 0, None, None, 0x80)
    assert lib.gumap_knn_partial(ctypes.byref(unknown), 5, None, None, None) == gumap.EINVAL
    # empty graph is a successful no-op
    empty = gumap.gumap_graph(0, 0, None, None, 0)
    assert lib.gumap_knn_partial(ctypes.byref(empty), 5, None, None, None) == gumap.OK
    assert lib.gumap_knn_build(ctypes.byref(empty), 5, None, 0, None, None, None, None) == gumap.OK
    # membership: negative rows, bad k, zero rows
    assert lib.gumap_membership(-1, 5, None, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_membership(3, 0, None, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_membership(0, 5, None, None, None, None, None) == gumap.OK
    assert lib.gumap_membership(3, 5, None, None, None, None, None) == gumap.EINVAL
    # batch
    assert lib.gumap_knn_partial_batch(None, 5, None, None, None, None, None, None) == gumap.EINVAL
    b = gumap.gumap_batch(0, 0, 0, None, None, None, None, 0)
    assert lib.gumap_knn_partial_batch(ctypes.byref(b), 5, None, None, None, None, None, None) == gumap.OK
    assert lib.gumap_knn_partial_batch(ctypes.byref(b), 0, None, None, None, None, None, None) == gumap.EINVAL
    plan = ctypes.c_void_p()
    unsorted = gumap.gumap_batch(0, 0, 0, None, None, None, None, 0)
    assert lib.gumap_batch_plan_create(ctypes.byref(unsorted), 5, None, None, None, None, None, None,
                                       ctypes.byref(plan)) == gumap.EINVAL
    assert lib.gumap_batch_plan_tuning(None, None) == gumap.EINVAL


def test_layout_entry_points_reject_bad_arguments(gumap):
    lib = gumap.lib
    nnz = ctypes.c_int64(7)
    assert lib.gumap_fuzzy_union(4, 5, None, None, None, None, None, 0, None, None) == gumap.EINVAL
    assert lib.gumap_fuzzy_union(-1, 5, None, None, None, None, None, 0, ctypes.byref(nnz), None) == gumap.EINVAL
    assert nnz.value == 0
    assert lib.gumap_fuzzy_union(4, 0, None, None, None, None, None, 0, ctypes.byref(nnz), None) == gumap.EINVAL
    assert lib.gumap_fuzzy_union(4, 255, None, None, None, None, None, 0, ctypes.byref(nnz), None) == gumap.EINVAL
    assert lib.gumap_fuzzy_union(0, 5, None, None, None, None, None, 0, ctypes.byref(nnz), None) == gumap.EINVAL
    assert lib.gumap_edge_shuffle(-1, None, None, None, 0, 0, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_edge_shuffle(3, None, None, None, 0, 0, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_edge_shuffle(3, None, None, None, 2**31, 0, None, None, None, None) == gumap.EINVAL
    p = gumap.layout_params(t=10)
    assert lib.gumap_grad_sample(2, None, 1, None, None, None, None, 0, 1, None) == gumap.EINVAL
    assert lib.gumap_grad_sample(0, None, 0, None, None, None, ctypes.byref(p), 0, 10, None) == gumap.OK
    assert lib.gumap_grad_sample(0, None, 3, None, None, None, ctypes.byref(p), 0, 10, None) == gumap.EINVAL
    assert lib.gumap_grad_sample(2, None, 3, None, None, None, ctypes.byref(p), 0, 11, None) == gumap.EINVAL
    assert lib.gumap_grad_sample(2, None, 3, None, None, None, ctypes.byref(p), 5, 4, None) == gumap.EINVAL
    assert lib.gumap_grad_sample(2, None, 3, None, None, None, ctypes.byref(p), 4, 4, None) == gumap.OK
    assert lib.gumap_grad_sample(2, None, 3, None, None, None, ctypes.byref(p), 0, 4, None) == gumap.EINVAL
    bad = gumap.layout_params(t=0)
    assert lib.gumap_grad_sample(2, None, 3, None, None, None, ctypes.byref(bad), 0, 0, None) == gumap.EINVAL
    neg = gumap.layout_params(neg=-1)
    assert lib.gumap_grad_sample(2, None, 3, None, None, None, ctypes.byref(neg), 0, 1, None) == gumap.EINVAL


def test_spectral_layout_rejects_bad_arguments(gumap):
    lib = gumap.lib
    assert lib.gumap_spectral_layout(2, None, None, None, None, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_spectral_layout(-5, None, None, None, None, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_spectral_layout(10, None, None, None, None, None, None, None, None) == gumap.EINVAL
    assert "NULL" in gumap.last_error()


def test_sparsify_entry_points_reject_bad_arguments(gumap):
    lib = gumap.lib
    g = gumap.gumap_graph(4, 6, None, None, 0)
    m = ctypes.c_int64(5)
    its = ctypes.c_int32(0)
    nnz = ctypes.c_int32(3)
    assert lib.gumap_effective_resistance(None, 8, 0, 1e-8, 10, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_effective_resistance(ctypes.byref(g), 0, 0, 1e-8, 10, None, ctypes.byref(m), None,
                                          None) == gumap.EINVAL
    assert lib.gumap_effective_resistance(ctypes.byref(g), 2000, 0, 1e-8, 10, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_effective_resistance(ctypes.byref(g), 8, 0, 0.0, 10, None, None, None, None) == gumap.EINVAL
    empty = gumap.gumap_graph(0, 0, None, None, 0)
    assert lib.gumap_effective_resistance(ctypes.byref(empty), 8, 0, 1e-8, 10, None, ctypes.byref(m),
                                          ctypes.byref(its), None) == gumap.OK
    assert m.value == 0
    assert lib.gumap_sparsify_select(ctypes.byref(g), None, 0, None, None, None, None) == gumap.EINVAL
    assert lib.gumap_sparsify_select(ctypes.byref(empty), None, 0, None, None, ctypes.byref(nnz), None) == gumap.OK
    assert nnz.value == 0


def test_python_names_mirror_c_entry_points(gumap):
    for name in ("gumap_knn_build", "gumap_knn_partial", "gumap_membership", "gumap_knn_partial_batch",
                 "gumap_fuzzy_union", "gumap_edge_shuffle", "gumap_grad_sample", "gumap_spectral_layout",
                 "gumap_effective_resistance", "gumap_sparsify_select"):
        assert callable(getattr(gumap, name))


def test_autotune_cache_round_trip_and_buckets(gumap, tmp_path):
    """The tuning cache is JSON that the library reads back; picks are found
    by the shape bucket of a call (floor(log2) of n, mean degree, sources
    and k, hop rows or not), and a malformed or foreign file is refused
    without touching the recorded picks.  Host only."""
    import json
    gumap.gumap_autotune_clear()
    assert gumap.gumap_build_tuning_lookup(100000, 800000, 4096, 15, True) is None
    entry = {"n_log2": 16, "deg_log2": 3, "rows_log2": 12, "k_log2": 3, "hop_matrix": 1, "fused": 0, "words": 4,
             "level_verts": 2, "first_level": 1, "heavy_degree": 128, "hist_levels": 15, "push_levels": 0,
             "candidates": 14, "best_ms": 0.9, "default_ms": 1.0}
    path = tmp_path / "tune.json"
    path.write_text(json.dumps({"format": "gumap-build-tuning", "version": 1, "entries": [entry]}))
    assert gumap.gumap_autotune_cache_load(str(path)) == gumap.OK
    # n in [2^16, 2^17), nnz / n in [8, 16), sources in [2^12, 2^13), k in [8, 16), hop rows
    got = gumap.gumap_build_tuning_lookup(100000, 800000, 4096, 15, True)
    assert got is not None and got["words"] == 4 and got["level_verts"] == 2 and got["heavy_degree"] == 128
    assert gumap.gumap_build_tuning_lookup(131071, 131071 * 15, 8191, 8, True)["words"] == 4
    assert gumap.gumap_build_tuning_lookup(100000, 800000, 4096, 15, False) is None
    assert gumap.gumap_build_tuning_lookup(100000, 800000, 8192, 15, True) is None
    assert gumap.gumap_build_tuning_lookup(100000, 1600000, 4096, 15, True) is None
    assert gumap.gumap_build_tuning_lookup(100000, 800000, 4096, 16, True) is None
    # written back by the library, read again: the same entry
    out = tmp_path / "again.json"
    assert gumap.gumap_autotune_cache_save(str(out)) == gumap.OK
    back = json.loads(out.read_text())
    assert back["format"] == "gumap-build-tuning" and len(back["entries"]) == 1
    assert {k2: back["entries"][0][k2] for k2 in entry if k2 not in ("best_ms", "default_ms")} == \
        {k2: v for k2, v in entry.items() if k2 not in ("best_ms", "default_ms")}
    # refused: not a cache, a setting out of range, a missing field, a missing file
    bad = tmp_path / "bad.json"
    for text in ('{"entries": []}',
                 json.dumps({"format": "gumap-build-tuning", "entries": [dict(entry, words=3)]}),
                 json.dumps({"format": "gumap-build-tuning", "entries": [{k2: v for k2, v in entry.items()
                                                                           if k2 != "push_levels"}]})):
        bad.write_text(text)
        with pytest.raises(gumap.GumapError):
            gumap.gumap_autotune_cache_load(str(bad))
    with pytest.raises(gumap.GumapError):
        gumap.gumap_autotune_cache_load(str(tmp_path / "missing.json"))
    assert gumap.gumap_build_tuning_lookup(100000, 800000, 4096, 15, True)["words"] == 4
    with pytest.raises(gumap.GumapError):
        gumap.gumap_build_tuning_lookup(-1, 0, 0, 15, True)
    gumap.gumap_autotune_clear()
    assert gumap.gumap_build_tuning_lookup(100000, 800000, 4096, 15, True) is None
