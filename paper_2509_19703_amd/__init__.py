"""Python binding of libgumap (the HIP/gfx950 BFS-kNN library).

Argument marshalling only: every step runs in the library's kernels.  The
functions named ``gumap_*`` mirror the C entry points of ``include/gumap.h``
one to one and take torch device tensors (or None) where the C call takes
device pointers; the lower-case helpers allocate the outputs and return
them.  Importing this package never touches the GPU; the library must have
been built (``__graft_entry__.build()``) or the import fails loudly.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgumap.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "gumap.h")

OK, PENDING = 0, 1
EINVAL, EGRAPH, ERANGE, ENOMEM, EDEVICE, E2BIG, ENOTFOUND = -1, -2, -3, -4, -5, -6, -7
CSR_SORTED, VALIDATE = 1, 2
MAX_K = 254
SERVER_NO_DEVICE = 1

_STATUS_NAMES = {0: "OK", 1: "PENDING", -1: "EINVAL", -2: "EGRAPH", -3: "ERANGE", -4: "ENOMEM",
                 -5: "EDEVICE", -6: "E2BIG", -7: "ENOTFOUND"}


class GumapError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS_NAMES.get(status, "?"), status, msg))
        self.status = status


class gumap_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class gumap_batch_tuning(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("chunk", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("candidates", ctypes.c_int32), ("best_ms", ctypes.c_float), ("default_ms", ctypes.c_float)]


class gumap_build_tuning(ctypes.Structure):
    _fields_ = [("fused", ctypes.c_int32), ("words", ctypes.c_int32), ("level_verts", ctypes.c_int32),
                ("first_level", ctypes.c_int32), ("heavy_degree", ctypes.c_int32), ("hist_levels", ctypes.c_int32),
                ("push_levels", ctypes.c_int32), ("candidates", ctypes.c_int32), ("best_ms", ctypes.c_float),
                ("default_ms", ctypes.c_float)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


class gumap_layout_params(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("beta", ctypes.c_double), ("gamma", ctypes.c_double),
                ("alpha0", ctypes.c_double), ("samp", ctypes.c_double), ("window", ctypes.c_int64),
                ("neg", ctypes.c_int32), ("t", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("parts", ctypes.c_int32), ("pad", ctypes.c_int32)]


class gumap_spectral_params(ctypes.Structure):
    _fields_ = [("max_steps", ctypes.c_int32), ("pad", ctypes.c_int32), ("tol", ctypes.c_double),
                ("seed", ctypes.c_uint64)]


# UMAP's curve parameters for min_dist 0.1 and spread 1 (its default fit of
# 1 / (1 + a d^(2b)) to the target membership curve of the drawing).
# Synchronous parts per GradSample window when the parameters leave it 0
# (GUMAP_LAYOUT_DEFAULT_PARTS of the header).
LAYOUT_DEFAULT_PARTS = 4

UMAP_A = 1.5769434603113077
UMAP_B = 0.8950608781227859


class gumap_batch(ctypes.Structure):
    _fields_ = [("n_graphs", ctypes.c_int32), ("total_vertices", ctypes.c_int64),
                ("total_nnz", ctypes.c_int64), ("vtx_offset", ctypes.c_void_p),
                ("edge_offset", ctypes.c_void_p), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("flags", ctypes.c_uint32)]


class gumap_job(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int32), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("k", ctypes.c_int32), ("want_weights", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class gumap_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("nbr_ids", ctypes.c_void_p), ("nbr_hops", ctypes.c_void_p), ("weights", ctypes.c_void_p),
                ("rho", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("t_submit_ns", ctypes.c_uint64),
                ("t_admit_ns", ctypes.c_uint64), ("t_start_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64)]


class gumap_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("failed", ctypes.c_uint64),
                ("iterations", ctypes.c_uint64), ("queued", ctypes.c_uint64), ("running", ctypes.c_uint64),
                ("resident_bytes", ctypes.c_uint64), ("peak_resident_bytes", ctypes.c_uint64),
                ("budget_bytes", ctypes.c_uint64)]


def _hip_runtimes() -> list[str]:
    try:
        with open("/proc/self/maps") as f:
            return sorted({ln.split()[-1] for ln in f if "libamdhip64" in ln})
    except OSError:
        return []


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError("libgumap.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    # torch ships its own HIP runtime (SONAME libamdhip64.so.7).  Loading torch
    # first makes the dynamic loader resolve libgumap's libamdhip64.so.7 to that
    # same copy, so device pointers and streams are shared by one runtime.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise ImportError("two HIP runtimes are loaded (%s); import torch before loading libgumap"
                          % ", ".join(runtimes))
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    G = ctypes.POINTER(gumap_graph)
    B = ctypes.POINTER(gumap_batch)
    lib.gumap_csr_canonicalize.argtypes = [G, vp, vp, ctypes.POINTER(i32), vp]
    lib.gumap_csr_canonicalize.restype = ctypes.c_int
    lib.gumap_knn_build.argtypes = [G, i32, vp, i32, vp, vp, vp, vp]
    lib.gumap_knn_partial.argtypes = [G, i32, vp, vp, vp]
    lib.gumap_knn_build_tune.argtypes = [G, i32, vp, i32, vp, vp, vp, vp, ctypes.POINTER(gumap_build_tuning)]
    lib.gumap_knn_build_tune.restype = ctypes.c_int
    lib.gumap_build_tuning_lookup.argtypes = [i32, i64, i64, i32, ctypes.c_int, ctypes.POINTER(gumap_build_tuning)]
    lib.gumap_build_tuning_lookup.restype = ctypes.c_int
    lib.gumap_autotune_cache_load.argtypes = [ctypes.c_char_p]
    lib.gumap_autotune_cache_load.restype = ctypes.c_int
    lib.gumap_autotune_cache_save.argtypes = [ctypes.c_char_p]
    lib.gumap_autotune_cache_save.restype = ctypes.c_int
    lib.gumap_autotune_clear.argtypes = []
    lib.gumap_autotune_clear.restype = None
    lib.gumap_stress.argtypes = [G, vp, vp, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64), vp]
    lib.gumap_stress.restype = ctypes.c_int
    lib.gumap_neighborhood.argtypes = [G, vp, i32, vp, i32, vp, vp, vp]
    lib.gumap_neighborhood.restype = ctypes.c_int
    lib.gumap_membership.argtypes = [i32, i32, vp, vp, vp, vp, vp]
    lib.gumap_fuzzy_union.argtypes = [i32, i32, vp, vp, vp, vp, vp, i64, ctypes.POINTER(i64), vp]
    lib.gumap_edge_shuffle.argtypes = [i32, vp, vp, vp, i64, ctypes.c_uint64, vp, vp, vp, vp]
    lib.gumap_grad_sample.argtypes = [i32, vp, i64, vp, vp, vp, ctypes.POINTER(gumap_layout_params), i32, i32, vp]
    lib.gumap_effective_resistance.argtypes = [G, i32, ctypes.c_uint64, ctypes.c_double, i32, vp,
                                               ctypes.POINTER(i64), ctypes.POINTER(i32), vp]
    lib.gumap_sparsify_select.argtypes = [G, vp, i64, vp, vp, ctypes.POINTER(i32), vp]
    lib.gumap_effective_resistance.restype = ctypes.c_int
    lib.gumap_sparsify_select.restype = ctypes.c_int
    lib.gumap_spectral_layout.argtypes = [i32, vp, vp, vp, ctypes.POINTER(gumap_spectral_params), vp,
                                          ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32), vp]
    for f in (lib.gumap_fuzzy_union, lib.gumap_edge_shuffle, lib.gumap_grad_sample, lib.gumap_spectral_layout):
        f.restype = ctypes.c_int
    lib.gumap_knn_partial_batch.argtypes = [B, i32, vp, vp, vp, vp, vp, vp]
    lib.gumap_batch_plan_create.argtypes = [B, i32, vp, vp, vp, vp, vp, vp, ctypes.POINTER(vp)]
    lib.gumap_batch_plan_launch.argtypes = [vp, vp]
    lib.gumap_batch_plan_destroy.argtypes = [vp]
    lib.gumap_batch_plan_destroy.restype = None
    lib.gumap_batch_plan_tuning.argtypes = [vp, ctypes.POINTER(gumap_batch_tuning)]
    lib.gumap_batch_plan_tuning.restype = ctypes.c_int
    lib.gumap_knn_partial_noalloc.argtypes = [G, i32, vp, vp, vp]
    for f in (lib.gumap_knn_build, lib.gumap_knn_partial, lib.gumap_membership, lib.gumap_knn_partial_noalloc,
              lib.gumap_knn_partial_batch, lib.gumap_batch_plan_create, lib.gumap_batch_plan_launch):
        f.restype = ctypes.c_int
    lib.gumap_profile_enable.argtypes = [ctypes.c_int]
    lib.gumap_profile_enable.restype = None
    lib.gumap_profile_only.argtypes = [ctypes.c_char_p]
    lib.gumap_profile_only.restype = None
    lib.gumap_profile_reset.argtypes = []
    lib.gumap_profile_reset.restype = None
    lib.gumap_profile_count.argtypes = []
    lib.gumap_profile_count.restype = ctypes.c_int
    lib.gumap_profile_entry.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.gumap_profile_entry.restype = ctypes.c_int
    lib.gumap_profile_extra.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_double)]
    lib.gumap_profile_extra.restype = ctypes.c_int
    lib.gumap_last_error.argtypes = []
    lib.gumap_last_error.restype = ctypes.c_char_p
    if hasattr(lib, "gumap_server_create"):
        lib.gumap_server_create.argtypes = [ctypes.c_size_t, i32, u32, ctypes.POINTER(ctypes.c_int)]
        lib.gumap_server_create.restype = vp
        lib.gumap_submit.argtypes = [vp, ctypes.POINTER(gumap_job), ctypes.POINTER(ctypes.c_uint64)]
        lib.gumap_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(gumap_result)]
        lib.gumap_wait.argtypes = [vp, ctypes.c_uint64, i64, ctypes.POINTER(gumap_result)]
        lib.gumap_release.argtypes = [vp, ctypes.c_uint64]
        lib.gumap_server_get_stats.argtypes = [vp, ctypes.POINTER(gumap_server_stats)]
        lib.gumap_server_destroy.argtypes = [vp]
        lib.gumap_server_destroy.restype = None
        for f in (lib.gumap_submit, lib.gumap_poll, lib.gumap_wait, lib.gumap_release,
                  lib.gumap_server_get_stats):
            f.restype = ctypes.c_int
    return lib


lib = _load()


def profile_enable(on: bool = True) -> None:
    """Record HIP-event timings of the library's kernel launches (gumap_profile.h)."""
    lib.gumap_profile_enable(1 if on else 0)


def profile_only(names=None) -> None:
    """Record only the kernels named (a list or comma-separated string; None: all)."""
    if names is not None and not isinstance(names, str):
        names = ",".join(names)
    lib.gumap_profile_only(names.encode() if names else None)


def profile_reset() -> None:
    lib.gumap_profile_reset()


def profile_entries() -> dict:
    """{kernel: {"launches", "total_ms", "alg_bytes", "extra_bytes"}} recorded
    so far (extra_bytes: bytes moved beyond the algorithmic bytes, see
    gumap_profile_extra)."""
    out = {}
    for i in range(lib.gumap_profile_count()):
        name = ctypes.c_char_p()
        launches = ctypes.c_int64()
        ms = ctypes.c_double()
        b = ctypes.c_double()
        x = ctypes.c_double()
        if lib.gumap_profile_entry(i, ctypes.byref(name), ctypes.byref(launches), ctypes.byref(ms),
                                   ctypes.byref(b)) == 0 and lib.gumap_profile_extra(i, ctypes.byref(x)) == 0:
            out[name.value.decode()] = {"launches": launches.value, "total_ms": ms.value, "alg_bytes": b.value,
                                        "extra_bytes": x.value}
    return out


def last_error() -> str:
    return lib.gumap_last_error().decode()


def _check(status: int) -> int:
    if status < 0:
        raise GumapError(status, last_error())
    return status


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def make_graph(row_ptr, col_idx, n: int | None = None, flags: int = 0) -> gumap_graph:
    """gumap_graph over torch int32 device tensors (kept alive by the caller)."""
    n = int(row_ptr.shape[0]) - 1 if n is None else n
    nnz = int(col_idx.shape[0])
    return gumap_graph(n, nnz, _ptr(row_ptr) if n > 0 or row_ptr is not None else None,
                       _ptr(col_idx) if nnz > 0 else None, flags)


# ------------------------------------------------- mirrors of the C calls ---

def gumap_csr_canonicalize(graph: gumap_graph, out_row_ptr, out_col_idx, stream=None) -> int:
    """Returns the kept entry count (the C call's *out_nnz)."""
    nnz = ctypes.c_int32(0)
    _check(lib.gumap_csr_canonicalize(ctypes.byref(graph), _ptr(out_row_ptr), _ptr(out_col_idx),
                                      ctypes.byref(nnz), _stream(stream)))
    return int(nnz.value)

def gumap_knn_build(graph: gumap_graph, k: int, sources, n_sources: int, nbr_ids, nbr_hops,
                    hop_matrix=None, stream=None) -> int:
    return _check(lib.gumap_knn_build(ctypes.byref(graph), k, _ptr(sources), n_sources, _ptr(nbr_ids),
                                      _ptr(nbr_hops), _ptr(hop_matrix), _stream(stream)))


def gumap_knn_build_tune(graph: gumap_graph, k: int, sources, n_sources: int, nbr_ids, nbr_hops,
                         hop_matrix=None, stream=None) -> dict:
    """Autotune gumap_knn_build on this call (it writes the outputs); returns the pick."""
    out = gumap_build_tuning()
    _check(lib.gumap_knn_build_tune(ctypes.byref(graph), k, _ptr(sources), n_sources, _ptr(nbr_ids),
                                    _ptr(nbr_hops), _ptr(hop_matrix), _stream(stream), ctypes.byref(out)))
    return out.as_dict()


def gumap_build_tuning_lookup(n: int, nnz: int, n_sources: int, k: int, hop_matrix: bool):
    """The recorded autotuner pick for calls of this shape, or None."""
    out = gumap_build_tuning()
    found = _check(lib.gumap_build_tuning_lookup(n, nnz, n_sources, k, 1 if hop_matrix else 0, ctypes.byref(out)))
    return out.as_dict() if found == 1 else None


def gumap_autotune_cache_load(path: str) -> int:
    return _check(lib.gumap_autotune_cache_load(path.encode()))


def gumap_autotune_cache_save(path: str) -> int:
    return _check(lib.gumap_autotune_cache_save(path.encode()))


def gumap_autotune_clear() -> None:
    lib.gumap_autotune_clear()


def gumap_knn_partial(graph: gumap_graph, k: int, nbr_ids, nbr_hops, stream=None) -> int:
    return _check(lib.gumap_knn_partial(ctypes.byref(graph), k, _ptr(nbr_ids), _ptr(nbr_hops),
                                        _stream(stream)))


def gumap_knn_partial_noalloc(graph: gumap_graph, k: int, nbr_ids, nbr_hops, stream=None) -> int:
    return _check(lib.gumap_knn_partial_noalloc(ctypes.byref(graph), k, _ptr(nbr_ids), _ptr(nbr_hops),
                                                _stream(stream)))


def gumap_membership(rows: int, k: int, nbr_hops, weights, rho=None, sigma=None, stream=None) -> int:
    return _check(lib.gumap_membership(rows, k, _ptr(nbr_hops), _ptr(weights), _ptr(rho), _ptr(sigma),
                                       _stream(stream)))


def gumap_knn_partial_batch(batch: gumap_batch, k: int, nbr_ids, nbr_hops, weights=None, rho=None,
                            sigma=None, stream=None) -> int:
    return _check(lib.gumap_knn_partial_batch(ctypes.byref(batch), k, _ptr(nbr_ids), _ptr(nbr_hops),
                                              _ptr(weights), _ptr(rho), _ptr(sigma), _stream(stream)))


# Bytes of gumap_knn_partial_noalloc's fixed device scratch
# (GUMAP_NOALLOC_SCRATCH_BYTES of the header).
NOALLOC_SCRATCH_BYTES = 64 << 20


# ------------------------------------------------------ allocating helpers ---

def _torch():
    import torch
    return torch


def csr_canonicalize(row_ptr, col_idx, flags: int = 0, stream=None):
    """Canonical CSR (sorted rows, no repeats or self-loops).  Returns (row_ptr, col_idx)."""
    torch = _torch()
    g = make_graph(row_ptr, col_idx, flags=flags)
    out_rp = torch.empty(g.n + 1, dtype=torch.int32, device=row_ptr.device)
    out_col = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=row_ptr.device)
    nnz = gumap_csr_canonicalize(g, out_rp, out_col, stream)
    return out_rp, out_col[:nnz]


def knn_build(row_ptr, col_idx, k: int, sources=None, hop_matrix: bool = False, flags: int = 0,
              stream=None):
    """All-source (or listed-source) BFS kNN.  Returns (ids, hops, hop_matrix or None)."""
    torch = _torch()
    dev = row_ptr.device
    g = make_graph(row_ptr, col_idx, flags=flags)
    rows = g.n if sources is None else int(sources.shape[0])
    ids = torch.empty((rows, k), dtype=torch.int32, device=dev)
    hops = torch.empty((rows, k), dtype=torch.uint8, device=dev)
    hm = torch.empty((rows, g.n), dtype=torch.uint8, device=dev) if hop_matrix else None
    gumap_knn_build(g, k, sources, rows if sources is not None else 0, ids, hops, hm, stream)
    return ids, hops, hm


def knn_build_tune(row_ptr, col_idx, k: int, sources=None, hop_matrix: bool = False, flags: int = 0,
                   stream=None):
    """knn_build through the autotuner.  Returns (ids, hops, hop_matrix or None, pick)."""
    torch = _torch()
    dev = row_ptr.device
    g = make_graph(row_ptr, col_idx, flags=flags)
    rows = g.n if sources is None else int(sources.shape[0])
    ids = torch.empty((rows, k), dtype=torch.int32, device=dev)
    hops = torch.empty((rows, k), dtype=torch.uint8, device=dev)
    hm = torch.empty((rows, g.n), dtype=torch.uint8, device=dev) if hop_matrix else None
    pick = gumap_knn_build_tune(g, k, sources, rows if sources is not None else 0, ids, hops, hm, stream)
    return ids, hops, hm, pick


def knn_partial(row_ptr, col_idx, k: int, flags: int = 0, stream=None):
    """Truncated partial BFS kNN from every vertex.  Returns (ids, hops)."""
    torch = _torch()
    dev = row_ptr.device
    g = make_graph(row_ptr, col_idx, flags=flags)
    ids = torch.empty((g.n, k), dtype=torch.int32, device=dev)
    hops = torch.empty((g.n, k), dtype=torch.uint8, device=dev)
    gumap_knn_partial(g, k, ids, hops, stream)
    return ids, hops


def gumap_stress(g, xy, sources, n_sources, stream=None):
    """C-ABI gumap_stress; returns (sum, pairs)."""
    out_sum = ctypes.c_double(0.0)
    out_pairs = ctypes.c_int64(0)
    _check(lib.gumap_stress(ctypes.byref(g), _ptr(xy), _ptr(sources), int(n_sources), ctypes.byref(out_sum),
                            ctypes.byref(out_pairs), _stream(stream)))
    return out_sum.value, out_pairs.value


def stress(row_ptr, col_idx, xy, sources=None, flags: int = 0, stream=None):
    """Aggregated stress of the drawing xy (device float32 [n, 2]) over hop
    distances.  Returns (sum, pairs); the metric is sum / pairs."""
    g = make_graph(row_ptr, col_idx, flags=flags)
    if sources is not None and int(sources.shape[0]) == 0:
        return 0.0, 0   # an empty list, not NULL (= every vertex)
    n_src = 0 if sources is None else int(sources.shape[0])
    return gumap_stress(g, xy.contiguous(), sources, n_src, stream)


def gumap_neighborhood(g, xy, r, vertices, n_vertices, score, ball=None, stream=None) -> int:
    return _check(lib.gumap_neighborhood(ctypes.byref(g), _ptr(xy), int(r), _ptr(vertices), int(n_vertices),
                                         _ptr(score), _ptr(ball), _stream(stream)))


def neighborhood(row_ptr, col_idx, xy, r: int = 2, vertices=None, flags: int = 0, stream=None):
    """Per-vertex neighbourhood preservation of the drawing xy (device
    float32 [n, 2]).  Returns (score float64 [rows], ball int32 [rows])."""
    torch = _torch()
    g = make_graph(row_ptr, col_idx, flags=flags)
    rows = g.n if vertices is None else int(vertices.shape[0])
    score = torch.empty(rows, dtype=torch.float64, device=row_ptr.device)
    ball = torch.empty(rows, dtype=torch.int32, device=row_ptr.device)
    if rows:
        gumap_neighborhood(g, xy.contiguous(), r, vertices, rows, score, ball, stream)
    return score, ball


def membership(hops, stream=None):
    """Fuzzy-membership weights of kNN rows.  Returns (weights, rho, sigma)."""
    torch = _torch()
    rows, k = hops.shape
    w = torch.empty((rows, k), dtype=torch.float32, device=hops.device)
    rho = torch.empty(rows, dtype=torch.float32, device=hops.device)
    sigma = torch.empty(rows, dtype=torch.float32, device=hops.device)
    gumap_membership(rows, k, hops, w, rho, sigma, stream)
    return w, rho, sigma


# ------------------------------------------------------- layout step C2 --
def gumap_fuzzy_union(rows, k, ids, weights, row_ptr, col, val, cap, stream=None) -> int:
    """C-ABI gumap_fuzzy_union; returns the entry count."""
    nnz = ctypes.c_int64(0)
    st = lib.gumap_fuzzy_union(int(rows), int(k), _ptr(ids), _ptr(weights), _ptr(row_ptr), _ptr(col), _ptr(val),
                               int(cap), ctypes.byref(nnz), _stream(stream))
    _check(st)
    return nnz.value


def fuzzy_union(ids, weights, stream=None):
    """Symmetric fuzzy union of a directed kNN membership graph (ids int32
    [n, k], weights float32 [n, k] on the device).  Returns (row_ptr, col, val)."""
    torch = _torch()
    rows, k = ids.shape
    dev = ids.device
    cap = 2 * rows * k
    row_ptr = torch.empty(rows + 1, dtype=torch.int32, device=dev)
    col = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    val = torch.empty(max(cap, 1), dtype=torch.float32, device=dev)
    m = gumap_fuzzy_union(rows, k, ids.contiguous(), weights.contiguous(), row_ptr, col, val, cap, stream)
    return row_ptr, col[:m], val[:m]


def gumap_edge_shuffle(n, row_ptr, col, val, m, seed, head, tail, w, stream=None) -> int:
    return _check(lib.gumap_edge_shuffle(int(n), _ptr(row_ptr), _ptr(col), _ptr(val), int(m),
                                         ctypes.c_uint64(int(seed) & (2**64 - 1)), _ptr(head), _ptr(tail), _ptr(w),
                                         _stream(stream)))


def edge_shuffle(row_ptr, col, val, seed: int, stream=None):
    """The edge array E_k of a symmetric CSR in shuffled order: (head, tail, w)."""
    torch = _torch()
    n = int(row_ptr.shape[0]) - 1
    m = int(col.shape[0])
    dev = row_ptr.device
    head = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    tail = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    w = torch.empty(max(m, 1), dtype=torch.float32, device=dev)
    gumap_edge_shuffle(n, row_ptr, col, val, m, seed, head, tail, w, stream)
    return head[:m], tail[:m], w[:m]


def layout_params(*, a: float = UMAP_A, b: float = UMAP_B, gamma: float = 1.0, alpha0: float = 1.0,
                  samp: float = 0.9, window: int = 0, neg: int = 5, t: int = 200, seed: int = 0, parts: int = 0):
    """parts: synchronous parts per window (0 = the library's default)."""
    return gumap_layout_params(float(a), float(b), float(gamma), float(alpha0), float(samp), int(window), int(neg),
                               int(t), int(seed) & (2**64 - 1), int(parts), 0)


def gumap_grad_sample(n, xy, m, head, tail, w, params, it_begin, it_end, stream=None) -> int:
    return _check(lib.gumap_grad_sample(int(n), _ptr(xy), int(m), _ptr(head), _ptr(tail), _ptr(w),
                                        ctypes.byref(params), int(it_begin), int(it_end), _stream(stream)))


def grad_sample(xy, head, tail, w, params=None, it_begin: int = 0, it_end=None, stream=None, **kw):
    """GradSample iterations [it_begin, it_end) of a t-iteration run, in
    place on xy (device float32 [n, 2]).  params: layout_params(...) or its
    keyword arguments."""
    p = params if params is not None else layout_params(**kw)
    n = int(xy.shape[0])
    it_end = p.t if it_end is None else it_end
    assert xy.is_contiguous() and xy.dtype.itemsize == 4
    gumap_grad_sample(n, xy, int(head.shape[0]), head, tail, w, p, it_begin, it_end, stream)
    return xy


def gumap_spectral_layout(n, row_ptr, col, val, params, xy, stream=None):
    """C-ABI gumap_spectral_layout; returns (eigenvalues (2,), Lanczos steps)."""
    ev = (ctypes.c_double * 2)()
    steps = ctypes.c_int32(0)
    _check(lib.gumap_spectral_layout(int(n), _ptr(row_ptr), _ptr(col), _ptr(val),
                                     ctypes.byref(params) if params is not None else None, _ptr(xy), ev,
                                     ctypes.byref(steps), _stream(stream)))
    return (ev[0], ev[1]), steps.value


def spectral_layout(row_ptr, col, val, max_steps: int = 0, tol: float = 0.0, seed: int = 0, stream=None):
    """Spectral initial drawing of a symmetric weighted CSR on the device.
    Returns (xy float32 [n, 2], eigenvalues, steps)."""
    torch = _torch()
    n = int(row_ptr.shape[0]) - 1
    xy = torch.empty((n, 2), dtype=torch.float32, device=row_ptr.device)
    p = gumap_spectral_params(int(max_steps), 0, float(tol), int(seed) & (2**64 - 1))
    ev, steps = gumap_spectral_layout(n, row_ptr, col, val, p, xy, stream)
    return xy, ev, steps


def gumap_effective_resistance(g, q, seed, tol, max_iters, resistance, stream=None):
    """C-ABI gumap_effective_resistance; returns (edges, CG iterations)."""
    m = ctypes.c_int64(0)
    its = ctypes.c_int32(0)
    _check(lib.gumap_effective_resistance(ctypes.byref(g), int(q), ctypes.c_uint64(int(seed) & (2**64 - 1)),
                                          float(tol), int(max_iters), _ptr(resistance), ctypes.byref(m),
                                          ctypes.byref(its), _stream(stream)))
    return m.value, its.value


def effective_resistance(row_ptr, col_idx, q: int = 32, seed: int = 0, tol: float = 1e-10, max_iters: int = 2000,
                         flags: int = 0, stream=None):
    """Effective resistances of the edges (u < v, CSR order) of a symmetric
    graph.  Returns (R float64 [m], CG iterations)."""
    torch = _torch()
    g = make_graph(row_ptr, col_idx, flags=flags)
    R = torch.empty(max(g.nnz // 2, 1), dtype=torch.float64, device=row_ptr.device)
    m, its = gumap_effective_resistance(g, q, seed, tol, max_iters, R, stream)
    return R[:m], its


def gumap_sparsify_select(g, resistance, target, out_row_ptr, out_col_idx, stream=None) -> int:
    """C-ABI gumap_sparsify_select; returns the entry count of G'."""
    nnz = ctypes.c_int32(0)
    _check(lib.gumap_sparsify_select(ctypes.byref(g), _ptr(resistance), int(target), _ptr(out_row_ptr),
                                     _ptr(out_col_idx), ctypes.byref(nnz), _stream(stream)))
    return nnz.value


def sparsify_select(row_ptr, col_idx, resistance, target: int = 0, flags: int = 0, stream=None):
    """The sparsified graph G' (symmetric CSR) for the given edge resistances."""
    torch = _torch()
    g = make_graph(row_ptr, col_idx, flags=flags)
    out_rp = torch.empty(g.n + 1, dtype=torch.int32, device=row_ptr.device)
    out_col = torch.empty(max(g.nnz, 1), dtype=torch.int32, device=row_ptr.device)
    nnz = gumap_sparsify_select(g, resistance, target, out_rp, out_col, stream)
    return out_rp, out_col[:nnz]


class PackedBatch:
    """Graphs packed in the batch layout of include/gumap.h, resident on a device."""

    def __init__(self, graphs, device="cuda", flags: int = CSR_SORTED):
        import numpy as np
        torch = _torch()
        ns = np.array([g.n for g in graphs], dtype=np.int64)
        es = np.array([g.nnz for g in graphs], dtype=np.int64)
        voff = np.zeros(len(graphs) + 1, dtype=np.int64)
        eoff = np.zeros(len(graphs) + 1, dtype=np.int64)
        np.cumsum(ns, out=voff[1:])
        np.cumsum(es, out=eoff[1:])
        rp = np.concatenate([g.row_ptr for g in graphs]) if graphs else np.zeros(0, np.int32)
        col = np.concatenate([g.col_idx for g in graphs]) if graphs else np.zeros(0, np.int32)
        self.n_graphs = len(graphs)
        self.vtx_offset_host = voff
        self.edge_offset_host = eoff
        self.vtx_offset = torch.from_numpy(voff).to(device)
        self.edge_offset = torch.from_numpy(eoff).to(device)
        self.row_ptr = torch.from_numpy(rp.astype(np.int32)).to(device)
        self.col_idx = torch.from_numpy(col.astype(np.int32)).to(device)
        self.flags = flags

    @property
    def total_vertices(self) -> int:
        return int(self.vtx_offset_host[-1])

    @property
    def total_nnz(self) -> int:
        return int(self.edge_offset_host[-1])

    def struct(self) -> gumap_batch:
        return gumap_batch(self.n_graphs, self.total_vertices, self.total_nnz, _ptr(self.vtx_offset),
                           _ptr(self.edge_offset), _ptr(self.row_ptr),
                           _ptr(self.col_idx) if self.total_nnz else None, self.flags)


def knn_partial_batch(batch: PackedBatch, k: int, weights: bool = True, stream=None):
    """Batched partial BFS (+ membership).  Returns (ids, hops, weights, rho, sigma)."""
    torch = _torch()
    dev = batch.row_ptr.device
    rows = batch.total_vertices
    ids = torch.empty((rows, k), dtype=torch.int32, device=dev)
    hops = torch.empty((rows, k), dtype=torch.uint8, device=dev)
    w = torch.empty((rows, k), dtype=torch.float32, device=dev) if weights else None
    rho = torch.empty(rows, dtype=torch.float32, device=dev) if weights else None
    sigma = torch.empty(rows, dtype=torch.float32, device=dev) if weights else None
    b = batch.struct()
    gumap_knn_partial_batch(b, k, ids, hops, w, rho, sigma, stream)
    return ids, hops, w, rho, sigma


class BatchPlan:
    """Captured (HIP graph) form of knn_partial_batch on fixed buffers."""

    def __init__(self, batch: PackedBatch, k: int, weights: bool = True, stream=None):
        torch = _torch()
        dev = batch.row_ptr.device
        rows = batch.total_vertices
        self.batch = batch
        self.ids = torch.empty((rows, k), dtype=torch.int32, device=dev)
        self.hops = torch.empty((rows, k), dtype=torch.uint8, device=dev)
        self.weights = torch.empty((rows, k), dtype=torch.float32, device=dev) if weights else None
        self.rho = torch.empty(rows, dtype=torch.float32, device=dev) if weights else None
        self.sigma = torch.empty(rows, dtype=torch.float32, device=dev) if weights else None
        self._b = batch.struct()
        h = ctypes.c_void_p()
        _check(lib.gumap_batch_plan_create(ctypes.byref(self._b), k, _ptr(self.ids), _ptr(self.hops),
                                           _ptr(self.weights), _ptr(self.rho), _ptr(self.sigma),
                                           _stream(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None):
        _check(lib.gumap_batch_plan_launch(self._h, _stream(stream)))
        return self.ids, self.hops, self.weights, self.rho, self.sigma

    def tuning(self) -> dict:
        t = gumap_batch_tuning()
        _check(lib.gumap_batch_plan_tuning(self._h, ctypes.byref(t)))
        return {"lanes": t.lanes, "chunk": t.chunk, "blocks": t.blocks, "candidates": t.candidates,
                "best_ms": t.best_ms, "default_ms": t.default_ms}

    def close(self):
        if self._h:
            lib.gumap_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ serving ---

class Server:
    """Request loop of include/gumap.h (gumap_server_*): submit host CSR jobs,
    poll or wait for their results.  Results are returned as numpy copies."""

    def __init__(self, hbm_budget_bytes: int, max_slots: int = 0, flags: int = 0):
        st = ctypes.c_int(0)
        h = lib.gumap_server_create(hbm_budget_bytes, max_slots, flags, ctypes.byref(st))
        if not h:
            raise GumapError(st.value, last_error())
        self._h = ctypes.c_void_p(h)
        self._keep = {}

    def submit(self, row_ptr, col_idx, k: int, want_weights: bool = True, flags: int = CSR_SORTED) -> int:
        import numpy as np
        rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(col_idx, dtype=np.int32)
        n = int(rp.shape[0]) - 1
        job = gumap_job(n, int(ci.shape[0]), rp.ctypes.data if rp.size else None,
                        ci.ctypes.data if ci.size else None, k, 1 if want_weights else 0, flags)
        t = ctypes.c_uint64(0)
        _check(lib.gumap_submit(self._h, ctypes.byref(job), ctypes.byref(t)))
        return int(t.value)

    @staticmethod
    def _unpack(r: gumap_result) -> dict:
        import numpy as np
        n, k = r.n, r.k
        out = {"status": r.status, "n": n, "k": k, "t_submit_ns": r.t_submit_ns, "t_admit_ns": r.t_admit_ns,
               "t_start_ns": r.t_start_ns, "t_done_ns": r.t_done_ns}

        def arr(ptr, count, ctype, dtype):
            if not ptr or count == 0:
                return np.zeros(count, dtype=dtype) if ptr else None
            buf = (ctype * count).from_address(ptr)
            return np.frombuffer(buf, dtype=dtype).copy()

        out["ids"] = arr(r.nbr_ids, n * k, ctypes.c_int32, np.int32)
        out["hops"] = arr(r.nbr_hops, n * k, ctypes.c_uint8, np.uint8)
        out["weights"] = arr(r.weights, n * k, ctypes.c_float, np.float32)
        out["rho"] = arr(r.rho, n, ctypes.c_float, np.float32)
        out["sigma"] = arr(r.sigma, n, ctypes.c_float, np.float32)
        for key in ("ids", "hops", "weights"):
            if out[key] is not None:
                out[key] = out[key].reshape(n, k)
        return out

    @staticmethod
    def _times(r: gumap_result) -> dict:
        return {"status": r.status, "n": r.n, "k": r.k, "t_submit_ns": r.t_submit_ns,
                "t_admit_ns": r.t_admit_ns, "t_start_ns": r.t_start_ns, "t_done_ns": r.t_done_ns}

    def poll(self, ticket: int, copy_results: bool = True):
        r = gumap_result()
        st = lib.gumap_poll(self._h, ticket, ctypes.byref(r))
        if st == PENDING:
            return None
        if st < 0 and st != r.status:
            raise GumapError(st, last_error())
        return self._unpack(r) if copy_results else self._times(r)

    def wait(self, ticket: int, timeout_ms: int = -1, copy_results: bool = True):
        """Blocks until the job ends; with copy_results=False only status and timestamps."""
        r = gumap_result()
        st = lib.gumap_wait(self._h, ticket, timeout_ms, ctypes.byref(r))
        if st == PENDING:
            return None
        if st < 0 and st != r.status:
            raise GumapError(st, last_error())
        return self._unpack(r) if copy_results else self._times(r)

    def release(self, ticket: int) -> int:
        return _check(lib.gumap_release(self._h, ticket))

    def stats(self) -> dict:
        s = gumap_server_stats()
        _check(lib.gumap_server_get_stats(self._h, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in s._fields_}

    def close(self):
        if self._h:
            lib.gumap_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
