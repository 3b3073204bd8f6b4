"""Seeded synthetic input graphs (input side only; no kNN arithmetic here).

Every function returns a :class:`CSR` of an undirected, unweighted graph with
int32 ``row_ptr`` (n+1) and ``col_idx`` (nnz) arrays.  Generated graphs come
out canonical (rows sorted, no duplicates, no self-loops, both directions of
every edge present); :func:`dirty` perturbs a canonical graph into an
equivalent non-canonical one (shuffled rows, repeated entries, self-loops) so
that canonicalisation can be exercised.

The shapes follow the families the paper evaluates on (its dataset table:
scale-free, mesh-like and RNA-network graphs) and the dense random graph that
its complexity discussion flags as the costly case; the workload recipes that
stand in for those datasets are the ``config*`` functions at the bottom.

Both the CPU oracle's tests and the GPU path's tests and benchmark draw their
inputs from here; nothing in this module depends on either of them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 250919703
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C generators into ``libgraphgen.so`` (host code, gcc)."""
    src = os.path.join(_HERE, "graphgen.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", src, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        p32 = ctypes.POINTER(ctypes.c_int32)
        pp32 = ctypes.POINTER(p32)
        lib.gg_ba.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, pp32]
        lib.gg_ba.restype = ctypes.c_int64
        lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, pp32]
        lib.gg_er.restype = ctypes.c_int64
        lib.gg_sbm.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                               ctypes.c_uint64, pp32]
        lib.gg_sbm.restype = ctypes.c_int64
        lib.gg_rgg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, pp32]
        lib.gg_rgg.restype = ctypes.c_int64
        lib.gg_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, p32, p32, p32]
        lib.gg_csr.restype = ctypes.c_int64
        lib.gg_free.argtypes = [ctypes.c_void_p]
        lib.gg_free.restype = None
        lib.gg_mix_seed.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        lib.gg_mix_seed.restype = ctypes.c_uint64
        lib.gg_uniform.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        lib.gg_uniform.restype = ctypes.c_double
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class CSR:
    """Undirected unweighted graph in compressed sparse row form."""

    n: int
    row_ptr: np.ndarray  # int32 [n+1]
    col_idx: np.ndarray  # int32 [nnz]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def m(self) -> int:
        """Undirected edge count (canonical graphs only)."""
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def neighbors(self, v: int) -> np.ndarray:
        return self.col_idx[self.row_ptr[v]:self.row_ptr[v + 1]]


def mix_seed(base: int, index: int) -> int:
    """Seed of item ``index`` of a family seeded with ``base`` (splitmix64 mix)."""
    return int(_load().gg_mix_seed(base & (2**64 - 1), index))


def uniform(seed: int, count: int) -> np.ndarray:
    """``count`` doubles uniform in [0, 1) from the xoshiro256** stream of ``seed``."""
    out = np.empty(count, dtype=np.float64)
    if count:
        _load().gg_uniform(seed & (2**64 - 1), count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return out


def from_edges(n: int, edges: np.ndarray, name: str = "", meta: dict | None = None) -> CSR:
    """Canonical CSR from an undirected edge array of shape (m, 2)."""
    edges = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
    m = edges.shape[0]
    row_ptr = np.zeros(n + 1, dtype=np.int32)
    col = np.empty(max(2 * m, 1), dtype=np.int32)
    nnz = _load().gg_csr(n, m, _p32(edges), _p32(row_ptr), _p32(col))
    if nnz < 0:
        raise MemoryError("gg_csr failed")
    return CSR(n, row_ptr, col[:nnz].copy(), name, dict(meta or {}))


def _take_edges(count: int, ptr) -> np.ndarray:
    if count < 0:
        raise MemoryError("generator allocation failed")
    if count == 0:
        if ptr:
            _load().gg_free(ptr)
        return np.zeros((0, 2), dtype=np.int32)
    arr = np.ctypeslib.as_array(ptr, shape=(count * 2,)).copy().reshape(count, 2)
    _load().gg_free(ptr)
    return arr


# ------------------------------------------------------- random families ---

def ba(n: int, m_attach: int, seed: int) -> CSR:
    """Barabasi-Albert graph started from a clique on ``m_attach + 1`` vertices."""
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = _load().gg_ba(n, m_attach, seed & (2**64 - 1), ctypes.byref(ptr))
    return from_edges(n, _take_edges(cnt, ptr), "ba", {"m_attach": m_attach, "seed": seed})


def er(n: int, p: float, seed: int) -> CSR:
    """Erdos-Renyi G(n, p) sampled with geometric skipping."""
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = _load().gg_er(n, float(p), seed & (2**64 - 1), ctypes.byref(ptr))
    return from_edges(n, _take_edges(cnt, ptr), "er", {"p": p, "seed": seed})


def sbm(n: int, mean_degree: float, seed: int, blocks: int = 8, ratio: float = 20.0) -> CSR:
    """Stochastic block model, ``blocks`` equal blocks, p_in = ratio * p_out.

    With equal blocks the expected degree is p_in (n/B - 1) + p_out n (B-1)/B;
    p_out is solved from that for the requested mean degree.
    """
    b = blocks
    p_out = mean_degree / (ratio * (n / b - 1.0) + n * (b - 1.0) / b) if n > b else 0.0
    p_in = min(1.0, ratio * p_out)
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = _load().gg_sbm(n, b, p_in, p_out, seed & (2**64 - 1), ctypes.byref(ptr))
    return from_edges(n, _take_edges(cnt, ptr), "sbm",
                      {"blocks": b, "p_in": p_in, "p_out": p_out, "seed": seed})


def rgg(n: int, mean_degree: float, seed: int) -> CSR:
    """2-D random geometric graph in the unit square, radius sqrt(d / (pi (n-1)))."""
    radius = math.sqrt(mean_degree / (math.pi * max(n - 1, 1)))
    ptr = ctypes.POINTER(ctypes.c_int32)()
    cnt = _load().gg_rgg(n, radius, seed & (2**64 - 1), ctypes.byref(ptr))
    return from_edges(n, _take_edges(cnt, ptr), "rgg", {"radius": radius, "seed": seed})


# ---------------------------------------------------- structured graphs ---

def grid_2d(rows: int, cols: int) -> CSR:
    """rows x cols grid, vertex id = r * cols + c, 4-neighbourhood."""
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    h = np.stack([ids[:, :-1].ravel(), ids[:, 1:].ravel()], axis=1)
    v = np.stack([ids[:-1, :].ravel(), ids[1:, :].ravel()], axis=1)
    return from_edges(rows * cols, np.concatenate([h, v]), "grid", {"rows": rows, "cols": cols})


def path(n: int) -> CSR:
    e = np.stack([np.arange(n - 1), np.arange(1, n)], axis=1) if n > 1 else np.zeros((0, 2))
    return from_edges(n, e, "path")


def cycle(n: int) -> CSR:
    if n < 3:
        return path(n)
    e = np.stack([np.arange(n), (np.arange(n) + 1) % n], axis=1)
    return from_edges(n, e, "cycle")


def star(leaves: int) -> CSR:
    """Hub 0 joined to leaves 1..leaves."""
    e = np.stack([np.zeros(leaves, dtype=np.int64), np.arange(1, leaves + 1)], axis=1)
    return from_edges(leaves + 1, e, "star")


def complete(n: int) -> CSR:
    iu = np.triu_indices(n, 1)
    return from_edges(n, np.stack(iu, axis=1), "complete")


def hypercube(d: int) -> CSR:
    n = 1 << d
    v = np.arange(n)
    e = [np.stack([v, v ^ (1 << b)], axis=1) for b in range(d)]
    e = np.concatenate(e) if e else np.zeros((0, 2))
    e = e[e[:, 0] < e[:, 1]]
    return from_edges(n, e, "hypercube", {"d": d})


def complete_bipartite(a: int, b: int) -> CSR:
    """Sides {0..a-1} and {a..a+b-1}."""
    u, w = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, np.stack([u.ravel(), w.ravel()], axis=1), "kab", {"a": a, "b": b})


def empty(n: int) -> CSR:
    return from_edges(n, np.zeros((0, 2)), "empty")


def tiny_random(n: int, p: float, seed: int) -> CSR:
    """Small G(n, p) for exhaustive checks (same sampler as :func:`er`)."""
    g = er(n, p, seed)
    g.name = "tiny"
    return g


def disjoint_union(graphs: list[CSR]) -> CSR:
    edges, off = [], 0
    for g in graphs:
        src = np.repeat(np.arange(g.n), g.degrees())
        e = np.stack([src, g.col_idx.astype(np.int64)], axis=1)
        e = e[e[:, 0] < e[:, 1]] + off
        edges.append(e)
        off += g.n
    e = np.concatenate(edges) if edges else np.zeros((0, 2))
    return from_edges(off, e, "union")


def relabel(g: CSR, perm: np.ndarray) -> CSR:
    """Graph with vertex v renamed perm[v]."""
    perm = np.asarray(perm, dtype=np.int64)
    src = np.repeat(np.arange(g.n), g.degrees())
    e = np.stack([perm[src], perm[g.col_idx.astype(np.int64)]], axis=1)
    return from_edges(g.n, e[e[:, 0] < e[:, 1]], g.name + "+relabel", g.meta)


def dirty(g: CSR, seed: int, dup_frac: float = 0.2, loop_frac: float = 0.1) -> CSR:
    """Same edge set as ``g`` but rows shuffled, entries repeated, self-loops added.

    Symmetry is kept (a repeated entry (u, w) is mirrored by one (w, u)).
    """
    u = uniform(seed, 4)
    rng = np.random.default_rng(int(u[0] * 2**53))
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.col_idx.astype(np.int64)
    keep = src < dst
    und = np.stack([src[keep], dst[keep]], axis=1)
    ndup = int(len(und) * dup_frac)
    if ndup and len(und):
        und = np.concatenate([und, und[rng.integers(0, len(und), ndup)]])
    pairs = np.concatenate([und, und[:, ::-1]])
    nloop = int(g.n * loop_frac)
    if nloop and g.n:
        lv = rng.integers(0, g.n, nloop)
        pairs = np.concatenate([pairs, np.stack([lv, lv], axis=1)])
    pairs = pairs[rng.permutation(len(pairs))]
    order = np.argsort(pairs[:, 0], kind="stable")
    pairs = pairs[order]
    counts = np.bincount(pairs[:, 0], minlength=g.n) if len(pairs) else np.zeros(g.n, np.int64)
    row_ptr = np.zeros(g.n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    return CSR(g.n, row_ptr.astype(np.int32), pairs[:, 1].astype(np.int32).copy(),
               g.name + "+dirty", dict(g.meta))


def sample_sources(n: int, count: int, seed: int) -> np.ndarray:
    """``count`` distinct vertex ids drawn uniformly (partial Fisher-Yates), in draw order."""
    count = min(count, n)
    u = uniform(seed, count)
    perm = np.arange(n, dtype=np.int64)
    for i in range(count):
        j = i + int(u[i] * (n - i))
        perm[i], perm[j] = perm[j], perm[i]
    return perm[:count].astype(np.int32)


# ------------------------------------------------------------ workloads ---
# Seeds: base 250919703; workload i uses base + i; per-graph seeds mix(base+i, j);
# sampled sources use base + 100; arrivals use base + 200.

def config_grid() -> CSR:
    """32 x 32 grid (n = 1,024, m = 1,984): the plain small all-source case."""
    return grid_2d(32, 32)


def config_ba() -> CSR:
    """Barabasi-Albert n = 100,000, 4 edges per new vertex (m = 399,990)."""
    g = ba(100_000, 4, BASE_SEED + 1)
    g.name = "ba100k"
    return g


def config_ba_sources(count: int = 4096) -> np.ndarray:
    return sample_sources(100_000, count, BASE_SEED + 100)


def config_er() -> CSR:
    """Erdos-Renyi G(16,384, 1/16): mean degree ~1,024, diameter 2 w.h.p."""
    g = er(16_384, 1.0 / 16.0, BASE_SEED + 2)
    g.name = "er16k"
    return g


def _family_graph(kind: int, n: int, deg: float, seed: int) -> CSR:
    if kind == 0:
        g = ba(n, max(1, int(round(deg / 2.0))), seed)
    elif kind == 1:
        g = rgg(n, deg, seed)
    else:
        g = sbm(n, deg, seed)
    g.meta.update({"n_target": n, "deg_target": deg})
    return g


def config_batch_params(count: int = 2048, seed: int = BASE_SEED + 3,
                        n_lo: int = 256, n_hi: int = 16_384, d_lo: float = 4.0, d_hi: float = 32.0):
    """(kind, n, degree, seed) of the uneven batch: n log-uniform, degree uniform,
    kinds cycling BA / RGG / SBM (one third each)."""
    out = []
    for j in range(count):
        s = mix_seed(seed, j)
        u = uniform(s, 2)
        n = int(round(math.exp(math.log(n_lo) + u[0] * (math.log(n_hi) - math.log(n_lo)))))
        d = d_lo + u[1] * (d_hi - d_lo)
        out.append((j % 3, n, d, mix_seed(s, 7)))
    return out


def config_batch_graphs(count: int = 2048, **kw) -> list[CSR]:
    """The uneven batch: ``count`` graphs, n log-uniform in [256, 16384],
    mean degree uniform in [4, 32], one third each BA / RGG / SBM."""
    return [_family_graph(k, n, d, s) for (k, n, d, s) in config_batch_params(count, **kw)]


def config_stream_jobs(count: int = 4096, seed: int = BASE_SEED + 4, rate_hz: float = 100.0,
                       n_lo: int = 1000, n_hi: int = 200_000, d_lo: float = 4.0, d_hi: float = 64.0):
    """Served stream: Poisson arrival times (s), and per job (kind, n, degree, k, seed)."""
    arr = uniform(BASE_SEED + 200, count)
    gaps = -np.log1p(-arr) / rate_hz
    times = np.cumsum(gaps)
    jobs = []
    for j in range(count):
        s = mix_seed(seed, j)
        u = uniform(s, 3)
        n = int(round(math.exp(math.log(n_lo) + u[0] * (math.log(n_hi) - math.log(n_lo)))))
        d = d_lo + u[1] * (d_hi - d_lo)
        k = (10, 15, 30)[min(2, int(u[2] * 3))]
        jobs.append({"t": float(times[j]), "kind": j % 3, "n": n, "deg": d, "k": k, "seed": mix_seed(s, 7)})
    return jobs


def stream_job_graph(job: dict) -> CSR:
    return _family_graph(job["kind"], job["n"], job["deg"], job["seed"])
