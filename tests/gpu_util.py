"""Shared helpers of the GPU parity tests."""
import numpy as np


def to_dev(g, device="cuda"):
    import torch
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr)).to(device),
            torch.from_numpy(np.ascontiguousarray(g.col_idx)).to(device))


def assert_weights_close(w_gpu, w_ref, rho_gpu=None, rho_ref=None, sig_gpu=None, sig_ref=None):
    """Weights within 1e-5 relative (plus 2^-126 absolute for denormals),
    rho bit-exact, sigma within 1e-5 relative when finite and nonzero and
    exactly equal otherwise."""
    w_gpu = np.asarray(w_gpu, dtype=np.float64)
    w_ref = np.asarray(w_ref, dtype=np.float64)
    err = np.abs(w_gpu - w_ref)
    tol = 1e-5 * np.abs(w_ref) + 2.0**-126
    bad = np.argwhere(err > tol)
    assert bad.size == 0, "weights differ at %s: gpu %r ref %r" % (
        bad[:5].tolist(), w_gpu[tuple(bad[0])], w_ref[tuple(bad[0])])
    if rho_gpu is not None:
        assert np.array_equal(np.asarray(rho_gpu), np.asarray(rho_ref))
    if sig_gpu is not None:
        sg = np.asarray(sig_gpu, dtype=np.float64)
        sr = np.asarray(sig_ref, dtype=np.float64)
        special = ~np.isfinite(sr) | (sr == 0)
        assert np.array_equal(sg[special], sr[special])
        fin = ~special
        assert np.all(np.abs(sg[fin] - sr[fin]) <= 1e-5 * np.abs(sr[fin]))


def first_mismatch(a, b):
    idx = np.argwhere(np.asarray(a) != np.asarray(b))
    return None if idx.size == 0 else idx[0].tolist()


def random_knn(n, k, seed, binary=False, zero_frac=0.2, fill=None):
    """Seeded synthetic kNN rows: ids int32 [n, k] (distinct, never the row
    itself, -1 padding at the end of short rows) and weights float32 [n, k]
    in [0, 1] with a share of exact zeros (or all ones when binary)."""
    rng = np.random.default_rng(seed)
    ids = np.full((n, k), -1, np.int32)
    w = np.zeros((n, k), np.float32)
    for i in range(n):
        cnt = min(n - 1, k if fill == "full" else int(rng.integers(0, k + 1)))
        others = rng.permutation(np.delete(np.arange(n), i))[:cnt]
        ids[i, :cnt] = others
        w[i, :cnt] = 1.0 if binary else rng.uniform(0.0, 1.0, cnt).astype(np.float32)
        w[i, :cnt][rng.uniform(size=cnt) < zero_frac] = 0.0
    return ids, w
