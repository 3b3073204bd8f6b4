"""The library's host-side eigen-solver for the Lanczos recurrence matrix
(the largest eigenvalue of a symmetric tridiagonal matrix and its unit
eigenvector, by Sturm bisection and inverse iteration) against SciPy's
tridiagonal eigensolver.  It is an internal C++ routine of libgumap, reached
here by its symbol; no GPU needed."""
import ctypes

import numpy as np
import pytest

SYMBOL = "_ZN2gm11tridiag_topEiPKdS1_PdS2_"   # gm::tridiag_top(int, const double*, const double*, double*, double*)


@pytest.fixture(scope="module")
def top(gumap):
    fn = getattr(gumap.lib, SYMBOL)
    dp = ctypes.POINTER(ctypes.c_double)
    fn.argtypes = [ctypes.c_int, dp, dp, dp, dp]
    fn.restype = ctypes.c_bool

    def call(a, b):
        a = np.ascontiguousarray(a, np.float64)
        b = np.ascontiguousarray(np.append(b, 0.0), np.float64)
        z = np.zeros(len(a))
        th = ctypes.c_double()
        ok = fn(len(a), a.ctypes.data_as(dp), b.ctypes.data_as(dp), ctypes.byref(th), z.ctypes.data_as(dp))
        assert ok
        return th.value, z
    return call


def _check(top, a, b, tol=1e-12):
    from scipy.linalg import eigh_tridiagonal
    th, z = top(a, b)
    w, v = eigh_tridiagonal(a, b)
    assert abs(th - w[-1]) <= tol * max(1.0, abs(w[-1]))
    assert abs(np.linalg.norm(z) - 1.0) < 1e-12
    # the same eigenvector up to sign (the top eigenvalue of an unreduced
    # tridiagonal matrix is simple)
    assert min(np.abs(z - v[:, -1]).max(), np.abs(z + v[:, -1]).max()) < 1e-9
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    assert np.abs(T @ z - th * z).max() < 1e-12 * max(1.0, np.abs(T).max())


@pytest.mark.parametrize("m", [1, 2, 3, 17, 64, 300])
def test_random_tridiagonal(top, m):
    rng = np.random.default_rng(1000 + m)
    a = rng.uniform(-1, 1, m)
    b = rng.uniform(0.05, 0.6, m - 1)
    if m == 1:
        th, z = top(a, b)
        assert th == a[0] and z[0] == 1.0
        return
    _check(top, a, b)


def test_closed_forms(top):
    # the path graph's adjacency (a = 0, b = 1): eigenvalues 2 cos(pi j / (m + 1)),
    # top eigenvector proportional to sin(pi i / (m + 1))
    m = 50
    th, z = top(np.zeros(m), np.ones(m - 1))
    assert abs(th - 2 * np.cos(np.pi / (m + 1))) < 1e-13
    ref = np.sin(np.pi * np.arange(1, m + 1) / (m + 1))
    ref /= np.linalg.norm(ref)
    assert min(np.abs(z - ref).max(), np.abs(z + ref).max()) < 1e-10
    # clustered spectrum (tiny couplings) and a constant diagonal shift
    rng = np.random.default_rng(7)
    _check(top, rng.uniform(-1, 1, 120), rng.uniform(1e-4, 1e-3, 119))
    _check(top, 5.0 + rng.uniform(-1e-3, 1e-3, 80), rng.uniform(0.5, 1.0, 79))
