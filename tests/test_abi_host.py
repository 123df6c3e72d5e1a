"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every entry point declared in include/nfft3.h, validates arguments before any
HIP call, and its host tables (deconvolution factors, window polynomials)
agree with the oracle's textbook formulas."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import nfft_steps as ns

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def nf():
    import paper_1605_01244_amd as mod
    return mod


def _declared():
    text = open(os.path.join(ROOT, "include", "nfft3.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nfft3_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(nf):
    lib = ctypes.CDLL(nf._lib.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _plan(nf, N=(8, 8, 8), sigma=2.0, m=4, dtype=1):
    h = ctypes.c_void_p(123)
    Narr = (ctypes.c_int64 * 3)(*N)
    rc = nf.lib.nfft3_plan(ctypes.byref(h), Narr, sigma, m, dtype, None)
    return rc, h


@pytest.mark.parametrize("N,sigma,m,dtype,code", [
    ((7, 8, 8), 2.0, 4, 1, -1),      # odd N
    ((0, 8, 8), 2.0, 4, 1, -1),      # N < 2
    ((8, 8, 8), 1.0, 4, 1, -1),      # sigma <= 1
    ((8, 8, 8), float("nan"), 4, 1, -1),
    ((8, 8, 8), 1.3, 4, 1, -1),      # sigma N not an integer
    ((6, 6, 6), 1.5, 2, 1, -1),      # sigma N odd (9)
    ((8, 8, 8), 2.0, 0, 1, -1),      # m < 1
    ((8, 8, 8), 2.0, 9, 1, -1),      # 2m > n
    ((8, 8, 8), 2.0, 11, 1, -1),     # m beyond the supported range
    ((22, 8, 8), 2.0, 4, 1, -1),     # n = 44 = 4*11: factor 11 unsupported
    ((8, 8, 8), 2.0, 4, 5, -2),      # bad dtype
    ((2048, 8, 8), 2.0, 4, 1, -1),   # n > 2048
    ((8, 1, 8), 2.0, 4, 1, -1),      # a unit axis that is not leading
    ((8, 8, 1), 2.0, 4, 1, -1),
    ((1, 8, 1), 2.0, 4, 1, -1),
])
def test_plan_rejects_invalid_arguments(nf, N, sigma, m, dtype, code):
    rc, h = _plan(nf, N, sigma, m, dtype)
    assert rc == code


@pytest.mark.parametrize("d,N,code", [
    (0, (8,), -1), (4, (8, 8, 8, 8), -1),     # one to three axes
    (1, (1,), -1), (2, (8, 1), -1),           # unit axes are not given explicitly
    (1, (7,), -1), (2, (8, 4096), -1),        # odd N; n > 2048
])
def test_plan_nd_rejects_invalid_arguments(nf, d, N, code):
    h = ctypes.c_void_p(123)
    Narr = (ctypes.c_int64 * len(N))(*N)
    assert nf.lib.nfft3_plan_nd(ctypes.byref(h), d, Narr, 2.0, 4, 1, None) == code
    assert h.value is None
    assert h.value is None


def test_null_handling(nf):
    lib = nf.lib
    Narr = (ctypes.c_int64 * 3)(8, 8, 8)
    assert lib.nfft3_plan(None, Narr, 2.0, 4, 1, None) == -7
    h = ctypes.c_void_p()
    assert lib.nfft3_plan(ctypes.byref(h), None, 2.0, 4, 1, None) == -7
    assert lib.nfft3_destroy(None) == 0
    assert lib.nfft3_trafo(None, None, None) == -7
    assert lib.nfft3_adjoint(None, None, None) == -7
    assert lib.nfft3_set_points(None, 0, None) == -7
    assert lib.nfft3_grad_points(None, None, None, None) == -7
    assert lib.nfft3_set_tuning(None, 16, 256) == -7
    assert lib.nfft3_get_tuning(None, None, None) == -7
    assert lib.nfft3_autotune(None, 0, None, None, None, 1, None, None) == -7
    for batch in (lib.nfft3_batch_trafo, lib.nfft3_batch_trafo_noalloc, lib.nfft3_batch_trafo_queue):
        assert batch(-1, None, None, None, 0) == -1          # negative count
        assert batch(0, None, None, None, 0) == 0            # empty batch: nothing to do
        assert batch(1, None, None, None, 0) == -7           # NULL arrays
        assert batch(1, None, None, None, 8) == -1           # mask beyond the three axes
    assert lib.nfft3_strerror(-5) == b"non-finite point coordinate"
    assert b"time limit" in lib.nfft3_strerror(-9)


def test_deconv_factors_match_textbook_pair(nf):
    """c[k] = phi(0) / (n phihat(k)) with the oracle's window and transform."""
    for m in (2, 4, 6, 8, 10):
        for Nd, sigma in ((32, 2.0), (64, 1.5), (20, 2.0)):
            c = nf.deconv_factors(Nd, sigma, m)
            n = int(round(sigma * Nd))
            k = np.arange(Nd) - Nd // 2
            ref = ns.kb_phi(np.array([0.0]), m, sigma)[0] / ns.kb_phihat_scaled(k, n, m, sigma)
            assert np.max(np.abs(c - ref) / ref) < 1e-12, (m, Nd, sigma)


def _window_mp(t, m, sigma):
    """phi(t)/phi(0) = (m/s) sinh(b s)/sinh(b m), s = sqrt(m^2 - t^2), in 40-digit arithmetic."""
    import mpmath
    mpmath.mp.dps = 40
    b = mpmath.pi * (2 - mpmath.mpf(1) / mpmath.mpf(sigma))
    out = []
    for v in t:
        s = mpmath.sqrt(mpmath.mpf(m) ** 2 - mpmath.mpf(float(v)) ** 2)
        val = (m * b / mpmath.sinh(b * m)) if s == 0 else (m / s) * mpmath.sinh(b * s) / mpmath.sinh(b * m)
        out.append(float(val))
    return np.array(out)


@pytest.mark.parametrize("m,sigma,dtype,tol", [
    (4, 2.0, "c64", 3e-8), (8, 2.0, "c128", 1e-15), (6, 2.0, "c128", 1e-15),
    (4, 2.0, "c128", 1e-15), (2, 2.0, "c128", 1e-15), (6, 1.5, "c128", 1e-15), (10, 2.0, "c128", 1e-15),
])
def test_window_polynomials_match_window(nf, m, sigma, dtype, tol):
    """Each window piece, as a polynomial in y = 2f - 1, against the window
    evaluated in 40-digit arithmetic, and the pieces against the oracle's
    double-precision window (whose own rounding grows like b m eps)."""
    import torch
    dt = torch.complex64 if dtype == "c64" else torch.complex128
    C = nf.window_poly(m, sigma, dt)
    f = np.linspace(0.0, 1.0, 101)
    y = 2 * f - 1
    phi0 = ns.kb_phi(np.array([0.0]), m, sigma)[0]
    for r in range(2 * m):
        off = r - m + 1
        p = np.zeros_like(y)
        for q in range(C.shape[1] - 1, -1, -1):
            p = p * y + C[r, q]
        exact = _window_mp(f - off, m, sigma)
        assert np.max(np.abs(p - exact)) < tol, (r, np.max(np.abs(p - exact)))
        textbook = ns.kb_phi(f - off, m, sigma) / phi0
        assert np.max(np.abs(p - textbook)) < tol + 4 * ns.kb_b(sigma) * m * 2.2e-16
