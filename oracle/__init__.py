"""TEST INFRASTRUCTURE ONLY -- the oracle.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding in ``paper_1605_01244_amd``) never imports it, and this
package imports nothing from there.

Two parts:

* ``ndft_*`` -- plain FP64 direct sums (the definition of the NFFT problem,
  Sec. 2.2.1, evaluated in the one-loop order of eq. (Fs)), in C
  (``oracle/ndft.c``) with POSIX threads, reached through ctypes.  These are
  the reference every GPU result is compared with.
* ``infftm_eval`` / ``infftm_coeffs`` / ``tube_refine`` -- the series of
  eq. (fs) on a physical domain [a, b) (direct sums), the trapezoidal
  coefficients of Sec. 2, and the vortex-tube refinement of Sec. 4.3.
* ``gpe_tssp`` -- Strang splitting of the Gross-Pitaevskii equation (Sec. 3.1)
  with numpy's FFT.
* ``rgrid_eval`` -- the series at a rectilinear grid as the nested per-axis
  sums of Sec. 2.1 (numpy FP64 matrix products with the E^d matrices).
* ``ndft_lowdim*`` / ``infft_lowdim`` / ``rgrid_lowdim`` -- the one- and
  two-dimensional series (Appendix B: the E psihat product, infft, infft2,
  igridft2) as numpy FP64 products with the per-axis phase matrices.
* ``oracle.nfft_steps`` -- a plain numpy FP64 statement of the windowed
  algorithm the GPU implements (deconvolve, oversampled FFT, window sum),
  used to check the GPU stages one at a time.

Pins for both live in ``tests/test_oracle_*.py`` (closed forms, library
special cases, invariants, brute force, error bounds).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ndft.c")
_LIB = os.path.join(_HERE, "libndft.so")

# The oracle is built for the plain x86-64 baseline (no -march=native) so the
# library built here also runs on a host with a different CPU.
_CFLAGS = ["-O2", "-std=c99", "-fPIC", "-shared", "-pthread"]


def build(verbose: bool = False) -> str:
    """Compile ``ndft.c`` into ``libndft.so`` with gcc (always recompiles)."""
    cmd = ["gcc", *_CFLAGS, _SRC, "-o", _LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_ndft_trafo.argtypes = [i64p, dp, ctypes.c_int64, dp, dp, ctypes.c_int]
    lib.oracle_ndft_grad.argtypes = [i64p, dp, ctypes.c_int64, dp, dp, ctypes.c_int]
    lib.oracle_ndft_adjoint.argtypes = [i64p, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
    lib.oracle_ndft_adjoint_at.argtypes = [i64p, ctypes.c_int64, dp, dp, ctypes.c_int64, i64p, dp, ctypes.c_int]
    for fn in (lib.oracle_ndft_trafo, lib.oracle_ndft_grad, lib.oracle_ndft_adjoint, lib.oracle_ndft_adjoint_at):
        fn.restype = ctypes.c_int
    _lib = lib
    return lib


def default_threads() -> int:
    env = os.environ.get("ORACLE_THREADS")
    if env:
        return max(1, int(env))
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _shape3(N) -> np.ndarray:
    N = np.asarray(N, dtype=np.int64).reshape(3)
    if np.any(N < 2) or np.any(N % 2):
        raise ValueError(f"N must hold three even sizes >= 2, got {N.tolist()}")
    return np.ascontiguousarray(N)


def _points(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim != 2 or x.shape[1] != 3:
        raise ValueError("points must have shape (M, 3)")
    return x


def ndft_trafo(fhat: np.ndarray, x: np.ndarray, threads: int | None = None) -> np.ndarray:
    """f_j = sum_{k in I_N} fhat_k exp(-2 pi i k.x_j)  (Sec. 2.2.1, eq. (Fs) order).

    ``fhat``: complex (N0, N1, N2), index i <-> frequency i - N/2.
    ``x``: (M, 3) real.  Returns complex128 (M,).
    """
    fhat = np.ascontiguousarray(fhat, dtype=np.complex128)
    N = _shape3(fhat.shape)
    x = _points(x)
    f = np.zeros(x.shape[0], dtype=np.complex128)
    rc = _load().oracle_ndft_trafo(N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                   _dptr(fhat.view(np.float64)), x.shape[0], _dptr(x),
                                   _dptr(f.view(np.float64)), threads or default_threads())
    if rc:
        raise RuntimeError(f"oracle_ndft_trafo failed ({rc})")
    return f


def ndft_adjoint(f: np.ndarray, x: np.ndarray, N, threads: int | None = None) -> np.ndarray:
    """fhat_k = sum_j f_j exp(+2 pi i k.x_j): the conjugate transpose of ``ndft_trafo``."""
    N = _shape3(N)
    x = _points(x)
    f = np.ascontiguousarray(np.asarray(f, dtype=np.complex128).reshape(-1))
    if f.shape[0] != x.shape[0]:
        raise ValueError("f and x disagree on M")
    out = np.zeros(tuple(N.tolist()), dtype=np.complex128)
    rc = _load().oracle_ndft_adjoint(N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     x.shape[0], _dptr(x), _dptr(f.view(np.float64)),
                                     _dptr(out.view(np.float64)), threads or default_threads())
    if rc:
        raise RuntimeError(f"oracle_ndft_adjoint failed ({rc})")
    return out


def ndft_adjoint_at(f: np.ndarray, x: np.ndarray, N, kidx, threads: int | None = None) -> np.ndarray:
    """fhat at sampled coefficients: out[q] = sum_j f_j exp(+2 pi i k_q.x_j) for
    the array-index triples ``kidx`` (K, 3) (frequency = index - N/2); the
    same sum as ``ndft_adjoint``, evaluated for K coefficients over all points."""
    N = _shape3(N)
    x = _points(x)
    f = np.ascontiguousarray(np.asarray(f, dtype=np.complex128).reshape(-1))
    if f.shape[0] != x.shape[0]:
        raise ValueError("f and x disagree on M")
    kidx = np.ascontiguousarray(np.asarray(kidx, dtype=np.int64).reshape(-1, 3))
    out = np.zeros(kidx.shape[0], dtype=np.complex128)
    rc = _load().oracle_ndft_adjoint_at(N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), x.shape[0], _dptr(x),
                                        _dptr(f.view(np.float64)), kidx.shape[0],
                                        kidx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                        _dptr(out.view(np.float64)), threads or default_threads())
    if rc:
        raise RuntimeError(f"oracle_ndft_adjoint_at failed ({rc})")
    return out


def ndft_grad(fhat: np.ndarray, x: np.ndarray, threads: int | None = None) -> np.ndarray:
    """df_j/dx_{j,d} = sum_k (-2 pi i k_d) fhat_k exp(-2 pi i k.x_j), shape (M, 3) complex.

    The multiplier is eq. (Lambda) on the unit period in the NFFT sign.
    """
    fhat = np.ascontiguousarray(fhat, dtype=np.complex128)
    N = _shape3(fhat.shape)
    x = _points(x)
    out = np.zeros((x.shape[0], 3), dtype=np.complex128)
    rc = _load().oracle_ndft_grad(N.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  _dptr(fhat.view(np.float64)), x.shape[0], _dptr(x),
                                  _dptr(out.view(np.float64)), threads or default_threads())
    if rc:
        raise RuntimeError(f"oracle_ndft_grad failed ({rc})")
    return out


def axis_phases(Nd: int, y) -> np.ndarray:
    """E[i, k] = exp(-2 pi i k y_i) for frequencies k = -Nd/2 .. Nd/2-1 (array
    index k + Nd/2): the matrix E^d of Sec. 2.1 in the NFFT sign on the unit
    period.  The phase k y is reduced mod 1 exactly (the product of an integer
    below 2^11 and a double is exact in 80-bit long double), then rounded once."""
    y = np.asarray(y, dtype=np.float64).reshape(-1)
    k = frequencies(Nd).astype(np.longdouble)
    p = y.astype(np.longdouble)[:, None] * k[None, :]
    r = (p - np.rint(p)).astype(np.float64)
    return np.cos(2.0 * np.pi * r) - 1j * np.sin(2.0 * np.pi * r)


def rgrid_eval(fhat: np.ndarray, y0, y1, y2) -> np.ndarray:
    """The series at the rectilinear grid y0 x y1 x y2 (Sec. 2.1):
    F[i0, i1, i2] = sum_k fhat_k exp(-2 pi i (k0 y0[i0] + k1 y1[i1] + k2 y2[i2])),
    evaluated as the nested sums of Sec. 2.1, one matrix product with E^d per
    axis: first over k2 (the contiguous axis), then k1, then k0.  FP64."""
    fhat = np.asarray(fhat, dtype=np.complex128)
    N0, N1, N2 = _shape3(fhat.shape).tolist()
    E0, E1, E2 = axis_phases(N0, y0), axis_phases(N1, y1), axis_phases(N2, y2)
    M0, M1, M2 = E0.shape[0], E1.shape[0], E2.shape[0]
    t = (fhat.reshape(N0 * N1, N2) @ E2.T).reshape(N0, N1, M2)      # sum over k2
    t = np.matmul(E1[None, :, :], t)                                 # sum over k1: (N0, M1, M2)
    return (E0 @ t.reshape(N0, M1 * M2)).reshape(M0, M1, M2)        # sum over k0


def _lowdim(fhat, x):
    fhat = np.asarray(fhat, dtype=np.complex128)
    d = fhat.ndim
    if d not in (1, 2) or any(n < 2 or n % 2 for n in fhat.shape):
        raise ValueError("coefficients must be a 1-D or 2-D array of even sizes >= 2")
    x = np.asarray(x, dtype=np.float64).reshape(-1, d)
    return fhat, x, d


def ndft_lowdim(fhat: np.ndarray, x: np.ndarray) -> np.ndarray:
    """f_j = sum_k fhat_k exp(-2 pi i k.x_j) for a one- or two-dimensional
    coefficient array (index i <-> frequency i - N/2) at points x (M, d).
    One dimension: the matrix-vector product E fhat that Appendix B writes
    out for this case, E[j, k] = exp(-2 pi i k x_j).  Two dimensions: that
    product along axis 1 for every k0 row, then the sum over k0 with the
    axis-0 phases.  FP64."""
    fhat, x, d = _lowdim(fhat, x)
    if d == 1:
        return axis_phases(fhat.shape[0], x[:, 0]) @ fhat
    E0 = axis_phases(fhat.shape[0], x[:, 0])              # (M, N0)
    E1 = axis_phases(fhat.shape[1], x[:, 1])              # (M, N1)
    inner = E1 @ fhat.T                                   # (M, N0): sum over k1
    return np.sum(E0 * inner, axis=1)                     # sum over k0


def ndft_lowdim_adjoint(f: np.ndarray, x: np.ndarray, N) -> np.ndarray:
    """fhat_k = sum_j f_j exp(+2 pi i k.x_j) (the conjugate transpose of
    ``ndft_lowdim``) for N of one or two entries."""
    N = tuple(int(v) for v in np.atleast_1d(N))
    _, x, d = _lowdim(np.zeros(N), x)
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    if d == 1:
        return np.conj(axis_phases(N[0], x[:, 0])).T @ f
    E0 = np.conj(axis_phases(N[0], x[:, 0]))
    E1 = np.conj(axis_phases(N[1], x[:, 1]))
    return (E0 * f[:, None]).T @ E1


def ndft_lowdim_grad(fhat: np.ndarray, x: np.ndarray) -> np.ndarray:
    """df_j/dx_{j,d} = sum_k (-2 pi i k_d) fhat_k exp(-2 pi i k.x_j), (M, d) complex."""
    fhat, x, d = _lowdim(fhat, x)
    cols = []
    for ax in range(d):
        k = frequencies(fhat.shape[ax]).astype(np.float64)
        shape = [1] * d
        shape[ax] = -1
        cols.append(ndft_lowdim(fhat * (-2j * np.pi * k.reshape(shape)), x))
    return np.stack(cols, axis=1)


def infft_lowdim(psihat: np.ndarray, a, b, xi: np.ndarray) -> np.ndarray:
    """The one- or two-dimensional series on prod [a_d, b_d) (Appendix B's
    infft / infft2): psi(x) = sum_k psihat_k prod_d exp(+2 pi i k_d (x_d - a_d)
    /(b_d - a_d)) / sqrt(b_d - a_d), as ``ndft_lowdim`` at y = -(x - a)/(b - a)."""
    psihat, xi, d = _lowdim(psihat, xi)
    a = np.asarray(a, dtype=np.float64).reshape(d)
    b = np.asarray(b, dtype=np.float64).reshape(d)
    y = -(xi - a[None, :]) / (b - a)[None, :]
    return ndft_lowdim(psihat, y) / float(np.prod(np.sqrt(b - a)))


def rgrid_lowdim(fhat: np.ndarray, *ys) -> np.ndarray:
    """The series at a one- or two-dimensional rectilinear grid: E0 fhat
    (one dimension, the matrix-vector product of Appendix B) or E0 fhat E1^T
    (two dimensions, the double matrix product of igridft2), E_d[i, k] =
    exp(-2 pi i k y_d[i])."""
    fhat = np.asarray(fhat, dtype=np.complex128)
    if fhat.ndim != len(ys) or fhat.ndim not in (1, 2):
        raise ValueError("one coordinate vector per axis, one or two axes")
    E = [axis_phases(n, y) for n, y in zip(fhat.shape, ys)]
    if fhat.ndim == 1:
        return E[0] @ fhat
    return E[0] @ fhat @ E[1].T


def infftm_eval(psihat: np.ndarray, a, b, xi: np.ndarray, threads: int | None = None) -> np.ndarray:
    """The truncated series of eq. (fs) on the domain prod [a_d, b_d) at points xi (M, 3):
    psi(x) = sum_k psihat_k prod_d exp(+2 pi i k_d (x_d - a_d)/(b_d - a_d)) / sqrt(b_d - a_d),
    k_d = i_d - N_d/2 for array index i_d (the paper's k_d - 1 - N_d/2).  The
    direct sum: the NFFT-sign direct sum ``ndft_trafo`` at y = -(x - a)/(b - a)."""
    a = np.asarray(a, dtype=np.float64).reshape(3)
    b = np.asarray(b, dtype=np.float64).reshape(3)
    xi = _points(xi)
    y = -(xi - a[None, :]) / (b - a)[None, :]
    return ndft_trafo(psihat, y, threads) / float(np.prod(np.sqrt(b - a)))


def infftm_coeffs(psi: np.ndarray, a, b) -> np.ndarray:
    """Coefficients of the samples psi on the regular grid X_N of the domain
    (x_{d,n} = a_d + n h_d, h_d = (b_d - a_d)/N_d): the trapezoidal rule of
    Sec. 2, psihat = fftshift(fftn(psi)) prod sqrt(b_d - a_d)/N_d."""
    a = np.asarray(a, dtype=np.float64).reshape(3)
    b = np.asarray(b, dtype=np.float64).reshape(3)
    N = np.asarray(psi.shape)
    return np.fft.fftshift(np.fft.fftn(psi)) * float(np.prod(np.sqrt(b - a) / N))


def regular_grid(N, a, b) -> np.ndarray:
    """The points of X_N (Sec. 2), (N0 N1 N2, 3) in C order of (n0, n1, n2)."""
    a = np.asarray(a, dtype=np.float64).reshape(3)
    b = np.asarray(b, dtype=np.float64).reshape(3)
    g = [a[d] + np.arange(N[d]) * ((b[d] - a[d]) / N[d]) for d in range(3)]
    G = np.meshgrid(*g, indexing="ij")
    return np.stack([x.reshape(-1) for x in G], axis=1)


def tube_refine(psihat: np.ndarray, a, b, rhobar) -> tuple[np.ndarray, np.ndarray, list]:
    """Evaluation within vortex tubes (Sec. 4.3): start from the points of X_N
    and rho = |psi|^2 there; for each threshold rhobar[l] keep the current
    points with rho <= rhobar[l], replace each by the 27 points of a regular
    grid of step h_d / 3^(l+1) centred on it, and evaluate rho there (direct
    sums).  Returns (points, rho) of the last refined set and the number of
    points kept at each level."""
    a = np.asarray(a, dtype=np.float64).reshape(3)
    b = np.asarray(b, dtype=np.float64).reshape(3)
    N = psihat.shape
    h = (b - a) / np.asarray(N)
    pts = regular_grid(N, a, b)
    rho = np.abs(infftm_eval(psihat, a, b, pts)) ** 2
    kept = []
    off = np.stack(np.meshgrid([-1, 0, 1], [-1, 0, 1], [-1, 0, 1], indexing="ij"), axis=-1).reshape(27, 3)
    for lev, rb in enumerate(rhobar):
        sel = pts[rho <= rb]
        kept.append(int(sel.shape[0]))
        step = h / 3.0 ** (lev + 1)
        pts = (sel[:, None, :] + off[None, :, :] * step[None, None, :]).reshape(-1, 3)
        rho = np.abs(infftm_eval(psihat, a, b, pts)) ** 2 if pts.shape[0] else np.zeros(0)
    return pts, rho, kept


def gpe_kinetic_phases(N, a, b, tau: float) -> np.ndarray:
    """exp(-i tau |kappa_k|^2 / 2) on numpy's FFT frequency order, kappa_{k,d} =
    2 pi k_d / (b_d - a_d): the exact flow over tau of du/dt = (i/2) Lap u
    for the Fourier mode k (eq. (Lambda): Lap E_k = sum_d Lambda_{k,d}^2 E_k)."""
    a = np.asarray(a, dtype=np.float64).reshape(3)
    b = np.asarray(b, dtype=np.float64).reshape(3)
    ks = [2.0 * np.pi * np.fft.fftfreq(N[d], d=1.0 / N[d]) / (b[d] - a[d]) for d in range(3)]
    K = np.meshgrid(*ks, indexing="ij")
    return np.exp(-0.5j * tau * (K[0] ** 2 + K[1] ** 2 + K[2] ** 2))


def gpe_tssp(psi: np.ndarray, a, b, tau: float, nsteps: int) -> np.ndarray:
    """Strang splitting of the GPE (Sec. 3.1) on the regular grid of the
    domain: per step, half a step of the potential part
    v <- exp((tau/2) (i/2) (1 - |v|^2)) v, a full step of the kinetic part in
    Fourier space (numpy FFT), and half a step of the potential part."""
    psi = np.array(psi, dtype=np.complex128)
    kin = gpe_kinetic_phases(psi.shape, a, b, tau)
    for _ in range(int(nsteps)):
        psi = np.exp(0.5j * (tau / 2) * (1.0 - np.abs(psi) ** 2)) * psi
        psi = np.fft.ifftn(kin * np.fft.fftn(psi))
        psi = np.exp(0.5j * (tau / 2) * (1.0 - np.abs(psi) ** 2)) * psi
    return psi


def frequencies(Nd: int) -> np.ndarray:
    """Frequencies of array indices 0..Nd-1 along one axis: -Nd/2 .. Nd/2-1."""
    return np.arange(Nd) - Nd // 2


def rel_errors(got: np.ndarray, ref: np.ndarray) -> tuple[float, float]:
    """(rel-l2, rel-linf) = (||got-ref||_2/||ref||_2, max|got-ref| / max|ref|)."""
    got = np.asarray(got).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    d = got - ref
    n2 = np.linalg.norm(ref)
    ninf = np.max(np.abs(ref)) if ref.size else 0.0
    l2 = float(np.linalg.norm(d) / n2) if n2 > 0 else float(np.linalg.norm(d))
    li = float(np.max(np.abs(d)) / ninf) if ninf > 0 else float(np.max(np.abs(d), initial=0.0))
    return l2, li
