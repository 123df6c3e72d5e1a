"""TEST INFRASTRUCTURE ONLY -- plain numpy FP64 statement of the windowed
algorithm (NFFT) whose result the paper obtains by calling the NFFT library
(Sec. 2.2.1; the method is the one of the cited NFFT reference [KKP09]).

The paper states the problem and the cost O(N log N + M |log eps|^3) (Sec. 1)
but not the algorithm's internals.  This module takes them from the NFFT
literature that the paper cites, in their textbook form (unnormalised window,
no precomputation, no tiling):

1.  window (Kaiser-Bessel, in units of oversampled grid cells t):
        phi(t) = sinh(b sqrt(m^2 - t^2)) / (pi sqrt(m^2 - t^2)),  |t| <= m,
    truncated to zero for |t| > m, with b = pi (2 - 1/sigma);
    its Fourier transform scaled by the grid size n is
        n phihat(k) = I0(m sqrt(b^2 - (2 pi k / n)^2))  for |k| <= n (1 - 1/(2 sigma)).
2.  deconvolve and zero-pad: ghat[k mod n] = fhat_k / prod_d n_d phihat_d(k_d).
3.  FFT on the oversampled grid n = sigma N:  g_l = sum_k ghat_k exp(-2 pi i k.l/n).
4.  window sum at the points: f_j ~ sum_{l} g_{l mod n} prod_d phi(n_d x_{j,d} - l_d)
    over the 2m grid indices per axis with -m < l - n x <= m.

The adjoint runs the transposed steps (spread, FFT with + sign, truncate and
deconvolve); the point gradient replaces one window factor by n_d phi'(t).

Every reading of the paper taken here (window, sigma, m, stencil, adjoint,
gradient) is listed with its justification in the design notes.
"""
from __future__ import annotations

import math

import numpy as np


def kb_b(sigma: float) -> float:
    """Shape parameter b = pi (2 - 1/sigma) of the Kaiser-Bessel window [KKP09]."""
    return math.pi * (2.0 - 1.0 / sigma)


def grid_size(N, sigma: float) -> np.ndarray:
    """Oversampled grid n_d = sigma N_d; must be an even integer per axis."""
    N = np.asarray(N, dtype=np.int64).reshape(-1)
    n = np.rint(sigma * N).astype(np.int64)
    if np.any(np.abs(sigma * N - n) > 1e-9) or np.any(n % 2):
        raise ValueError(f"sigma*N = {sigma * N} is not an even integer per axis")
    return n


def kb_phi(t, m: int, sigma: float) -> np.ndarray:
    """Kaiser-Bessel window phi(t) in grid units, truncated to |t| <= m."""
    b = kb_b(sigma)
    t = np.asarray(t, dtype=np.float64)
    s2 = m * m - t * t
    out = np.zeros_like(t)
    pos = s2 > 0
    s = np.sqrt(s2[pos])
    out[pos] = np.sinh(b * s) / (math.pi * s)
    out[s2 == 0] = b / math.pi           # limit of sinh(bs)/(pi s) as s -> 0
    return out


def kb_phi_deriv(t, m: int, sigma: float) -> np.ndarray:
    """d phi / dt = -t (b s cosh(bs) - sinh(bs)) / (pi s^3), s = sqrt(m^2 - t^2).

    For small b s the bracket is expanded: (z cosh z - sinh z)/z^3 =
    sum_{q>=1} 2q z^(2q-2) / (2q+1)!, which avoids the cancellation.
    """
    b = kb_b(sigma)
    t = np.asarray(t, dtype=np.float64)
    s2 = m * m - t * t
    out = np.zeros_like(t)
    pos = s2 >= 0
    s = np.sqrt(np.maximum(s2[pos], 0.0))
    z = b * s
    big = z > 0.25
    F = np.empty_like(z)
    zb = z[big]
    F[big] = (zb * np.cosh(zb) - np.sinh(zb)) / zb ** 3
    zs = z[~big]
    acc = np.zeros_like(zs)
    for q in range(1, 12):
        acc += 2 * q * zs ** (2 * q - 2) / math.factorial(2 * q + 1)
    F[~big] = acc
    out[pos] = -t[pos] * b ** 3 * F / math.pi
    return out


def kb_phihat_scaled(k, n: int, m: int, sigma: float) -> np.ndarray:
    """n * phihat(k) = I0(m sqrt(b^2 - (2 pi k/n)^2)) on the band, 0 beyond."""
    b = kb_b(sigma)
    k = np.asarray(k, dtype=np.float64)
    arg = b * b - (2.0 * math.pi * k / n) ** 2
    out = np.zeros_like(k)
    ok = arg >= 0
    out[ok] = np.i0(m * np.sqrt(arg[ok]))
    return out


def pst_error_bound(m: int, sigma: float) -> float:
    """Kaiser-Bessel NFFT error estimate relative to ||fhat||_1 (Potts, Steidl,
    Tasche 2001): 4 pi (sqrt m + m) (1 - 1/sigma)^(1/4) exp(-2 pi m sqrt(1 - 1/sigma))."""
    q = 1.0 - 1.0 / sigma
    return 4 * math.pi * (math.sqrt(m) + m) * q ** 0.25 * math.exp(-2 * math.pi * m * math.sqrt(q))


def _freqs(Nd: int) -> np.ndarray:
    return np.arange(Nd) - Nd // 2


def deconvolve_pad(fhat: np.ndarray, m: int, sigma: float) -> np.ndarray:
    """Step 2: ghat[k mod n] = fhat_k / prod_d n_d phihat(k_d), zero elsewhere."""
    fhat = np.asarray(fhat, dtype=np.complex128)
    N = fhat.shape
    n = grid_size(N, sigma)
    c = [1.0 / kb_phihat_scaled(_freqs(N[d]), n[d], m, sigma) for d in range(3)]
    ghat = np.zeros(tuple(n.tolist()), dtype=np.complex128)
    idx = np.ix_(*[_freqs(N[d]) % n[d] for d in range(3)])
    ghat[idx] = fhat * c[0][:, None, None] * c[1][None, :, None] * c[2][None, None, :]
    return ghat


def oversampled_grid(fhat: np.ndarray, m: int, sigma: float) -> np.ndarray:
    """Steps 2-3: g = FFT_n(ghat), forward sign, unnormalised (numpy fftn)."""
    return np.fft.fftn(deconvolve_pad(fhat, m, sigma))


def _stencil(x: np.ndarray, n: np.ndarray, m: int, sigma: float, deriv_axis=None):
    """Per axis: grid indices (M, 2m) mod n and window values phi(n x - l)."""
    x = np.asarray(x, dtype=np.float64)
    x = x - np.floor(x + 0.5)                      # fold to [-1/2, 1/2)
    idx, w = [], []
    r = np.arange(-m + 1, m + 1)
    for d in range(3):
        t = n[d] * x[:, d]
        u = np.floor(t)
        l = u[:, None] + r[None, :]
        tt = t[:, None] - l
        if deriv_axis == d:
            w.append(n[d] * kb_phi_deriv(tt, m, sigma))
        else:
            w.append(kb_phi(tt, m, sigma))
        idx.append(np.mod(l.astype(np.int64), n[d]))
    return idx, w


def interpolate(g: np.ndarray, x: np.ndarray, m: int, sigma: float,
                deriv_axis=None, chunk: int = 512) -> np.ndarray:
    """Step 4: f_j = sum_l g_{l mod n} prod_d phi(n_d x_{j,d} - l_d) (2m points per axis).

    With ``deriv_axis = d`` the factor of axis d is n_d phi'(.), which is the
    derivative of the same sum with respect to x_{j,d}.
    """
    n = np.asarray(g.shape, dtype=np.int64)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros(x.shape[0], dtype=np.complex128)
    for s in range(0, x.shape[0], chunk):
        idx, w = _stencil(x[s:s + chunk], n, m, sigma, deriv_axis)
        vals = g[idx[0][:, :, None, None], idx[1][:, None, :, None], idx[2][:, None, None, :]]
        out[s:s + chunk] = np.einsum("jabc,ja,jb,jc->j", vals, w[0], w[1], w[2])
    return out


def trafo(fhat: np.ndarray, x: np.ndarray, m: int, sigma: float = 2.0) -> np.ndarray:
    """The windowed approximation of sum_k fhat_k exp(-2 pi i k.x_j)."""
    return interpolate(oversampled_grid(fhat, m, sigma), x, m, sigma)


def spread(f: np.ndarray, x: np.ndarray, n, m: int, sigma: float) -> np.ndarray:
    """Transpose of step 4: g_l = sum_j f_j prod_d phi(n_d x_{j,d} - l_d)."""
    n = np.asarray(n, dtype=np.int64)
    g = np.zeros(tuple(n.tolist()), dtype=np.complex128)
    f = np.asarray(f, dtype=np.complex128).reshape(-1)
    idx, w = _stencil(x, n, m, sigma)
    vals = f[:, None, None, None] * w[0][:, :, None, None] * w[1][:, None, :, None] * w[2][:, None, None, :]
    I = np.ravel_multi_index(np.broadcast_arrays(idx[0][:, :, None, None], idx[1][:, None, :, None],
                                                 idx[2][:, None, None, :]), tuple(n.tolist()))
    np.add.at(g.reshape(-1), I.reshape(-1), vals.reshape(-1))
    return g


def adjoint(f: np.ndarray, x: np.ndarray, N, m: int, sigma: float = 2.0) -> np.ndarray:
    """Transposed steps: spread, FFT with + sign (unnormalised), keep I_N, deconvolve."""
    N = tuple(int(v) for v in N)
    n = grid_size(N, sigma)
    g = spread(f, x, n, m, sigma)
    ghat = np.fft.ifftn(g) * float(np.prod(n))     # sum_l g_l exp(+2 pi i k.l/n)
    idx = np.ix_(*[_freqs(N[d]) % n[d] for d in range(3)])
    c = [1.0 / kb_phihat_scaled(_freqs(N[d]), n[d], m, sigma) for d in range(3)]
    return ghat[idx] * c[0][:, None, None] * c[1][None, :, None] * c[2][None, None, :]


def grad_points(fhat: np.ndarray, x: np.ndarray, m: int, sigma: float = 2.0) -> np.ndarray:
    """(M, 3) complex: d f_j / d x_{j,d} of the windowed sum."""
    g = oversampled_grid(fhat, m, sigma)
    return np.stack([interpolate(g, x, m, sigma, deriv_axis=d) for d in range(3)], axis=1)
