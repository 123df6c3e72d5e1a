"""Pins of the one- and two-dimensional oracle (Appendix B: the E psihat
product, infft, infft2, igridft2) against brute force, FFT identities on the
regular grid, closed forms and invariants."""
import cmath
import math

import numpy as np
import pytest

import oracle


def brute_1d(fhat, x):
    N = len(fhat)
    return np.array([sum(fhat[i] * cmath.exp(-2j * math.pi * (i - N // 2) * xj) for i in range(N)) for xj in x])


def brute_2d(fhat, x):
    N0, N1 = fhat.shape
    out = []
    for x0, x1 in x:
        s = 0j
        for i0 in range(N0):
            for i1 in range(N1):
                s += fhat[i0, i1] * cmath.exp(-2j * math.pi * ((i0 - N0 // 2) * x0 + (i1 - N1 // 2) * x1))
        out.append(s)
    return np.array(out)


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("N", [2, 4, 6, 10])
def test_1d_brute_force(N):
    rng = np.random.default_rng(N)
    fh = rand_c(rng, N)
    x = rng.uniform(-3, 3, (17, 1))
    np.testing.assert_allclose(oracle.ndft_lowdim(fh, x), brute_1d(fh, x[:, 0]), rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [(2, 4), (6, 2), (4, 8)])
def test_2d_brute_force(N):
    rng = np.random.default_rng(sum(N))
    fh = rand_c(rng, N)
    x = rng.uniform(-2, 2, (13, 2))
    np.testing.assert_allclose(oracle.ndft_lowdim(fh, x), brute_2d(fh, x), rtol=0, atol=1e-13)


@pytest.mark.parametrize("N", [(16,), (64,), (8, 12), (32, 16)])
def test_regular_grid_is_an_fft(N):
    # x_j = j/N - 1/2: f = fftn(ifftshift(fhat (-1)^sum k)) (the sign from e^{i pi k})
    rng = np.random.default_rng(7)
    fh = rand_c(rng, N)
    grids = np.meshgrid(*[np.arange(n) / n - 0.5 for n in N], indexing="ij")
    x = np.stack([g.reshape(-1) for g in grids], axis=1)
    ks = np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij")
    sign = (-1.0) ** (sum(ks) % 2)
    want = np.fft.fftn(np.fft.ifftshift(fh * sign)).reshape(-1)
    np.testing.assert_allclose(oracle.ndft_lowdim(fh, x), want, rtol=0, atol=1e-11 * np.abs(fh).sum())


@pytest.mark.parametrize("N", [(8,), (6, 10)])
def test_single_mode_closed_form(N):
    rng = np.random.default_rng(3)
    x = rng.uniform(-0.5, 0.5, (50, len(N)))
    for corner in [tuple(0 for _ in N), tuple(n - 1 for n in N), tuple(n // 2 for n in N)]:
        fh = np.zeros(N, dtype=np.complex128)
        fh[corner] = 1.0
        k = np.array([c - n // 2 for c, n in zip(corner, N)], dtype=np.float64)
        want = np.exp(-2j * np.pi * (x @ k))
        np.testing.assert_allclose(oracle.ndft_lowdim(fh, x), want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("N", [(12,), (6, 8)])
def test_adjoint_dot_and_brute(N):
    rng = np.random.default_rng(11)
    fh = rand_c(rng, N)
    x = rng.uniform(-0.5, 0.5, (40, len(N)))
    f = rand_c(rng, 40)
    lhs = np.vdot(f, oracle.ndft_lowdim(fh, x))
    rhs = np.vdot(oracle.ndft_lowdim_adjoint(f, x, N), fh)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    # brute force of one coefficient
    idx = tuple(n // 2 - 1 for n in N)
    k = np.array([i - n // 2 for i, n in zip(idx, N)], dtype=np.float64)
    want = sum(f[j] * cmath.exp(2j * math.pi * float(x[j] @ k)) for j in range(40))
    assert abs(oracle.ndft_lowdim_adjoint(f, x, N)[idx] - want) < 1e-12


@pytest.mark.parametrize("N", [(16,), (8, 6)])
def test_grad_is_the_derivative(N):
    rng = np.random.default_rng(5)
    fh = rand_c(rng, N)
    x = rng.uniform(-0.5, 0.5, (20, len(N)))
    g = oracle.ndft_lowdim_grad(fh, x)
    h = 1e-4
    for d in range(len(N)):
        e = np.zeros(len(N))
        e[d] = h
        fd = (-oracle.ndft_lowdim(fh, x + 2 * e) + 8 * oracle.ndft_lowdim(fh, x + e)
              - 8 * oracle.ndft_lowdim(fh, x - e) + oracle.ndft_lowdim(fh, x - 2 * e)) / (12 * h)
        np.testing.assert_allclose(g[:, d], fd, rtol=0, atol=1e-8 * np.abs(fh).sum() * max(N) ** 2)


def test_infft_1d_matches_appendix_product():
    # Appendix B: E = exp(2 pi i (xi - a) k / (b - a)) / sqrt(b - a), psi = E psihat,
    # written here with literal complex exponentials
    rng = np.random.default_rng(2)
    N, a, b = 10, -1.5, 2.5
    ph = rand_c(rng, N)
    xi = rng.uniform(-6, 6, 25)
    want = np.array([sum(ph[i] * cmath.exp(2j * math.pi * (xj - a) * (i - N // 2) / (b - a)) for i in range(N))
                     for xj in xi]) / math.sqrt(b - a)
    np.testing.assert_allclose(oracle.infft_lowdim(ph, [a], [b], xi[:, None]), want, rtol=0, atol=1e-13)


def test_infft_2d_literal():
    rng = np.random.default_rng(4)
    N, a, b = (4, 6), np.array([-1.0, 0.5]), np.array([3.0, 2.0])
    ph = rand_c(rng, N)
    xi = rng.uniform(-4, 4, (9, 2))
    want = []
    for p in xi:
        s = 0j
        for i0 in range(N[0]):
            for i1 in range(N[1]):
                s += ph[i0, i1] * cmath.exp(2j * math.pi * ((i0 - N[0] // 2) * (p[0] - a[0]) / (b[0] - a[0])
                                                          + (i1 - N[1] // 2) * (p[1] - a[1]) / (b[1] - a[1])))
        want.append(s / math.sqrt((b[0] - a[0]) * (b[1] - a[1])))
    np.testing.assert_allclose(oracle.infft_lowdim(ph, a, b, xi), np.array(want), rtol=0, atol=1e-13)


def test_rgrid_lowdim_is_the_series_on_the_tensor_grid():
    rng = np.random.default_rng(8)
    fh = rand_c(rng, (6, 8))
    y0, y1 = rng.uniform(-1, 1, 5), rng.uniform(-1, 1, 7)
    F = oracle.rgrid_lowdim(fh, y0, y1)
    pts = np.array([(u, v) for u in y0 for v in y1])
    np.testing.assert_allclose(F.reshape(-1), brute_2d(fh, pts), rtol=0, atol=1e-13)
    f1 = rand_c(rng, 12)
    np.testing.assert_allclose(oracle.rgrid_lowdim(f1, y0), brute_1d(f1, y0), rtol=0, atol=1e-13)


def test_2d_is_separable_for_rank_one_coefficients():
    # fhat = u v^T  =>  f(x) = (sum_k0 u e^{-2 pi i k0 x0}) (sum_k1 v e^{-2 pi i k1 x1})
    rng = np.random.default_rng(9)
    u, v = rand_c(rng, 8), rand_c(rng, 6)
    x = rng.uniform(-0.5, 0.5, (30, 2))
    want = oracle.ndft_lowdim(u, x[:, :1]) * oracle.ndft_lowdim(v, x[:, 1:])
    np.testing.assert_allclose(oracle.ndft_lowdim(np.outer(u, v), x), want, rtol=0, atol=1e-12)
