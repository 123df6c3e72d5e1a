"""Pins of the oracle's physical-domain evaluation (eq. (fs)), trapezoidal
coefficients (Sec. 2) and vortex-tube refinement (Sec. 4.3)."""
import cmath
import math

import numpy as np
import pytest

import oracle


def _rand(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


A = np.array([-3.0, 1.5, -0.25])
B = np.array([5.0, 2.75, 4.0])


def test_direct_sum_is_eq_fs_written_out():
    """Literal eq. (fs) with cmath, 1-based k as in the paper, on tiny N."""
    N = (2, 4, 6)
    ph = _rand(N, 1)
    xi = np.random.default_rng(2).uniform(A, B, size=(7, 3))
    got = oracle.infftm_eval(ph, A, B, xi)
    for m in range(xi.shape[0]):
        acc = 0j
        for k1 in range(1, N[0] + 1):
            for k2 in range(1, N[1] + 1):
                for k3 in range(1, N[2] + 1):
                    e = 1.0 + 0j
                    for d, kd in enumerate((k1, k2, k3)):
                        L = B[d] - A[d]
                        e *= cmath.exp(2j * math.pi * (kd - 1 - N[d] / 2) * (xi[m, d] - A[d]) / L) / math.sqrt(L)
                    acc += ph[k1 - 1, k2 - 1, k3 - 1] * e
        assert abs(got[m] - acc) <= 1e-13 * max(1.0, abs(acc))


def test_interpolation_and_parseval_on_regular_grid():
    """Sec. 2: the series built from samples by the trapezoidal rule
    interpolates them at X_N, and sum |psihat|^2 = h1 h2 h3 sum |psi(x_n)|^2."""
    N = (8, 6, 10)
    psi = _rand(N, 3)
    ph = oracle.infftm_coeffs(psi, A, B)
    X = oracle.regular_grid(N, A, B)
    vals = oracle.infftm_eval(ph, A, B, X).reshape(N)
    assert np.max(np.abs(vals - psi)) <= 1e-12 * np.max(np.abs(psi))
    h = (B - A) / np.asarray(N)
    assert abs(np.sum(np.abs(ph) ** 2) - np.prod(h) * np.sum(np.abs(vals) ** 2)) <= 1e-12 * np.sum(np.abs(ph) ** 2)


def test_tube_refinement_structure():
    """Each level keeps the points with rho <= rhobar and puts a 27-point
    grid of step h/3^l around each; a threshold above max rho keeps all of
    X_N, one below min rho keeps none."""
    N = (6, 8, 4)
    ph = _rand(N, 4) / 50
    X = oracle.regular_grid(N, A, B)
    rho0 = np.abs(oracle.infftm_eval(ph, A, B, X)) ** 2
    pts, rho, kept = oracle.tube_refine(ph, A, B, [rho0.max() + 1.0])
    assert kept == [X.shape[0]] and pts.shape == (27 * X.shape[0], 3)
    h = (B - A) / np.asarray(N)
    c = pts.reshape(-1, 27, 3)[:, 13, :]                 # centre of each little grid
    assert np.allclose(c, X)
    assert np.allclose(pts.reshape(-1, 27, 3)[:, 0, :], X - h / 3)
    assert np.allclose(rho, np.abs(oracle.infftm_eval(ph, A, B, pts)) ** 2)
    med = float(np.median(rho0))
    pts2, rho2, kept2 = oracle.tube_refine(ph, A, B, [med, np.median(rho)])
    assert kept2[0] == int(np.sum(rho0 <= med)) and pts2.shape[0] == 27 * kept2[1]
    _, _, kept3 = oracle.tube_refine(ph, A, B, [rho0.min() - 1.0])
    assert kept3 == [0]
