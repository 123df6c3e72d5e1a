"""Pins for the numpy statement of the windowed algorithm (oracle.nfft_steps).

* the window / Fourier-transform pair is checked by numerical quadrature
  (scipy.integrate.quad), independent of the closed forms in the module;
* the whole windowed map agrees with the direct-sum oracle within the
  Kaiser-Bessel error estimate, and the error falls with m as that estimate does;
* the adjoint steps are the exact transpose of the forward steps (dot test to
  rounding) and agree with the direct adjoint sum within the estimate;
* the window derivative matches a central difference of the window, and the
  point gradient agrees with the direct derivative sum.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from oracle import nfft_steps as ns


def _coeffs(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def _pts(M, seed):
    return np.random.default_rng(seed).uniform(-0.5, 0.5, size=(M, 3))


@pytest.mark.parametrize("m,sigma", [(2, 2.0), (4, 2.0), (6, 2.0), (8, 2.0), (4, 1.5)])
def test_window_transform_pair_by_quadrature(m, sigma):
    """int_{-m}^{m} phi(t) exp(2 pi i k t / n) dt = I0(m sqrt(b^2 - (2 pi k/n)^2)) up to
    the truncation tail, for |k| <= N/2."""
    n = 64
    N = int(round(n / sigma))
    worst = 0.0
    for k in [0, 1, 5, N // 4, N // 2 - 1, N // 2]:
        val, _ = integrate.quad(lambda t: ns.kb_phi(np.array([t]), m, sigma)[0] * math.cos(2 * math.pi * k * t / n),
                                -m, m, limit=400, epsabs=0, epsrel=1e-13)
        ref = ns.kb_phihat_scaled(np.array([k]), n, m, sigma)[0]
        worst = max(worst, abs(val - ref) / ref)
    # the dropped tail of the window (|t| > m) is what the truncation error measures
    assert worst < 50 * ns.pst_error_bound(m, sigma), worst


def test_window_derivative_vs_central_difference():
    for m in (4, 8):
        t = np.linspace(-m + 1e-3, m - 1e-3, 301)
        h = 1e-5
        fd = (ns.kb_phi(t + h, m, 2.0) - ns.kb_phi(t - h, m, 2.0)) / (2 * h)
        an = ns.kb_phi_deriv(t, m, 2.0)
        assert np.max(np.abs(fd - an)) / np.max(np.abs(an)) < 1e-8


def test_window_even_and_peaked():
    t = np.linspace(0, 8, 50)
    assert np.allclose(ns.kb_phi(t, 8, 2.0), ns.kb_phi(-t, 8, 2.0), rtol=0, atol=0)
    assert np.all(np.diff(ns.kb_phi(t, 8, 2.0)) < 0)
    assert ns.kb_phi(np.array([8.0001]), 8, 2.0)[0] == 0.0


@pytest.mark.parametrize("m", [2, 3, 4, 6, 8])
def test_windowed_map_within_error_estimate(m):
    N = (16, 12, 20)
    fh = _coeffs(N, 60 + m)
    x = _pts(300, 70 + m)
    ref = oracle.ndft_trafo(fh, x)
    got = ns.trafo(fh, x, m, 2.0)
    err = np.max(np.abs(got - ref))
    bound = ns.pst_error_bound(m, 2.0) * np.sum(np.abs(fh))
    assert err <= max(bound, 1e-13 * np.sum(np.abs(fh))), (m, err, bound)


@pytest.mark.parametrize("sigma,ms", [(2.0, (2, 3, 4, 5, 6, 7)), (1.5, (2, 3, 4, 5, 6, 7, 8))])
def test_error_estimate_is_tight_on_band_edge_modes(sigma, ms):
    """Both sides of E(m, sigma): single modes at the corners and edges of
    I_N (where the window's transform is smallest, so the aliasing error is
    largest) and an interior mode, at random points.  The worst error of the
    windowed map, relative to ||fhat||_1 = 1, lies within a factor 4 of E on
    either side (measured 0.49 - 1.26 E); a wrong factor or exponent in E
    (e.g. (1 - 1/sigma) in place of its square root, 180x looser at m = 4)
    fails one side.  m = 8 at sigma = 2 is left out: there E = 4e-14 is
    below the FP64 rounding of the numpy steps."""
    N = (16, 16, 16)
    x = _pts(400, 5)
    for m in ms:
        worst = 0.0
        for kstar in [(0, 0, 0), (0, 8, 0), (15, 15, 15), (0, 0, 8), (8, 8, 8)]:
            fh = np.zeros(N, dtype=np.complex128)
            fh[kstar] = 1.0
            err = np.max(np.abs(ns.trafo(fh, x, m, sigma) - oracle.ndft_trafo(fh, x)))
            worst = max(worst, err)
        E = ns.pst_error_bound(m, sigma)
        assert E / 4 <= worst <= 4 * E, (sigma, m, worst, E, worst / E)


def test_error_decreases_with_m():
    N = (16, 16, 16)
    fh = _coeffs(N, 80)
    x = _pts(200, 81)
    ref = oracle.ndft_trafo(fh, x)
    errs = [oracle.rel_errors(ns.trafo(fh, x, m, 2.0), ref)[0] for m in (2, 3, 4, 5, 6)]
    assert all(a > 10 * b for a, b in zip(errs[:-1], errs[1:])), errs


def test_nonsquare_sigma():
    """sigma = 1.5 (n = 1.5 N) also converges."""
    N = (16, 8, 12)
    fh = _coeffs(N, 82)
    x = _pts(150, 83)
    ref = oracle.ndft_trafo(fh, x)
    got = ns.trafo(fh, x, 6, 1.5)
    assert np.max(np.abs(got - ref)) <= ns.pst_error_bound(6, 1.5) * np.sum(np.abs(fh))


def test_adjoint_steps_are_exact_transpose():
    N = (8, 10, 6)
    m = 3
    fh = _coeffs(N, 90)
    x = _pts(64, 91)
    r = np.random.default_rng(92)
    y = r.standard_normal(64) + 1j * r.standard_normal(64)
    lhs = np.vdot(y, ns.trafo(fh, x, m, 2.0))
    rhs = np.vdot(ns.adjoint(y, x, N, m, 2.0), fh)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_adjoint_steps_vs_direct_sum():
    N = (12, 8, 10)
    x = _pts(120, 93)
    r = np.random.default_rng(94)
    y = r.standard_normal(120) + 1j * r.standard_normal(120)
    ref = oracle.ndft_adjoint(y, x, N)
    got = ns.adjoint(y, x, N, 6, 2.0)
    assert np.max(np.abs(got - ref)) <= ns.pst_error_bound(6, 2.0) * np.sum(np.abs(y))


def test_grad_steps_vs_direct_derivative():
    N = (12, 10, 8)
    fh = _coeffs(N, 95)
    x = _pts(80, 96)
    ref = oracle.ndft_grad(fh, x)
    got = ns.grad_points(fh, x, 8, 2.0)
    l2, _ = oracle.rel_errors(got, ref)
    assert l2 < 1e-11, l2


_BOUND_MUTANTS = {
    # (1 - 1/sigma) in place of its square root in the exponent
    "exponent_without_sqrt": lambda m, s: 4 * math.pi * (math.sqrt(m) + m) * (1 - 1 / s) ** 0.25
    * math.exp(-2 * math.pi * m * (1 - 1 / s)),
    "dropped_4pi": lambda m, s: _TRUE_BOUND(m, s) / (4 * math.pi),
    "dropped_m_factor": lambda m, s: _TRUE_BOUND(m, s) / (math.sqrt(m) + m),
    "pi_for_2pi": lambda m, s: 4 * math.pi * (math.sqrt(m) + m) * (1 - 1 / s) ** 0.25
    * math.exp(-math.pi * m * math.sqrt(1 - 1 / s)),
    "m_off_by_one": lambda m, s: _TRUE_BOUND(m + 1, s),
}
_TRUE_BOUND = ns.pst_error_bound


@pytest.mark.parametrize("mutant", sorted(_BOUND_MUTANTS))
def test_planted_mistakes_in_error_estimate(mutant, monkeypatch):
    """Each plausible mistake in E(m, sigma) fails the two-sided pin."""
    monkeypatch.setattr(ns, "pst_error_bound", _BOUND_MUTANTS[mutant])
    failed = False
    for sigma, ms in [(2.0, (2, 4, 6)), (1.5, (3, 5, 8))]:
        try:
            test_error_estimate_is_tight_on_band_edge_modes(sigma, ms)
        except AssertionError:
            failed = True
    assert failed, mutant
