"""Pins for the direct-sum oracle (oracle.ndft_*), all on the CPU.

Each pin checks the oracle against something other than itself:
closed forms of the problem statement (Sec. 2.2.1), numpy's FFT on the
regular grid (Sec. 2.1), Parseval (Sec. 2), a literal brute-force sum with no
tables, and algebraic invariants.  ``test_planted_mistakes`` shows that
plausible mistakes (transposed axes, wrong sign, shifted index, conjugation,
dropped factor) each fail at least one pin.
"""
import cmath
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle

RNG = np.random.default_rng(12345)


def _rand_coeffs(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def _rand_points(M, seed):
    return np.random.default_rng(seed).uniform(-0.5, 0.5, size=(M, 3))


def _freqs(n):
    return np.arange(n) - n // 2


# ---------------------------------------------------------------- pins ----
# Each pin takes a trafo-like callable T(fhat, x) -> f and returns the error
# measure it checks; the tests assert these are at rounding level.

def pin_single_mode(T, N=(8, 6, 4), M=40, seed=1):
    """fhat = delta_{k*} gives exactly f_j = exp(-2 pi i k*.x_j)."""
    x = _rand_points(M, seed)
    worst = 0.0
    ks = [(-N[0] // 2, -N[1] // 2, -N[2] // 2), (N[0] // 2 - 1, N[1] // 2 - 1, N[2] // 2 - 1),
          (-N[0] // 2, N[1] // 2 - 1, 0), (0, 0, 0), (1, -2, 1), (3, 0, -1), (-1, 2, -2)]
    for k in ks:
        fhat = np.zeros(N, dtype=np.complex128)
        fhat[k[0] + N[0] // 2, k[1] + N[1] // 2, k[2] + N[2] // 2] = 1.0
        f = T(fhat, x)
        ref = np.exp(-2j * np.pi * (x @ np.asarray(k, dtype=np.float64)))
        worst = max(worst, float(np.max(np.abs(f - ref))))
    return worst


def pin_regular_grid(T, N=(8, 6, 10), seed=2):
    """On x_n = n/N - 1/2 the sum is an FFT: f = fftn(ifftshift((-1)^{sum k} fhat))."""
    fhat = _rand_coeffs(N, seed)
    g = [np.arange(n) / n - 0.5 for n in N]
    X = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    k0, k1, k2 = np.meshgrid(*[_freqs(n) for n in N], indexing="ij")
    s = 1 - 2 * ((k0 + k1 + k2) & 1)
    ref = np.fft.fftn(np.fft.ifftshift(fhat * s)).reshape(-1)
    f = T(fhat, X)
    return float(np.max(np.abs(f - ref)) / np.max(np.abs(ref)))


def pin_parseval(T, N=(6, 8, 4), seed=3):
    """On the regular grid sum |f|^2 = N0 N1 N2 sum |fhat|^2 (Sec. 2)."""
    fhat = _rand_coeffs(N, seed)
    g = [np.arange(n) / n - 0.5 for n in N]
    X = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    f = T(fhat, X)
    lhs = np.sum(np.abs(f) ** 2)
    rhs = np.prod(N) * np.sum(np.abs(fhat) ** 2)
    return float(abs(lhs - rhs) / rhs)


def brute_force(fhat, x):
    """Literal sum over every k with cmath.exp, no tables or argument reduction."""
    N = fhat.shape
    out = np.zeros(x.shape[0], dtype=np.complex128)
    for j in range(x.shape[0]):
        s = 0j
        for a in range(N[0]):
            for b in range(N[1]):
                for c in range(N[2]):
                    k = (a - N[0] // 2, b - N[1] // 2, c - N[2] // 2)
                    s += complex(fhat[a, b, c]) * cmath.exp(
                        -2j * math.pi * (k[0] * x[j, 0] + k[1] * x[j, 1] + k[2] * x[j, 2]))
        out[j] = s
    return out


def pin_brute_force(T, N=(4, 2, 6), M=12, seed=4):
    fhat = _rand_coeffs(N, seed)
    x = _rand_points(M, seed + 1)
    ref = brute_force(fhat, x)
    return float(np.max(np.abs(T(fhat, x) - ref)) / np.sum(np.abs(fhat)))


def pin_shift(T, N=(8, 4, 6), M=30, seed=5):
    """f(x + delta) with fhat equals f(x) with fhat_k exp(-2 pi i k.delta)."""
    fhat = _rand_coeffs(N, seed)
    x = _rand_points(M, seed + 1) * 0.5
    delta = np.array([0.137, -0.021, 0.3])
    k0, k1, k2 = np.meshgrid(*[_freqs(n) for n in N], indexing="ij")
    mod = np.exp(-2j * np.pi * (k0 * delta[0] + k1 * delta[1] + k2 * delta[2]))
    a = T(fhat, x + delta)
    b = T(fhat * mod, x)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(a)))


PINS = {
    "single_mode": pin_single_mode,
    "regular_grid": pin_regular_grid,
    "parseval": pin_parseval,
    "brute_force": pin_brute_force,
    "shift": pin_shift,
}
TOL = 1e-13


@pytest.mark.parametrize("name", sorted(PINS))
def test_trafo_pins(name):
    err = PINS[name](oracle.ndft_trafo)
    assert err < TOL, (name, err)


def test_single_mode_far_frequency():
    """Exact argument reduction: |k| = 128 modes stay exact to 1e-14."""
    N = (256, 2, 2)
    x = _rand_points(64, 9)
    for k0 in (-128, 127, 77):
        fhat = np.zeros(N, dtype=np.complex128)
        fhat[k0 + 128, 1, 1] = 1.0
        f = oracle.ndft_trafo(fhat, x)
        # reference phase reduced modulo 1 in exact rational arithmetic
        r = [float((Fraction(k0) * Fraction(float(v))) % 1) for v in x[:, 0]]
        ref = np.exp(-2j * np.pi * np.asarray(r))
        assert np.max(np.abs(f - ref)) < 1e-14


def test_periodicity_and_linearity():
    N = (6, 4, 8)
    fa, fb = _rand_coeffs(N, 20), _rand_coeffs(N, 21)
    x = _rand_points(25, 22)
    a = oracle.ndft_trafo(fa, x)
    # integer shifts of the points do not change the sum
    assert np.max(np.abs(oracle.ndft_trafo(fa, x + np.array([1.0, -2.0, 3.0])) - a)) < 1e-12
    lin = oracle.ndft_trafo(2.5 * fa - 1j * fb, x)
    ref = 2.5 * a - 1j * oracle.ndft_trafo(fb, x)
    assert np.max(np.abs(lin - ref)) < 1e-12


def test_threads_agree():
    N = (8, 8, 8)
    fh = _rand_coeffs(N, 30)
    x = _rand_points(37, 31)
    a = oracle.ndft_trafo(fh, x, threads=1)
    b = oracle.ndft_trafo(fh, x, threads=7)
    assert np.array_equal(a, b)
    ya = oracle.ndft_adjoint(a, x, N, threads=1)
    yb = oracle.ndft_adjoint(a, x, N, threads=5)
    assert np.array_equal(ya, yb)


def test_empty_points():
    N = (4, 4, 4)
    f = oracle.ndft_trafo(_rand_coeffs(N, 1), np.zeros((0, 3)))
    assert f.shape == (0,)
    a = oracle.ndft_adjoint(np.zeros(0), np.zeros((0, 3)), N)
    assert a.shape == N and not np.any(a)


def test_rejects_odd_sizes():
    with pytest.raises(ValueError):
        oracle.ndft_trafo(np.zeros((3, 4, 4), dtype=complex), np.zeros((1, 3)))


# ---------------------------------------------------------- adjoint ----

def test_adjoint_single_point_closed_form():
    """f = delta_j gives fhat_k = exp(+2 pi i k.x_j)."""
    N = (6, 4, 8)
    x = _rand_points(5, 40)
    f = np.zeros(5, dtype=np.complex128)
    f[3] = 1.0
    out = oracle.ndft_adjoint(f, x, N)
    k0, k1, k2 = np.meshgrid(*[_freqs(n) for n in N], indexing="ij")
    ref = np.exp(2j * np.pi * (k0 * x[3, 0] + k1 * x[3, 1] + k2 * x[3, 2]))
    assert np.max(np.abs(out - ref)) < 1e-13


def test_adjoint_dot_product():
    """<A fhat, y> = <fhat, A^H y> (the adjoint is the conjugate transpose)."""
    N = (8, 6, 4)
    fh = _rand_coeffs(N, 41)
    x = _rand_points(50, 42)
    r = np.random.default_rng(43)
    y = r.standard_normal(50) + 1j * r.standard_normal(50)
    lhs = np.vdot(y, oracle.ndft_trafo(fh, x))
    rhs = np.vdot(oracle.ndft_adjoint(y, x, N), fh)
    assert abs(lhs - rhs) / abs(lhs) < 1e-13


def test_adjoint_brute_force():
    N = (2, 4, 4)
    x = _rand_points(7, 44)
    r = np.random.default_rng(45)
    y = r.standard_normal(7) + 1j * r.standard_normal(7)
    ref = np.zeros(N, dtype=np.complex128)
    for a in range(N[0]):
        for b in range(N[1]):
            for c in range(N[2]):
                k = (a - N[0] // 2, b - N[1] // 2, c - N[2] // 2)
                ref[a, b, c] = sum(complex(y[j]) * cmath.exp(2j * math.pi * (k[0] * x[j, 0] + k[1] * x[j, 1] + k[2] * x[j, 2]))
                                   for j in range(7))
    assert np.max(np.abs(oracle.ndft_adjoint(y, x, N) - ref)) < 1e-13


def test_adjoint_at_sampled_coefficients():
    """The sampled adjoint: the single-point closed form at every corner of
    I_N and at random indices, and agreement with the full adjoint (a
    separate code path: per-axis exponential tables, slabs of k0) on many
    points, including large |k| where phase reduction matters."""
    N = (16, 12, 256)
    corners = np.array([[a, b, c] for a in (0, N[0] - 1) for b in (0, N[1] - 1) for c in (0, N[2] - 1)])
    r = np.random.default_rng(46)
    kidx = np.concatenate([corners, np.stack([r.integers(0, n, 10) for n in N], axis=1)])
    x = _rand_points(1, 47) * 1000.0 + 0.123456789      # far outside the box: folding by the phase itself
    out = oracle.ndft_adjoint_at(np.ones(1), x, N, kidx)
    k = kidx - np.array(N) // 2
    ref = np.array([cmath.exp(2j * math.pi * math.fsum(float(k[q, d]) * float(x[0, d]) for d in range(3)))
                    for q in range(len(kidx))])
    # the reference phase itself carries the rounding of k.x at |x| ~ 1e3
    assert np.max(np.abs(out - ref)) < 1e-9
    x = _rand_points(3000, 48)
    y = r.standard_normal(3000) + 1j * r.standard_normal(3000)
    full = oracle.ndft_adjoint(y, x, N)
    got = oracle.ndft_adjoint_at(y, x, N, kidx)
    ref = full[kidx[:, 0], kidx[:, 1], kidx[:, 2]]
    assert np.max(np.abs(got - ref)) / np.max(np.abs(full)) < 1e-13
    with pytest.raises(RuntimeError):
        oracle.ndft_adjoint_at(y, x, N, np.array([[0, 0, N[2]]]))


# ------------------------------------------------------------- grad ----

def test_grad_single_mode_closed_form():
    """d/dx_d exp(-2 pi i k*.x) = -2 pi i k*_d exp(-2 pi i k*.x)  (eq. (Lambda))."""
    N = (8, 6, 4)
    x = _rand_points(20, 50)
    for k in [(-4, 2, 1), (3, -3, -2), (0, 1, 0)]:
        fh = np.zeros(N, dtype=np.complex128)
        fh[k[0] + 4, k[1] + 3, k[2] + 2] = 1.0
        g = oracle.ndft_grad(fh, x)
        e = np.exp(-2j * np.pi * (x @ np.asarray(k, float)))
        ref = np.stack([-2j * np.pi * k[d] * e for d in range(3)], axis=1)
        assert np.max(np.abs(g - ref)) < 1e-12


def test_grad_matches_central_differences():
    """4th-order central differences of the trafo oracle, h = 1e-4."""
    N = (8, 6, 10)
    fh = _rand_coeffs(N, 51)
    x = _rand_points(15, 52)
    g = oracle.ndft_grad(fh, x)
    h = 1e-4
    for d in range(3):
        e = np.zeros(3)
        e[d] = h
        fd = (-oracle.ndft_trafo(fh, x + 2 * e) + 8 * oracle.ndft_trafo(fh, x + e)
              - 8 * oracle.ndft_trafo(fh, x - e) + oracle.ndft_trafo(fh, x - 2 * e)) / (12 * h)
        assert np.max(np.abs(fd - g[:, d])) / np.max(np.abs(g[:, d])) < 1e-8


# ---------------------------------------------------- planted mistakes ----

def _mutants():
    T = oracle.ndft_trafo
    return {
        "transposed_coeff_axes": lambda fh, x: T(np.ascontiguousarray(fh.transpose(2, 1, 0)), x),
        "swapped_point_columns": lambda fh, x: T(fh, x[:, [2, 1, 0]].copy()),
        "wrong_sign": lambda fh, x: T(fh, -x),
        "index_off_by_one": lambda fh, x: T(np.roll(fh, 1, axis=1), x),
        "conjugated": lambda fh, x: np.conj(T(fh, x)),
        "half_cell_shift": lambda fh, x: T(fh, x + 0.5 / np.array(fh.shape)),
        "dropped_axis": lambda fh, x: T(fh, x * np.array([1.0, 1.0, 0.0])),
        "scaled_by_two": lambda fh, x: 2.0 * T(fh, x),
    }


@pytest.mark.parametrize("mutant", sorted(_mutants()))
def test_planted_mistakes(mutant):
    T = _mutants()[mutant]
    fails = [name for name, pin in PINS.items() if not pin(T) < TOL]
    assert fails, f"no pin catches the planted mistake {mutant}"
