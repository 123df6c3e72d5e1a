"""Pins of the oracle's GPE time splitting (Sec. 3.1): exact plane-wave
solutions, conservation of the discrete mass, time reversibility and second
order in time."""
import numpy as np

import oracle

A = np.array([-20.0, -20.0, -20.0])
B = np.array([60.0, 40.0, 20.0])


def test_plane_waves_are_exact():
    """psi = c exp(i kappa.x) solves the GPE exactly with
    psi(t) = psi(0) exp(i t (1 - |c|^2 - |kappa|^2) / 2): both split flows are
    exact for it, so the scheme returns it to rounding for any tau."""
    N = (16, 12, 8)
    X = oracle.regular_grid(N, A, B)
    for kidx, c in (((1, -2, 3), 1.0), ((0, 5, -1), 0.7 + 0.2j), ((-8, 6, 4), 1.3)):
        kap = 2 * np.pi * np.asarray(kidx) / (B - A)
        psi0 = (c * np.exp(1j * (X @ kap))).reshape(N)
        tau, n = 0.37, 9
        t = tau * n
        ref = psi0 * np.exp(0.5j * t * (1 - abs(c) ** 2 - kap @ kap))
        got = oracle.gpe_tssp(psi0, A, B, tau, n)
        assert np.max(np.abs(got - ref)) <= 1e-12


def test_mass_conserved_and_reversible():
    N = (12, 10, 8)
    r = np.random.default_rng(1)
    psi0 = 1 + 0.3 * (r.standard_normal(N) + 1j * r.standard_normal(N))
    p1 = oracle.gpe_tssp(psi0, A, B, 0.05, 20)
    assert abs(np.sum(np.abs(p1) ** 2) - np.sum(np.abs(psi0) ** 2)) <= 1e-12 * np.sum(np.abs(psi0) ** 2)
    back = oracle.gpe_tssp(p1, A, B, -0.05, 20)
    assert np.max(np.abs(back - psi0)) <= 1e-11


def test_second_order_in_time():
    """Halving tau divides the error at a fixed time by about 4."""
    N = (16, 16, 16)
    g = [np.linspace(A[d], B[d], N[d], endpoint=False) for d in range(3)]
    X = np.meshgrid(*g, indexing="ij")
    psi0 = (1.0 + 0.2 * np.exp(1j * 2 * np.pi * X[0] / 80) * np.cos(2 * np.pi * X[1] / 60)
            + 0.1 * np.sin(2 * np.pi * X[2] / 40))
    T = 1.0
    ref = oracle.gpe_tssp(psi0, A, B, T / 512, 512)
    e1 = np.max(np.abs(oracle.gpe_tssp(psi0, A, B, T / 8, 8) - ref))
    e2 = np.max(np.abs(oracle.gpe_tssp(psi0, A, B, T / 16, 16) - ref))
    assert 3.2 < e1 / e2 < 4.8, (e1, e2)
