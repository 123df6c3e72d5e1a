"""Pins of the rectilinear-grid oracle (Sec. 2.1): the nested per-axis sums
against the direct sum at every grid point, numpy's FFT on the regular grid,
the single-mode closed form, and planted mistakes."""
import numpy as np
import pytest

import oracle


def _rand(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(N) + 1j * r.standard_normal(N)


def _grid_points(y0, y1, y2):
    Y = np.meshgrid(y0, y1, y2, indexing="ij")
    return np.stack([g.reshape(-1) for g in Y], axis=1)


@pytest.mark.parametrize("N,M", [((4, 6, 8), (5, 7, 3)), ((8, 8, 8), (9, 1, 12)), ((2, 10, 4), (6, 6, 6))])
def test_nested_sums_equal_direct_sum_at_grid_points(N, M):
    fh = _rand(N, 1)
    r = np.random.default_rng(2)
    ys = [r.uniform(-3.0, 3.0, size=Md) for Md in M]       # any real coordinates (periodic)
    F = oracle.rgrid_eval(fh, *ys)
    ref = oracle.ndft_trafo(fh, _grid_points(*ys)).reshape(M)
    assert F.shape == tuple(M)
    assert np.max(np.abs(F - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_regular_grid_is_an_fft():
    """y_d = j/N_d - 1/2 (the regular grid X_N of Sec. 2 on the unit box):
    F = fftn(ifftshift(fhat * (-1)^{sum (i_d - N_d/2)})) (Sec. 2.1's FFT route)."""
    N = (8, 6, 10)
    fh = _rand(N, 3)
    ys = [np.arange(n) / n - 0.5 for n in N]
    F = oracle.rgrid_eval(fh, *ys)
    I = np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij")
    sgn = (-1.0) ** (I[0] + I[1] + I[2])
    ref = np.fft.fftn(np.fft.ifftshift(fh * sgn))
    assert np.max(np.abs(F - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_single_mode_closed_form():
    N = (6, 4, 8)
    r = np.random.default_rng(4)
    ys = [r.uniform(-0.5, 0.5, size=m) for m in (3, 5, 4)]
    for kidx in [(0, 0, 0), (5, 3, 7), (0, 3, 4), (2, 1, 0)]:
        fh = np.zeros(N, dtype=np.complex128)
        fh[kidx] = 1.0
        k = [kidx[d] - N[d] // 2 for d in range(3)]
        F = oracle.rgrid_eval(fh, *ys)
        ref = (np.exp(-2j * np.pi * k[0] * ys[0])[:, None, None] * np.exp(-2j * np.pi * k[1] * ys[1])[None, :, None]
               * np.exp(-2j * np.pi * k[2] * ys[2])[None, None, :])
        assert np.max(np.abs(F - ref)) <= 1e-14


def test_planted_mistakes_fail_the_direct_sum_pin():
    """Mistakes in the nested sums (axes swapped, E not transposed, wrong sign,
    frequencies off by one) each fail the comparison with the direct sum."""
    N, M = (4, 6, 8), (5, 7, 3)
    fh = _rand(N, 5)
    r = np.random.default_rng(6)
    ys = [r.uniform(-0.5, 0.5, size=Md) for Md in M]
    ref = oracle.ndft_trafo(fh, _grid_points(*ys)).reshape(M)
    E0, E1, E2 = (oracle.axis_phases(N[d], ys[d]) for d in range(3))

    def nested(fh, E0, E1, E2):
        N0, N1, N2 = fh.shape
        t = (fh.reshape(N0 * N1, N2) @ E2.T).reshape(N0, N1, -1)
        t = np.matmul(E1[None], t)
        return (E0 @ t.reshape(N0, -1)).reshape(E0.shape[0], E1.shape[0], E2.shape[0])

    assert np.max(np.abs(nested(fh, E0, E1, E2) - ref)) <= 1e-13 * np.max(np.abs(ref))
    bad = [
        nested(fh, E0, E1, np.conj(E2)),                                       # wrong sign on one axis
        nested(fh, E0, E1, oracle.axis_phases(N[2], ys[2]) * np.exp(-2j * np.pi * ys[2])[:, None]),  # k off by one
        nested(fh[:, ::-1, :], E0, E1, E2),                                    # frequencies reversed on axis 1
        nested(np.ascontiguousarray(np.swapaxes(fh, 0, 2)).reshape(N), E0, E1, E2),  # axes 0 and 2 mixed up
    ]
    for b in bad:
        assert np.max(np.abs(b - ref)) > 1e-3 * np.max(np.abs(ref))
