"""Gross-Pitaevskii time splitting (Sec. 3.1) on the device against the
oracle's numpy splitting, exact plane waves, mass conservation, time
reversibility, and the state's coefficients against the trapezoidal rule."""
import numpy as np
import pytest

import oracle
from gpu_common import log, rel, to_dev, torch_dtype

pytestmark = pytest.mark.gpu

A = np.array([-20.0, -20.0, -20.0])
B = np.array([60.0, 40.0, 20.0])
GATE = {"c128": 1e-12, "c64": 2e-5}


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available()
    import paper_1605_01244_amd as mod
    return mod


def _init(N, seed):
    r = np.random.default_rng(seed)
    return 1 + 0.3 * (r.standard_normal(N) + 1j * r.standard_normal(N))


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("N", [(32, 24, 20), (64, 16, 30), (80, 80, 80)])
def test_gpe_matches_oracle(nf, dtype, N):
    """Strang steps (tau = 0.1) against the numpy splitting, on static and
    generic FFT lengths (80 is the paper's grid)."""
    psi0 = _init(N, 91)
    nsteps = 10 if N[0] < 80 else 4
    log(f"gpe N={N} {dtype}")
    g = nf.GPE(N, A, B, dtype=torch_dtype(dtype), device="cuda:0")
    g.set_state(to_dev(psi0, dtype))
    g.step(0.1, nsteps)
    got = g.state().cpu().numpy()
    ref = oracle.gpe_tssp(psi0, A, B, 0.1, nsteps)
    l2, li = rel(got, ref)
    assert l2 <= GATE[dtype] and li <= GATE[dtype], (l2, li)


def test_gpe_plane_wave_exact(nf):
    N = (32, 20, 16)
    X = oracle.regular_grid(N, A, B)
    kap = 2 * np.pi * np.array([2, -3, 1]) / (B - A)
    c = 0.8 + 0.3j
    psi0 = (c * np.exp(1j * (X @ kap))).reshape(N)
    g = nf.GPE(N, A, B, device="cuda:0")
    g.set_state(to_dev(psi0, "c128"))
    g.step(0.25, 12)
    t = 3.0
    ref = psi0 * np.exp(0.5j * t * (1 - abs(c) ** 2 - kap @ kap))
    assert np.max(np.abs(g.state().cpu().numpy() - ref)) <= 1e-12


def test_gpe_mass_and_reversibility(nf):
    N = (24, 20, 16)
    psi0 = _init(N, 92)
    g = nf.GPE(N, A, B, device="cuda:0")
    g.set_state(to_dev(psi0, "c128"))
    g.step(0.05, 20)
    p1 = g.state().cpu().numpy()
    assert abs(np.sum(np.abs(p1) ** 2) - np.sum(np.abs(psi0) ** 2)) <= 1e-12 * np.sum(np.abs(psi0) ** 2)
    g.step(-0.05, 20)
    assert np.max(np.abs(g.state().cpu().numpy() - psi0)) <= 1e-11


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_gpe_coeffs_are_the_trapezoidal_rule(nf, dtype):
    """The snapshot's coefficients feed the physical-domain evaluation: they
    equal fftshift(fftn(psi)) prod sqrt(L)/N, and the series returns psi at X_N."""
    N = (32, 20, 16)
    psi0 = _init(N, 93)
    g = nf.GPE(N, A, B, dtype=torch_dtype(dtype), device="cuda:0")
    g.set_state(to_dev(psi0, dtype))
    ph = g.coeffs().cpu().numpy()
    ref = oracle.infftm_coeffs(psi0, A, B)
    l2, li = rel(ph, ref)
    assert l2 <= GATE[dtype] and li <= GATE[dtype], (l2, li)
    if dtype == "c128":
        m = 8
        p = nf.Plan(N, m=m, dtype=torch_dtype(dtype), device="cuda:0")
        X = oracle.regular_grid(N, A, B)
        vals = p.infft3(g.coeffs(), A, B, to_dev(X)).cpu().numpy()
        assert rel(vals, psi0.reshape(-1))[1] <= 1e-12


def test_gpe_errors(nf):
    with pytest.raises(nf.NFFT3Error) as e:
        nf.GPE((8, 16, 16), A, B, device="cuda:0")        # fewer than two radix stages on an axis
    assert e.value.code == -1
    with pytest.raises(nf.NFFT3Error) as e:
        nf.GPE((22, 16, 16), A, B, device="cuda:0")       # prime factor 11
    assert e.value.code == -1
