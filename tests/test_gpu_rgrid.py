"""Evaluation at a rectilinear grid (Sec. 2.1) on the matrix cores, against
the oracle's nested sums (every output), numpy's FFT on the regular grid (the
paper's 64^3 -> 64^3 experiment), and the direct sum at sampled points of a
256^3 -> 321^3 grid."""
import numpy as np
import pytest

import oracle
from gpu_common import log, rand_coeffs, rel, to_dev, torch_dtype

pytestmark = pytest.mark.gpu

EPS = {"c128": np.finfo(np.float64).eps, "c64": np.finfo(np.float32).eps}


def gate(N, dtype):
    """Three chained complex products with contraction lengths N0, N1, N2 and
    tables rounded once: rounding error below 4 (N0 + N1 + N2) eps relative
    to the result (a generous worst case; random data sit far below it)."""
    return max(4.0 * sum(N) * EPS[dtype], 1e-13)


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available()
    import paper_1605_01244_amd as mod
    return mod


def _run(nf, N, ys, fh, dtype):
    import torch
    g = nf.RectGrid(N, [len(y) for y in ys], dtype=torch_dtype(dtype), device="cuda:0")
    g.set_axes(*[torch.from_numpy(np.ascontiguousarray(y)).to("cuda:0") for y in ys])
    out = g.eval(to_dev(fh, dtype)).cpu().numpy()
    g.close()
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("N,M", [((16, 16, 16), (16, 16, 16)), ((8, 12, 20), (70, 3, 129)), ((2, 4, 2), (1, 1, 1)),
                                 ((32, 6, 66), (65, 64, 63)), ((64, 64, 64), (40, 33, 100))])
def test_rgrid_matches_nested_sums(nf, N, M, dtype):
    """Ragged sizes (tiles of 64 x 64 x 16 cut at every edge), M = 1, N != M."""
    fh = rand_coeffs(N, 11)
    r = np.random.default_rng(12)
    ys = [r.uniform(-0.5, 0.5, size=m) for m in M]
    log(f"rgrid N={N} M={M} {dtype}")
    got = _run(nf, N, ys, fh, dtype)
    ref = oracle.rgrid_eval(fh, *ys)
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.2e} rel-linf {li:.2e} (gate {gate(N, dtype):.1e})")
    assert l2 <= gate(N, dtype) and li <= gate(N, dtype), (l2, li)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_rgrid_regular_64_is_the_fft(nf, dtype):
    """64^3 random coefficients at the regular 64^3 grid (the timing
    experiment of Sec. 2.1): the series there is an FFT of the coefficients."""
    N = (64, 64, 64)
    fh = rand_coeffs(N, 13)
    ys = [np.arange(n) / n - 0.5 for n in N]
    log(f"rgrid regular 64^3 {dtype}")
    got = _run(nf, N, ys, fh, dtype)
    I = np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij")
    ref = np.fft.fftn(np.fft.ifftshift(fh * (-1.0) ** (I[0] + I[1] + I[2])))
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.2e} rel-linf {li:.2e} (gate {gate(N, dtype):.1e})")
    assert l2 <= gate(N, dtype) and li <= gate(N, dtype), (l2, li)


def test_rgrid_far_coordinates_and_periodicity(nf):
    """Coordinates far from the unit box give the values at their folded
    positions (exact phase reduction): y and y + 1000 agree to rounding."""
    N, M = (10, 8, 12), (7, 9, 5)
    fh = rand_coeffs(N, 14)
    r = np.random.default_rng(15)
    ys = [r.uniform(-0.5, 0.5, size=m) for m in M]
    far = [y + 1000.0 for y in ys]
    a = _run(nf, N, ys, fh, "c128")
    b = _run(nf, N, far, fh, "c128")
    ref = oracle.rgrid_eval(fh, *far)
    assert rel(b, ref)[1] <= gate(N, "c128")
    assert rel(a, b)[1] <= 1e-11       # the shift's own rounding in y (1000 + y)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_rgrid_256_to_321_sampled(nf, dtype):
    """N = 256^3 coefficients (power law) at a 321^3 nonuniform rectilinear
    grid, 400 sampled outputs against the direct sum."""
    import torch
    import workloads
    N, M = (256, 256, 256), (321, 321, 321)
    fh = workloads.powerlaw_coeffs((256, 256, 256), 301)
    r = np.random.default_rng(16)
    ys = [np.sort(r.uniform(-0.5, 0.5, size=m)) for m in M]
    log(f"rgrid 256^3 -> 321^3 {dtype}")
    g = nf.RectGrid(N, M, dtype=torch_dtype(dtype), device="cuda:0")
    g.set_axes(*[torch.from_numpy(y).to("cuda:0") for y in ys])
    out = g.eval(to_dev(fh, dtype))
    s = np.random.default_rng(17).integers(0, M, size=(400, 3))
    got = out[tuple(torch.from_numpy(s[:, d]).to("cuda:0") for d in range(3))].cpu().numpy()
    pts = np.stack([ys[d][s[:, d]] for d in range(3)], axis=1)
    ref = oracle.ndft_trafo(fh, pts)
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.2e} rel-linf {li:.2e}")
    assert l2 <= gate(N, dtype) and li <= gate(N, dtype), (l2, li)
    g.close()
    del out
    torch.cuda.empty_cache()


def test_rgrid_errors(nf):
    import torch
    with pytest.raises(nf.NFFT3Error) as e:
        nf.RectGrid((7, 8, 8), (4, 4, 4), device="cuda:0")
    assert e.value.code == -1
    g = nf.RectGrid((8, 8, 8), (4, 5, 6), device="cuda:0")
    fh = to_dev(rand_coeffs((8, 8, 8), 1), "c128")
    with pytest.raises(nf.NFFT3Error) as e:
        g.eval(fh)
    assert e.value.code == -4          # no axes yet
    y = [torch.zeros(m, dtype=torch.float64, device="cuda:0") for m in (4, 5, 6)]
    y[1][2] = float("inf")
    with pytest.raises(nf.NFFT3Error) as e:
        g.set_axes(*y)
    assert e.value.code == -5
    g.close()
