"""GPU parity: the HIP path (through the C ABI) against the oracle.

Stage tests compare one kernel stage with the numpy statement of the same
windowed step (oracle.nfft_steps) to rounding; end-to-end tests compare with
the direct-sum oracle (oracle.ndft_*) within the m/sigma/dtype tolerance.
"""
import numpy as np
import pytest

import oracle
from oracle import nfft_steps as ns
import workloads
from gpu_common import dot_tol, log, phi0, rand_coeffs, rand_points, rel, stage_tol, to_dev, tol, torch_dtype

pytestmark = pytest.mark.gpu

DTYPES = ["c128", "c64"]


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_1605_01244_amd as mod
    return mod


def make_plan(nf, N, m, dtype, sigma=2.0):
    return nf.Plan(N, sigma=sigma, m=m, dtype=torch_dtype(dtype), device="cuda:0")


# ------------------------------------------------------------- stages ----

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,sigma,m", [((8, 12, 16), 2.0, 3), ((32, 32, 32), 2.0, 6), ((16, 24, 20), 1.5, 4),
                                       ((6, 10, 4), 2.0, 2), ((32, 64, 256), 2.0, 4), ((128, 2, 64), 2.0, 1),
                                       ((48, 96, 192), 2.0, 4), ((14, 28, 42), 2.0, 4), ((56, 70, 98), 2.0, 5),
                                       ((40, 80, 160), 2.0, 4)])
def test_stage_grid_matches_fft_of_deconvolved(nf, N, sigma, m, dtype):
    """Deconvolve + zero-pad + 3-D FFT equals numpy fftn of the textbook
    deconvolved array (GPU window normalised: factor phi(0)^3); lengths with
    factors 2, 3, 5 and 7 (n = 28 ... 196)."""
    log(f"stage_grid N={N} sigma={sigma} m={m} {dtype}")
    fh = rand_coeffs(N, 1)
    p = make_plan(nf, N, m, dtype, sigma)
    for axis in (-1, 0, 2):
        p.stage_grid(to_dev(fh, dtype), axis)
        g = p.grid().cpu().numpy()
        f2 = fh
        if axis >= 0:
            k = (np.arange(N[axis]) - N[axis] // 2).astype(float)
            shape = [1, 1, 1]
            shape[axis] = N[axis]
            f2 = fh * (-2j * np.pi * k.reshape(shape))
        ref = ns.oversampled_grid(f2, m, sigma) * phi0(m, sigma) ** 3
        l2, li = rel(g, ref)
        assert l2 < (1e-14 if dtype == "c128" else 2e-6), (axis, l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,m,M", [((16, 16, 16), 4, 3000), ((8, 12, 10), 3, 777), ((32, 16, 8), 8, 1234)])
def test_stage_interp_matches_window_sum(nf, N, m, M, dtype):
    """Window sum of an arbitrary loaded grid vs the numpy window sum."""
    log(f"stage_interp N={N} m={m} M={M} {dtype}")
    p = make_plan(nf, N, m, dtype)
    r = np.random.default_rng(5)
    g = r.standard_normal(p.n) + 1j * r.standard_normal(p.n)
    x = rand_points(M, 6)
    p.set_points(to_dev(x))
    p.load_grid(to_dev(g, dtype))
    got = p.stage_interp().cpu().numpy()
    ref = ns.interpolate(g, x, m, 2.0) / phi0(m, 2.0) ** 3
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.3g} rel-linf {li:.3g}")
    assert l2 < (1e-14 if dtype == "c128" else 1e-6), (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m", [1, 2, 3, 5, 6, 7, 9, 10])
def test_stage_interp_every_m(nf, m, dtype):
    """Every window width: the stencil-read layout (row stride, rotation
    cosets, complex<float> pair offsets) depends on 2m."""
    N, M = (24, 20, 30), 1500
    log(f"stage_interp N={N} m={m} M={M} {dtype}")
    p = make_plan(nf, N, m, dtype)
    r = np.random.default_rng(50 + m)
    g = r.standard_normal(p.n) + 1j * r.standard_normal(p.n)
    x = rand_points(M, 60 + m)
    p.set_points(to_dev(x))
    p.load_grid(to_dev(g, dtype))
    got = p.stage_interp().cpu().numpy()
    ref = ns.interpolate(g, x, m, 2.0) / phi0(m, 2.0) ** 3
    l2, li = rel(got, ref)
    assert l2 < stage_tol(m, dtype), (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("tile,items", [(8, 256), (8, 512), (16, 256), (20, 512), (24, 256), (28, 512),
                                        (32, 256), (32, 512)])
def test_stage_interp_tunings(nf, tile, items, dtype):
    """Every binning setting gives the same window sums (clustered and
    uniform points, tiles cut by the grid edge)."""
    m = 8 if dtype == "c128" else 4
    N, M = (40, 24, 36), 6000
    log(f"stage_interp tuning tile={tile} items={items} N={N} m={m} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_tuning(tile, items)
    assert p.tuning() == (tile, items)
    r = np.random.default_rng(70)
    g = r.standard_normal(p.n) + 1j * r.standard_normal(p.n)
    x = np.concatenate([rand_points(M // 2, 71),
                        workloads.wrap(0.1 + 0.01 * np.random.default_rng(72).standard_normal((M - M // 2, 3)))])
    p.set_points(to_dev(x))
    p.load_grid(to_dev(g, dtype))
    got = p.stage_interp().cpu().numpy()
    ref = ns.interpolate(g, x, m, 2.0) / phi0(m, 2.0) ** 3
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.3g} rel-linf {li:.3g}")
    assert l2 < (1e-14 if dtype == "c128" else 1e-6), (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
def test_autotune(nf, dtype):
    """The autotuner picks a candidate, leaves the points set, and the
    transform with its choice matches the direct sum."""
    import torch
    m = 8 if dtype == "c128" else 4
    fh, x = workloads.smooth_uniform_case(32, 20_000)
    p = make_plan(nf, fh.shape, m, dtype)
    fd = to_dev(fh, dtype)
    tile, items = p.autotune(to_dev(x), fd, reps=2)
    log(f"autotune {dtype}: tile={tile} items={items}")
    assert tile in (16, 24, 32) and items in (256, 512)
    assert p.tuning() == (tile, items) and p.M == x.shape[0]
    got = p.trafo(fd).cpu().numpy()
    s = workloads.sample_indices(x.shape[0], 2000, 73)
    l2, li = rel(got[s], oracle.ndft_trafo(fh, x[s]))
    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype)
    torch.cuda.synchronize()


@pytest.mark.parametrize("dtype", DTYPES)
def test_stage_spread_matches_numpy(nf, dtype):
    N, m, M = (12, 16, 8), 4, 900
    log(f"stage_spread N={N} m={m} M={M} {dtype}")
    p = make_plan(nf, N, m, dtype)
    x = rand_points(M, 7)
    r = np.random.default_rng(8)
    f = r.standard_normal(M) + 1j * r.standard_normal(M)
    p.set_points(to_dev(x))
    p.stage_spread(to_dev(f, dtype))
    got = p.grid().cpu().numpy()
    ref = ns.spread(f, x, p.n, m, 2.0) / phi0(m, 2.0) ** 3
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.3g} rel-linf {li:.3g}")
    assert l2 < (1e-14 if dtype == "c128" else 1e-6), (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m,tile,items", [(1, 16, 512), (2, 16, 256), (3, 16, 512), (4, 16, 256), (4, 16, 512),
                                          (5, 16, 512), (8, 16, 256), (8, 16, 512), (4, 32, 512), (8, 32, 512),
                                          (4, 8, 256), (6, 28, 512)])
def test_stage_spread_every_m_and_items(nf, m, tile, items, dtype):
    """The spread kernel takes one or two points per thread depending on the
    form and m, and walks each work item in 512-point chunks: ragged item
    sizes, both item settings, several tiles, clustered and uniform points."""
    N, M = (24, 20, 30), 2300
    log(f"stage_spread N={N} m={m} tile={tile} items={items} M={M} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_tuning(tile, items)
    x = np.concatenate([rand_points(M // 2, 80 + m),
                        workloads.wrap(-0.2 + 0.02 * np.random.default_rng(90 + m).standard_normal((M - M // 2, 3)))])
    r = np.random.default_rng(100 + m)
    f = r.standard_normal(M) + 1j * r.standard_normal(M)
    p.set_points(to_dev(x))
    p.stage_spread(to_dev(f, dtype))
    got = p.grid().cpu().numpy()
    ref = ns.spread(f, x, p.n, m, 2.0) / phi0(m, 2.0) ** 3
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.3g} rel-linf {li:.3g}")
    assert l2 < stage_tol(m, dtype), (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
def test_stage_spread_pileup_and_dynamic_range(nf, dtype):
    """1500 points inside one grid cell (every chunk adds up to 512
    contributions to the same LDS cells: the fixed-point headroom) with
    values spread over eight orders of magnitude (one chunk scale)."""
    m, M = 4, 1500
    N = (16, 16, 16)
    log(f"stage_spread pile-up N={N} m={m} M={M} {dtype}")
    p = make_plan(nf, N, m, dtype)
    r = np.random.default_rng(120)
    x = workloads.wrap(10.0 / 32 + 0.001 + r.random((M, 3)) / 64)   # inside cell 10 of the n = 32 grid
    f = (r.standard_normal(M) + 1j * r.standard_normal(M)) * 10.0 ** r.uniform(-8, 0, M)
    p.set_points(to_dev(x))
    p.stage_spread(to_dev(f, dtype))
    got = p.grid().cpu().numpy()
    ref = ns.spread(f, x, p.n, m, 2.0) / phi0(m, 2.0) ** 3
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.3g} rel-linf {li:.3g}")
    assert l2 < stage_tol(m, dtype), (l2, li)


# ---------------------------------------------------------- end to end ----

@pytest.mark.parametrize("dtype", DTYPES)
def test_smooth_uniform_case(nf, dtype):
    """N = 32^3 smooth coefficients, 1e4 uniform points, sigma 2, m 6 (FP64)
    and m 4 (FP32): every output against the direct sum."""
    m = 6 if dtype == "c128" else 4
    fh, x = workloads.smooth_uniform_case(32, 10_000)
    log(f"smooth_uniform N=32 M=1e4 m={m} {dtype}")
    p = make_plan(nf, fh.shape, m, dtype)
    p.set_points(to_dev(x))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    ref = oracle.ndft_trafo(fh, x)
    l2, li = rel(got, ref)
    log(f"  rel-l2 {l2:.3e} rel-linf {li:.3e} tol {tol(m, 2.0, dtype):.1e}")
    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("m", [1, 2, 4, 8, 10])
def test_error_vs_m(nf, m, dtype):
    """Error against the direct sum stays under the estimate for every m."""
    N = (16, 12, 20)
    fh = rand_coeffs(N, 10 + m)
    x = rand_points(700, 20 + m)
    log(f"error_vs_m N={N} m={m} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    ref = oracle.ndft_trafo(fh, x)
    err = np.max(np.abs(got - ref))
    bound = ns.pst_error_bound(m, 2.0) * np.sum(np.abs(fh))
    rounding = (1e-13 if dtype == "c128" else 3e-6) * np.sum(np.abs(fh))
    assert err <= bound + rounding, (err, bound)


@pytest.mark.parametrize("dtype", DTYPES)
def test_single_mode_closed_form(nf, dtype):
    """fhat = delta_{k*} gives exp(-2 pi i k*.x) at every corner of I_N."""
    N = (16, 8, 12)
    m = 8 if dtype == "c128" else 4
    x = rand_points(500, 30)
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    corners = [(a, b, c) for a in (-8, 7) for b in (-4, 3) for c in (-6, 5)] + [(0, 0, 0), (3, -1, 2)]
    for k in corners:
        log(f"single_mode k={k} {dtype}")
        fh = np.zeros(N, dtype=np.complex128)
        fh[k[0] + 8, k[1] + 4, k[2] + 6] = 1.0
        got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
        ref = np.exp(-2j * np.pi * (x @ np.asarray(k, float)))
        assert np.max(np.abs(got - ref)) <= tol(m, 2.0, dtype), k


@pytest.mark.parametrize("dtype", DTYPES)
def test_regular_grid_points(nf, dtype):
    """Points on x_n = n/N - 1/2: the sum is fftn((-1)^{sum k} fhat) (Sec. 2.1)."""
    N = (16, 16, 16)
    m = 8 if dtype == "c128" else 4
    fh = rand_coeffs(N, 31)
    g = [np.arange(n) / n - 0.5 for n in N]
    X = np.stack(np.meshgrid(*g, indexing="ij"), axis=-1).reshape(-1, 3)
    k0, k1, k2 = np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij")
    s = 1 - 2 * ((k0 + k1 + k2) & 1)
    ref = np.fft.fftn(np.fft.ifftshift(fh * s)).reshape(-1)
    log(f"regular_grid {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(X))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    l2, li = rel(got, ref)
    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
def test_folding_and_edges(nf, dtype):
    """Points at -1/2, just below +1/2, exactly +1/2 (= -1/2) and shifted by
    integers evaluate as their folded copies."""
    N = (8, 8, 8)
    m = 6 if dtype == "c128" else 4
    fh = rand_coeffs(N, 32)
    base = np.array([[-0.5, -0.5, -0.5], [0.5 - 1e-16, 0.25, -0.125], [0.0, 0.0, 0.0],
                     [0.3, -0.49999999, 0.4999999999]])
    shifted = base + np.array([[3.0, -7.0, 1.0], [-2.0, 0.0, 5.0], [1.0, 1.0, -1.0], [0.0, 2.0, -4.0]])
    halfplus = np.array([[0.5, 0.5, 0.5]])
    x = np.concatenate([base, shifted, halfplus])
    log(f"folding {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    ref = oracle.ndft_trafo(fh, x)
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= tol(m, 2.0, dtype)
    assert np.max(np.abs(got[:4] - got[4:8])) <= 10 * tol(m, 2.0, dtype) * np.max(np.abs(ref))
    assert abs(got[8] - got[0]) <= 10 * tol(m, 2.0, dtype) * np.max(np.abs(ref))


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,sigma", [((2, 2, 2), 2.0), ((4, 6, 2), 2.0), ((12, 8, 20), 1.5), ((10, 10, 10), 2.0),
                                     ((64, 4, 8), 2.0), ((14, 28, 6), 2.0), ((16, 32, 8), 1.75)])
def test_shapes_and_sigma(nf, N, sigma, dtype):
    """Small, non-cubic, radix-3/5/7 and sigma = 1.5 / 1.75 grids."""
    m = min(4, min(int(sigma * n) for n in N) // 2)
    fh = rand_coeffs(N, 33)
    x = rand_points(333, 34)
    log(f"shapes N={N} sigma={sigma} m={m} {dtype}")
    p = make_plan(nf, N, m, dtype, sigma)
    p.set_points(to_dev(x))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    ref = oracle.ndft_trafo(fh, x)
    err = np.max(np.abs(got - ref))
    bound = ns.pst_error_bound(m, sigma) * np.sum(np.abs(fh))
    assert err <= bound + (1e-13 if dtype == "c128" else 3e-6) * np.sum(np.abs(fh)), (err, bound)


def test_empty_points_and_errors(nf):
    import torch
    N = (8, 8, 8)
    p = make_plan(nf, N, 4, "c128")
    fh = to_dev(rand_coeffs(N, 35), "c128")
    log("errors: no points")
    with pytest.raises(nf.NFFT3Error) as e:
        p.trafo(fh, out=torch.empty(0, dtype=torch.complex128, device="cuda:0"))
    assert e.value.code == -4
    p.set_points(torch.zeros((0, 3), dtype=torch.float64, device="cuda:0"))
    out = p.trafo(fh)
    assert out.numel() == 0
    adj = p.adjoint(torch.zeros(0, dtype=torch.complex128, device="cuda:0"))
    assert torch.count_nonzero(adj).item() == 0
    log("errors: non-finite")
    bad = torch.tensor([[0.1, float("nan"), 0.2], [0.0, 0.0, 0.0]], dtype=torch.float64, device="cuda:0")
    with pytest.raises(nf.NFFT3Error) as e:
        p.set_points(bad)
    assert e.value.code == -5
    with pytest.raises(nf.NFFT3Error) as e:
        p.trafo(fh, out=torch.empty(0, dtype=torch.complex128, device="cuda:0"))
    assert e.value.code == -4
    bad = torch.tensor([[0.1, float("inf"), 0.2]], dtype=torch.float64, device="cuda:0")
    with pytest.raises(nf.NFFT3Error):
        p.set_points(bad)


# ------------------------------------------------------------- adjoint ----

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [(16, 12, 20), (32, 64, 128), (96, 48, 32), (40, 160, 80)])
def test_adjoint_dot_product_and_direct_sum(nf, N, dtype):
    m = 8 if dtype == "c128" else 4
    fh = rand_coeffs(N, 40)
    x = rand_points(2000, 41)
    r = np.random.default_rng(42)
    y = r.standard_normal(2000) + 1j * r.standard_normal(2000)
    log(f"adjoint N={N} m={m} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    Af = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    Ahy = p.adjoint(to_dev(y, dtype)).cpu().numpy()
    lhs = np.vdot(y, Af)
    rhs = np.vdot(Ahy, fh)
    assert abs(lhs - rhs) / abs(lhs) < dot_tol(dtype)
    ref = oracle.ndft_adjoint(y, x, N)
    l2, li = rel(Ahy, ref)
    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (l2, li)


@pytest.mark.parametrize("dtype,scales", [("c128", (1e-60, 1e-300, 1e300)), ("c64", (1e-30, 1e30))])
def test_adjoint_extreme_values_and_nan(nf, dtype, scales):
    """The adjoint's fixed-point accumulation takes its scale from each
    chunk's largest value in f's own precision: values far from 1 (down to
    1e-300, up to 1e300 in FP64) keep their relative accuracy against the
    scaled direct adjoint; a NaN or infinite value makes the result NaN."""
    import torch
    N = (8, 10, 12)
    m = 8 if dtype == "c128" else 4
    x = rand_points(900, 43)
    r = np.random.default_rng(44)
    y = r.standard_normal(900) + 1j * r.standard_normal(900)
    ref = oracle.ndft_adjoint(y, x, N)
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    for sc in scales:
        log(f"adjoint scale {sc:g} {dtype}")
        got = p.adjoint(to_dev(y * sc, dtype)).cpu().numpy().astype(np.complex128) / sc
        l2, li = rel(got, ref)
        assert np.all(np.isfinite(got)) and l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (sc, l2, li)
    for bad in (float("nan"), float("inf")):
        yb = y.copy()
        yb[123] = bad
        got = p.adjoint(to_dev(yb, dtype)).cpu().numpy()
        assert np.all(np.isnan(got)), bad
    # a finite call afterwards is unaffected
    got = p.adjoint(to_dev(y, dtype)).cpu().numpy()
    assert rel(got, ref)[0] <= tol(m, 2.0, dtype)
    torch.cuda.synchronize()


# ---------------------------------------------------------------- grad ----

@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("tile,items", [(32, 512), (8, 256), (24, 512)])
def test_grad_points_vs_direct_derivative(nf, dtype, tile, items):
    """Point gradient (the window-sum body in its derivative mode, 256 points
    of an item at a time) against the oracle's derivative sums, at several
    binning settings."""
    N = (16, 16, 12)
    m = 8 if dtype == "c128" else 4
    fh = rand_coeffs(N, 50)
    x = rand_points(1500, 51)
    r = np.random.default_rng(52)
    G = r.standard_normal(1500) + 1j * r.standard_normal(1500)
    log(f"grad N={N} m={m} tile={tile} items={items} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_tuning(tile, items)
    p.set_points(to_dev(x))
    got = p.grad_points(to_dev(fh, dtype), to_dev(G, dtype)).cpu().numpy()
    D = oracle.ndft_grad(fh, x)
    ref = (np.conj(G)[:, None] * D).real
    l2, li = rel(got, ref)
    gate = 10 * tol(m, 2.0, dtype)
    assert l2 <= gate and li <= gate, (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
def test_derivative_fields(nf, dtype):
    """trafo_fields: the field and the three fields of -2 pi i k_d fhat."""
    N = (12, 16, 8)
    m = 8 if dtype == "c128" else 4
    fh = rand_coeffs(N, 60)
    x = rand_points(800, 61)
    log(f"fields N={N} m={m} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    out = p.trafo_fields(to_dev(fh, dtype), 7).cpu().numpy()
    ref0 = oracle.ndft_trafo(fh, x)
    D = oracle.ndft_grad(fh, x)
    for i, ref in enumerate([ref0, D[:, 0], D[:, 1], D[:, 2]]):
        l2, li = rel(out[i], ref)
        assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (i, l2, li)
    out5 = p.trafo_fields(to_dev(fh, dtype), 5).cpu().numpy()
    assert out5.shape[0] == 3
    assert np.allclose(out5[1], out[1]) and np.allclose(out5[2], out[3])


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [(32, 32, 32), (64, 8, 8), (48, 16, 16)])
def test_full_item_segments(nf, N, dtype):
    """Grids whose z-axis fills whole 64-cell segments of the work-item walk
    (n0 = 64, 128) and one that leaves a partial segment (n0 = 96): every
    cell's count comes from its neighbour's start, up to the segment's last."""
    m = 8 if dtype == "c128" else 4
    fh = rand_coeffs(N, 140)
    x = np.concatenate([rand_points(1500, 141),
                        workloads.wrap(0.1 + 0.01 * np.random.default_rng(142).standard_normal((1500, 3)))])
    log(f"full item segments N={N} {dtype}")
    p = make_plan(nf, N, m, dtype)
    p.set_points(to_dev(x))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    l2, li = rel(got, oracle.ndft_trafo(fh, x))
    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (l2, li)
