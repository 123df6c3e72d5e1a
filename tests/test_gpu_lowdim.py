"""One- and two-dimensional plans (Appendix B: infft, infft2, igridft2, the
E psihat product): the 3-D kernels with leading unit axes, against the
oracle's per-axis phase products."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_common import dot_tol, log, rand_coeffs, rel, to_dev, tol, torch_dtype

pytestmark = pytest.mark.gpu

DTYPES = ["c128", "c64"]
M_OF = {"c128": 8, "c64": 4}


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available()
    import paper_1605_01244_amd as mod
    return mod


def pts(M, d, seed, lo=-0.5, hi=0.5):
    return np.random.default_rng(seed).uniform(lo, hi, size=(int(M), d))


def plan(nf, N, dtype, m=None):
    return nf.Plan(N, m=M_OF[dtype] if m is None else m, dtype=torch_dtype(dtype), device="cuda:0")


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,M", [((16,), 300), ((64,), 2000), ((1024,), 7001), ((16, 16), 500),
                                 ((64, 48), 3001), ((256, 256), 20000), ((8, 1024), 999)])
def test_trafo_lowdim(nf, N, M, dtype):
    """Sizes from one tile to many, ragged M, points also outside the unit box."""
    fh = rand_coeffs(N, 1)
    x = pts(M, len(N), 2, -2.0, 2.0)
    log(f"lowdim trafo N={N} M={M} {dtype}")
    p = plan(nf, N, dtype)
    p.set_points(to_dev(x))
    got = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    ref = oracle.ndft_lowdim(fh, x)
    l2, li = rel(got, ref)
    g = tol(M_OF[dtype], 2.0, dtype)
    assert l2 <= g and li <= g, (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
def test_paper_1d_case(nf, dtype):
    """The one-dimensional size the paper tabulates its accuracy on (N = 64,
    M = 2000), at m = 4, 6, 8 (FP64)."""
    fh = rand_coeffs((64,), 3)
    x = pts(2000, 1, 4)
    ref = oracle.ndft_lowdim(fh, x)
    for m in ([4, 6, 8] if dtype == "c128" else [4]):
        p = plan(nf, (64,), dtype, m)
        p.set_points(to_dev(x))
        l2, li = rel(p.trafo(to_dev(fh, dtype)).cpu().numpy(), ref)
        log(f"1-D N=64 M=2000 m={m} {dtype}: rel-l2 {l2:.2e}")
        assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (m, l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [(32,), (24, 40)])
def test_adjoint_lowdim(nf, N, dtype):
    M = 1500
    x = pts(M, len(N), 5)
    r = np.random.default_rng(6)
    f = r.standard_normal(M) + 1j * r.standard_normal(M)
    fh = rand_coeffs(N, 7)
    log(f"lowdim adjoint N={N} {dtype}")
    p = plan(nf, N, dtype)
    p.set_points(to_dev(x))
    got = p.adjoint(to_dev(f, dtype)).cpu().numpy()
    assert got.shape == N
    ref = oracle.ndft_lowdim_adjoint(f, x, N)
    l2, li = rel(got, ref)
    g = tol(M_OF[dtype], 2.0, dtype)
    assert l2 <= g and li <= g, (l2, li)
    # the pair is the exact transpose of one discrete operator
    Af = p.trafo(to_dev(fh, dtype)).cpu().numpy()
    lhs, rhs = np.vdot(f, Af), np.vdot(got, fh)
    assert abs(lhs - rhs) <= dot_tol(dtype) * abs(lhs), (lhs, rhs)


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N", [(48,), (16, 24)])
def test_grad_points_lowdim(nf, N, dtype):
    M = 1200
    fh = rand_coeffs(N, 8)
    x = pts(M, len(N), 9)
    r = np.random.default_rng(10)
    G = r.standard_normal(M) + 1j * r.standard_normal(M)
    log(f"lowdim grad N={N} {dtype}")
    p = plan(nf, N, dtype)
    p.set_points(to_dev(x))
    got = p.grad_points(to_dev(fh, dtype), to_dev(G, dtype)).cpu().numpy()
    assert got.shape == (M, len(N))
    ref = (np.conj(G)[:, None] * oracle.ndft_lowdim_grad(fh, x)).real
    l2, li = rel(got, ref)
    g = 10 * tol(M_OF[dtype], 2.0, dtype)
    assert l2 <= g and li <= g, (l2, li)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fields_lowdim(nf, dtype):
    """trafo_fields on a 2-D plan: mask bit d = the plan's axis d."""
    N = (20, 12)
    fh = rand_coeffs(N, 11)
    x = pts(900, 2, 12)
    p = plan(nf, N, dtype)
    p.set_points(to_dev(x))
    D = oracle.ndft_lowdim_grad(fh, x)
    g = 10 * tol(M_OF[dtype], 2.0, dtype)
    for mask in (1, 2, 3):
        out = p.trafo_fields(to_dev(fh, dtype), mask).cpu().numpy()
        refs = [oracle.ndft_lowdim(fh, x)] + [D[:, d] for d in range(2) if mask >> d & 1]
        assert out.shape == (len(refs), 900)
        for o, r in zip(out, refs):
            l2, li = rel(o, r)
            assert l2 <= g and li <= g, (mask, l2, li)
    with pytest.raises(nf.NFFT3Error):
        p.trafo_fields(to_dev(fh, dtype), 4)         # no third axis


@pytest.mark.parametrize("dtype", DTYPES)
def test_infft_and_infft2(nf, dtype):
    """The paper's infft / infft2 on physical domains, points inside and far outside."""
    m = M_OF[dtype]
    g = tol(m, 2.0, dtype)
    ph = rand_coeffs((40,), 13)
    xi = np.concatenate([np.random.default_rng(14).uniform(-2.0, 3.0, 700), [-2.0, 3.0, 47.25]])
    got = nf.infft(to_dev(ph, dtype), -2.0, 3.0, to_dev(xi), m=m).cpu().numpy()
    l2, li = rel(got, oracle.infft_lowdim(ph, [-2.0], [3.0], xi[:, None]))
    assert l2 <= g and li <= g, (l2, li)
    a, b = np.array([-1.0, 0.5]), np.array([4.0, 2.0])
    ph2 = rand_coeffs((24, 18), 15)
    xi2 = np.random.default_rng(16).uniform(a - 5, b + 5, size=(900, 2))
    got = nf.infft2(to_dev(ph2, dtype), a, b, to_dev(xi2), m=m).cpu().numpy()
    l2, li = rel(got, oracle.infft_lowdim(ph2, a, b, xi2))
    assert l2 <= g and li <= g, (l2, li)


EPS = {"c128": np.finfo(np.float64).eps, "c64": np.finfo(np.float32).eps}


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("N,M", [((64,), (64,)), ((30,), (1,)), ((64, 64), (64, 64)), ((6, 130), (70, 3)),
                                 ((256, 128), (321, 100))])
def test_rectgrid_lowdim(nf, N, M, dtype):
    """igridft2's double product and the 1-D E psihat product on the matrix cores."""
    import torch
    fh = rand_coeffs(N, 17)
    r = np.random.default_rng(18)
    ys = [r.uniform(-0.5, 0.5, size=m) for m in M]
    log(f"lowdim rgrid N={N} M={M} {dtype}")
    g = nf.RectGrid(N, M, dtype=torch_dtype(dtype), device="cuda:0")
    g.set_axes(*[torch.from_numpy(y).to("cuda:0") for y in ys])
    got = g.eval(to_dev(fh, dtype)).cpu().numpy()
    assert got.shape == M
    ref = oracle.rgrid_lowdim(fh, *ys)
    l2, li = rel(got, ref)
    gate = max(4.0 * sum(N) * EPS[dtype], 1e-13)
    assert l2 <= gate and li <= gate, (l2, li)


def test_three_axis_plan_with_unit_axis(nf):
    """nfft3_plan with N_0 = 1 and (M, 3) points: the unit coordinate is ignored."""
    import torch
    from paper_1605_01244_amd._lib import check, lib
    N = (1, 32, 20)
    fh = rand_coeffs(N, 19)
    x = pts(1000, 3, 20, -3.0, 3.0)
    h = ctypes.c_void_p()
    s = torch.cuda.current_stream().cuda_stream
    check(lib.nfft3_plan(ctypes.byref(h), (ctypes.c_int64 * 3)(*N), 2.0, 8, 1, ctypes.c_void_p(s)), "plan")
    try:
        xd = to_dev(x)
        fd = to_dev(fh, "c128")
        out = torch.empty(1000, dtype=torch.complex128, device="cuda:0")
        check(lib.nfft3_set_points(h, 1000, ctypes.c_void_p(xd.data_ptr())), "set_points")
        check(lib.nfft3_trafo(h, ctypes.c_void_p(fd.data_ptr()), ctypes.c_void_p(out.data_ptr())), "trafo")
        l2, li = rel(out.cpu().numpy(), oracle.ndft_lowdim(fh[0], x[:, 1:]))
        assert l2 <= tol(8, 2.0, "c128") and li <= tol(8, 2.0, "c128"), (l2, li)
    finally:
        lib.nfft3_destroy(h)


def test_lowdim_edge_cases(nf):
    import torch
    p = plan(nf, (32, 16), "c128")
    # no points: trafo writes nothing, adjoint gives zeros
    p.set_points(torch.empty((0, 2), dtype=torch.float64, device="cuda:0"))
    assert p.trafo(to_dev(rand_coeffs((32, 16), 21), "c128")).numel() == 0
    z = p.adjoint(torch.empty(0, dtype=torch.complex128, device="cuda:0")).cpu().numpy()
    assert np.all(z == 0)
    # a NaN coordinate is reported
    x = pts(10, 2, 22)
    x[3, 1] = np.nan
    with pytest.raises(nf.NFFT3Error):
        p.set_points(to_dev(x))
    # wrong point width
    with pytest.raises(ValueError):
        p.set_points(to_dev(pts(10, 3, 23)))
    # unchanged points are recognised; a changed coordinate is not
    x = pts(500, 2, 24)
    xd = to_dev(x)
    assert p.set_points_if_changed(xd) is True
    assert p.set_points_if_changed(xd) is False
    xd[7, 0] += 0.25
    assert p.set_points_if_changed(xd) is True
    # three-dimensional plans only: batch and tube refinement
    p.set_points(to_dev(x))
    with pytest.raises(nf.NFFT3Error):
        nf.batch_trafo([p], [to_dev(rand_coeffs((32, 16), 25), "c128")])
    with pytest.raises(nf.NFFT3Error):
        p.tube_refine(to_dev(rand_coeffs((32, 16), 25), "c128"), [0, 0], [1, 1], [0.1])


def test_autograd_lowdim(nf):
    """type2 on a 2-D plan: gradients in the coefficients and the points."""
    import torch
    N = (16, 12)
    fh = rand_coeffs(N, 26)
    x = pts(400, 2, 27)
    w = np.random.default_rng(28).standard_normal(400) + 1j * np.random.default_rng(29).standard_normal(400)
    p = plan(nf, N, "c128")
    fd = to_dev(fh, "c128").requires_grad_(True)
    xd = to_dev(x).requires_grad_(True)
    f = nf.type2(fd, xd, p)
    L = (torch.conj(to_dev(w, "c128")) * f).real.sum()
    L.backward()
    # dL/dRe fhat + i dL/dIm fhat = A^H w; dL/dx = Re(conj(w) df/dx)
    gf = oracle.ndft_lowdim_adjoint(w, x, N)
    gx = (np.conj(w)[:, None] * oracle.ndft_lowdim_grad(fh, x)).real
    l2, _ = rel(fd.grad.cpu().numpy(), gf)
    assert l2 <= tol(8, 2.0, "c128"), l2
    l2, _ = rel(xd.grad.cpu().numpy(), gx)
    assert l2 <= 10 * tol(8, 2.0, "c128"), l2
