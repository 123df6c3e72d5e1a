"""Differentiation: torch.autograd through the HIP type-2 transform.

grad wrt coefficients = adjoint (type-1) spreading; grad wrt points = window
derivative.  Checked with torch.autograd.gradcheck (finite differences of the
GPU forward), against the oracle's direct adjoint and derivative sums, and
with central differences of the oracle."""
import numpy as np
import pytest

import oracle
from gpu_common import log, rand_coeffs, rand_points, rel, to_dev, tol, torch_dtype

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nf():
    import torch
    assert torch.cuda.is_available()
    import paper_1605_01244_amd as mod
    return mod


def test_gradcheck_small(nf):
    """gradcheck at N = 8^3, M = 20, FP64, m = 8 (f64 inputs require grad)."""
    import torch
    N = (8, 8, 8)
    plan = nf.Plan(N, m=8, dtype=torch.complex128, device="cuda:0")
    fh = to_dev(rand_coeffs(N, 1), "c128").requires_grad_(True)
    x = to_dev(rand_points(20, 2) * 0.9).requires_grad_(True)
    log("gradcheck")
    assert torch.autograd.gradcheck(lambda a, b: nf.type2(a, b, plan), (fh, x), eps=1e-6, atol=1e-7, rtol=1e-5)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_gradients_vs_oracle(nf, dtype):
    """L = sum_j Re(conj(w_j) f_j): dL/dfhat = A^H w, dL/dx_{j,d} = Re(conj(w_j) df_j/dx_{j,d})."""
    import torch
    m = 8 if dtype == "c128" else 4
    N = (16, 12, 20)
    M = 1000
    fh_np = rand_coeffs(N, 3)
    x_np = rand_points(M, 4)
    r = np.random.default_rng(5)
    w_np = (r.standard_normal(M) + 1j * r.standard_normal(M)) / np.sqrt(2)
    plan = nf.Plan(N, m=m, dtype=torch_dtype(dtype), device="cuda:0")
    fh = to_dev(fh_np, dtype).requires_grad_(True)
    x = to_dev(x_np).requires_grad_(True)
    w = to_dev(w_np, dtype)
    log(f"autograd {dtype}")
    f = nf.type2(fh, x, plan)
    L = (torch.conj(w) * f).real.sum()
    L.backward()
    g_f = fh.grad.cpu().numpy()
    g_x = x.grad.cpu().numpy()
    # torch's convention: grad of a real L wrt complex fhat is dL/dRe + i dL/dIm = A^H w
    ref_f = oracle.ndft_adjoint(w_np, x_np, N)
    l2, li = rel(g_f, ref_f)
    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (l2, li)
    D = oracle.ndft_grad(fh_np, x_np)
    ref_x = (np.conj(w_np)[:, None] * D).real
    l2, li = rel(g_x, ref_x)
    assert l2 <= 10 * tol(m, 2.0, dtype) and li <= 10 * tol(m, 2.0, dtype), (l2, li)


def test_point_gradient_vs_central_differences_of_oracle(nf):
    """30 (j, d) entries of dL/dx against central differences (h = 1e-6) of the
    oracle's L."""
    import torch
    N = (12, 12, 12)
    M = 200
    fh_np = rand_coeffs(N, 6)
    x_np = rand_points(M, 7)
    r = np.random.default_rng(8)
    w_np = r.standard_normal(M) + 1j * r.standard_normal(M)
    plan = nf.Plan(N, m=8, dtype=torch.complex128, device="cuda:0")
    x = to_dev(x_np).requires_grad_(True)
    f = nf.type2(to_dev(fh_np, "c128"), x, plan)
    (torch.conj(to_dev(w_np, "c128")) * f).real.sum().backward()
    g = x.grad.cpu().numpy()
    pick = np.random.default_rng(9).choice(M * 3, size=30, replace=False)
    h = 1e-6
    for q in pick:
        j, d = divmod(int(q), 3)
        xp, xm = x_np[j:j + 1].copy(), x_np[j:j + 1].copy()
        xp[0, d] += h
        xm[0, d] -= h
        Lp = (np.conj(w_np[j]) * oracle.ndft_trafo(fh_np, xp)[0]).real
        Lm = (np.conj(w_np[j]) * oracle.ndft_trafo(fh_np, xm)[0]).real
        fd = (Lp - Lm) / (2 * h)
        assert abs(fd - g[j, d]) <= 1e-6 * max(1.0, abs(fd)), (j, d, fd, g[j, d])


def test_backward_after_points_replaced(nf):
    """The plan's points are reset to the forward's points if they changed."""
    import torch
    N = (8, 8, 8)
    plan = nf.Plan(N, m=6, dtype=torch.complex128, device="cuda:0")
    fh = to_dev(rand_coeffs(N, 10), "c128").requires_grad_(True)
    x1 = to_dev(rand_points(50, 11))
    f = nf.type2(fh, x1, plan)
    plan.set_points(to_dev(rand_points(70, 12)))     # another user of the plan
    G = to_dev(rand_coeffs((50,), 13), "c128")
    f.backward(G)
    ref = oracle.ndft_adjoint(G.cpu().numpy(), x1.cpu().numpy(), N)
    l2, _ = rel(fh.grad.cpu().numpy(), ref)
    assert l2 <= tol(6, 2.0, "c128")


def test_forward_resorts_only_changed_points(nf):
    """The autograd forward skips the sort only when every folded coordinate
    still equals the plan's sorted copy: an unchanged tensor, or one shifted
    by whole periods (same folded values), is not re-sorted; a write through
    .data (which bypasses the version counter) and a different M are."""
    import torch
    N = (10, 8, 12)
    plan = nf.Plan(N, m=6, dtype=torch.complex128, device="cuda:0")
    fh_np = rand_coeffs(N, 20)
    fh = to_dev(fh_np, "c128")
    # multiples of 2^-20, so x + 2 is exact and folds back to x bit for bit
    x_np = np.round(rand_points(300, 21) * 2.0**20) / 2.0**20
    x = to_dev(x_np)
    log("points cache")
    assert plan.set_points_if_changed(x) is True
    assert plan.set_points_if_changed(x) is False
    assert plan.set_points_if_changed(x.clone()) is False
    assert plan.set_points_if_changed(x + 2.0) is False      # folds to the same coordinates
    x.data[17, 1] += 1e-3                                      # not seen by the version counter
    f = nf.type2(fh, x, plan).cpu().numpy()
    ref = oracle.ndft_trafo(fh_np, x.cpu().numpy())
    l2, li = rel(f, ref)
    assert l2 <= tol(6, 2.0, "c128") and li <= tol(6, 2.0, "c128"), (l2, li)
    assert plan.set_points_if_changed(x[:200]) is True
    assert plan.M == 200
    ab = torch.tensor([[0.1, float("nan"), 0.2]], dtype=torch.float64, device="cuda:0")
    with pytest.raises(nf.NFFT3Error):
        plan.set_points_if_changed(ab)
