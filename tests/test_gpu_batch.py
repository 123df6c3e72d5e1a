"""Batched evaluation (per stage one launch per transform length over all plans and fields):
uneven N, own point sets, derivative fields; against sequential single-plan
calls and the oracle."""
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


def _sets(spec, seed):
    out = []
    for i, (N, M) in enumerate(spec):
        out.append((N, rand_coeffs(N, seed + i), rand_points(M, seed + 100 + i)))
    return out


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("mask", [0, 7, 5])
def test_batch_matches_sequential_and_oracle(nf, dtype, mask):
    m = 8 if dtype == "c128" else 4
    spec = [((8, 8, 8), 300), ((12, 16, 10), 1000), ((16, 16, 16), 1), ((8, 10, 12), 2500), ((16, 12, 8), 700)]
    sets = _sets(spec, 10)
    log(f"batch {dtype} mask={mask} T={len(sets)}")
    plans, fh = [], []
    for N, f, x in sets:
        p = nf.Plan(N, sigma=2.0, m=m, dtype=torch_dtype(dtype), device="cuda:0")
        p.set_points(to_dev(x))
        plans.append(p)
        fh.append(to_dev(f, dtype))
    outs = nf.batch_trafo(plans, fh, mask)
    fields = [-1] + [d for d in range(3) if mask & (1 << d)]
    for t, (N, f, x) in enumerate(sets):
        got = outs[t].cpu().numpy()
        seq = plans[t].trafo_fields(fh[t], mask).cpu().numpy()
        assert np.array_equal(got, seq), t       # same kernels, same arithmetic
        ref0 = oracle.ndft_trafo(f, x)
        D = oracle.ndft_grad(f, x) if mask else None
        for i, fl in enumerate(fields):
            ref = ref0 if fl < 0 else D[:, fl]
            l2, li = rel(got[i], ref)
            assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (t, fl, l2, li)


def test_batch_mixed_radices(nf):
    """N = 64/96/128 style mix at small scale: 16, 24, 32 (n = 32, 48, 64)."""
    spec = [((16, 16, 16), 2000), ((24, 24, 24), 1500), ((32, 32, 32), 1800), ((24, 24, 24), 10)]
    sets = _sets(spec, 50)
    log("batch mixed radices")
    plans, fh = [], []
    for N, f, x in sets:
        p = nf.Plan(N, sigma=2.0, m=4, dtype=torch_dtype("c64"), device="cuda:0")
        p.set_points(to_dev(x))
        plans.append(p)
        fh.append(to_dev(f, "c64"))
    outs = nf.batch_trafo(plans, fh, 7)
    for t, (N, f, x) in enumerate(sets):
        assert np.array_equal(outs[t].cpu().numpy(), plans[t].trafo_fields(fh[t], 7).cpu().numpy())
        l2, li = rel(outs[t][0].cpu().numpy(), oracle.ndft_trafo(f, x))
        assert l2 <= tol(4, 2.0, "c64") and li <= tol(4, 2.0, "c64")


def test_batch_plans_with_different_tiles(nf):
    """Plans of one batch may use different tiles (same points per item):
    each transform keeps its own geometry."""
    spec = [((16, 16, 16), 2500), ((24, 24, 24), 1500), ((32, 32, 32), 3000)]
    sets = _sets(spec, 70)
    log("batch with per-plan tiles 8 / 20 / 32")
    plans, fh = [], []
    for (N, f, x), tile in zip(sets, (8, 20, 32)):
        p = nf.Plan(N, sigma=2.0, m=8, dtype=torch_dtype("c128"), device="cuda:0")
        p.set_tuning(tile, 512)
        p.set_points(to_dev(x))
        plans.append(p)
        fh.append(to_dev(f, "c128"))
    outs = nf.batch_trafo(plans, fh, 5)
    for t, (N, f, x) in enumerate(sets):
        assert plans[t].tuning()[0] == (8, 20, 32)[t]
        assert np.array_equal(outs[t].cpu().numpy(), plans[t].trafo_fields(fh[t], 5).cpu().numpy())
        l2, li = rel(outs[t][0].cpu().numpy(), oracle.ndft_trafo(f, x))
        assert l2 <= tol(8, 2.0, "c128") and li <= tol(8, 2.0, "c128")


def test_batch_argument_errors(nf):
    import torch
    p1 = nf.Plan((8, 8, 8), m=4, dtype=torch.complex128, device="cuda:0")
    p2 = nf.Plan((8, 8, 8), m=5, dtype=torch.complex128, device="cuda:0")
    p3 = nf.Plan((8, 8, 8), m=4, dtype=torch.complex64, device="cuda:0")
    f64 = to_dev(rand_coeffs((8, 8, 8), 1), "c128")
    f32 = to_dev(rand_coeffs((8, 8, 8), 1), "c64")
    x = to_dev(rand_points(10, 2))
    for p in (p1, p2, p3):
        p.set_points(x)
    with pytest.raises(nf.NFFT3Error) as e:
        nf.batch_trafo([p1, p2], [f64, f64])
    assert e.value.code == -1          # different m
    with pytest.raises(nf.NFFT3Error) as e:
        nf.batch_trafo([p1, p1], [f64, f64])
    assert e.value.code == -1          # same plan twice
    with pytest.raises((nf.NFFT3Error, TypeError)):
        nf.batch_trafo([p1, p3], [f64, f32])
    p4 = nf.Plan((8, 8, 8), m=4, dtype=torch.complex128, device="cuda:0")
    with pytest.raises(nf.NFFT3Error) as e:
        nf.batch_trafo([p1, p4], [f64, f64])
    assert e.value.code == -4          # no points on p4
