"""The batch as one work-queue launch (nfft3_batch_trafo_queue): bit-equal to
the per-length launches (same stage bodies), checked against the oracle, with
uneven lengths per axis, empty point sets, repeated calls and the bounded
wait's abort path (forced from the host through the wait limit)."""
import os

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


def _plans(nf, spec, dtype, m, seed):
    sets, plans, fh = [], [], []
    for i, (N, M) in enumerate(spec):
        f, x = rand_coeffs(N, seed + i), rand_points(M, seed + 100 + i)
        p = nf.Plan(N, sigma=2.0, m=m, dtype=torch_dtype(dtype), device="cuda:0")
        p.set_points(to_dev(x))
        sets.append((N, f, x))
        plans.append(p)
        fh.append(to_dev(f, dtype))
    return sets, plans, fh


# oversampled lengths 64 / 80 / 96 / 128 (the compile-time engine's), uneven per axis
SPEC = [((32, 32, 32), 3000), ((48, 40, 32), 1200), ((64, 48, 40), 5000), ((40, 64, 48), 1),
        ((32, 48, 64), 2500), ((48, 48, 48), 0)]


@pytest.mark.parametrize("dtype", ["c64", "c128"])
@pytest.mark.parametrize("mask", [0, 7, 2])
def test_queue_equals_launches_and_oracle(nf, dtype, mask):
    m = 4 if dtype == "c64" else 8
    sets, plans, fh = _plans(nf, SPEC, dtype, m, 300)
    log(f"queue {dtype} mask={mask} T={len(plans)}")
    ref_outs = nf.batch_trafo(plans, fh, mask)
    outs = nf.batch_trafo(plans, fh, mask, queue=True)
    fields = [-1] + [d for d in range(3) if mask & (1 << d)]
    for t, (N, f, x) in enumerate(sets):
        got = outs[t].cpu().numpy()
        assert np.array_equal(got, ref_outs[t].cpu().numpy()), t
        if x.shape[0] == 0:
            continue
        ref0 = oracle.ndft_trafo(f, x)
        D = oracle.ndft_grad(f, x) if mask else None
        for i, fl in enumerate(fields):
            ref = ref0 if fl < 0 else D[:, fl]
            l2, li = rel(got[i], ref)
            assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (t, fl, l2, li)


def test_queue_many_transforms_repeated(nf):
    """A larger mix (128 transforms) three times in a row: every call clears
    its counters, and each equals the per-length form bit for bit."""
    rng = np.random.default_rng(5)
    lens = [32, 40, 48, 64]
    spec = [(tuple(int(v) for v in rng.choice(lens, 3)), int(rng.integers(500, 20000))) for _ in range(32)]
    sets, plans, fh = _plans(nf, spec, "c64", 4, 700)
    log("queue 32 plans x 4 fields, three calls")
    ref = [o.cpu().numpy() for o in nf.batch_trafo(plans, fh, 7)]
    for rep in range(3):
        outs = nf.batch_trafo(plans, fh, 7, queue=True)
        for t in range(len(plans)):
            assert np.array_equal(outs[t].cpu().numpy(), ref[t]), (rep, t)


@pytest.mark.parametrize("dtype,m,pts", [("c64", 4, 256), ("c128", 8, 512), ("c64", 2, 512), ("c128", 5, 256)])
def test_queue_tunings_and_window_widths(nf, dtype, m, pts):
    """Per-plan tiles (8 / 20 / 32 cells) and both item sizes (256 points:
    one per thread; 512: two), at several m: the queue equals the per-length
    launches bit for bit and meets the oracle gate."""
    spec = [((32, 32, 32), 2500), ((40, 48, 32), 1500), ((64, 40, 48), 3000)]
    sets, plans, fh = [], [], []
    for i, ((N, M), tile) in enumerate(zip(spec, (8, 20, 32))):
        f, x = rand_coeffs(N, 1100 + i), rand_points(M, 1200 + i)
        p = nf.Plan(N, sigma=2.0, m=m, dtype=torch_dtype(dtype), device="cuda:0")
        p.set_tuning(tile, pts)
        p.set_points(to_dev(x))
        sets.append((N, f, x))
        plans.append(p)
        fh.append(to_dev(f, dtype))
    log(f"queue {dtype} m={m} items of {pts} points, tiles 8 / 20 / 32")
    ref = nf.batch_trafo(plans, fh, 5)
    outs = nf.batch_trafo(plans, fh, 5, queue=True)
    for t, (N, f, x) in enumerate(sets):
        got = outs[t].cpu().numpy()
        assert np.array_equal(got, ref[t].cpu().numpy()), t
        l2, li = rel(got[0], oracle.ndft_trafo(f, x))
        assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (t, l2, li)


def test_queue_wait_limit_abort_then_recovers(nf):
    """With a zero wait limit any task that finds its previous stage still
    running abandons the batch: the call returns NFFT3_ERR_TIMEOUT (or, if no
    task ever had to wait, completes).  Every workgroup still exits, and the
    next call with the default limit is exact."""
    sets, plans, fh = _plans(nf, SPEC[:3], "c64", 4, 900)
    ref = [o.cpu().numpy() for o in nf.batch_trafo(plans, fh, 7)]
    log("queue with NFFT3_QUEUE_WAIT_US=0")
    os.environ["NFFT3_QUEUE_WAIT_US"] = "0"
    try:
        try:
            outs = nf.batch_trafo(plans, fh, 7, queue=True)
            completed = True
        except RuntimeError as e:
            assert "NFFT3_ERR_TIMEOUT" in str(e), e
            completed = False
    finally:
        del os.environ["NFFT3_QUEUE_WAIT_US"]
    log(f"zero limit: {'completed' if completed else 'abandoned'}")
    if completed:
        for t in range(len(plans)):
            assert np.array_equal(outs[t].cpu().numpy(), ref[t])
    outs = nf.batch_trafo(plans, fh, 7, queue=True)
    for t in range(len(plans)):
        assert np.array_equal(outs[t].cpu().numpy(), ref[t]), t


def test_queue_argument_errors(nf):
    """Lengths outside the compile-time engine (n = 72 here) are refused
    before any work, as are the per-length form's own argument errors."""
    import torch
    log("queue argument errors")
    p = nf.Plan((36, 32, 32), sigma=2.0, m=4, dtype=torch.complex64, device="cuda:0")
    p.set_points(to_dev(rand_points(100, 3)))
    f = to_dev(rand_coeffs((36, 32, 32), 4), "c64")
    with pytest.raises(RuntimeError, match="INVALID_ARG"):
        nf.batch_trafo([p], [f], 0, queue=True)
    with pytest.raises(ValueError):
        nf.batch_trafo([p], [f], 0, allocate=False, queue=True)
    q = nf.Plan((32, 32, 32), sigma=2.0, m=4, dtype=torch.complex64, device="cuda:0")
    q.set_points(to_dev(rand_points(100, 5)))
    g = to_dev(rand_coeffs((32, 32, 32), 6), "c64")
    with pytest.raises(RuntimeError, match="INVALID_ARG"):
        nf.batch_trafo([q, q], [g, g], 0, queue=True)       # one plan twice
    out = nf.batch_trafo([q], [g], 0, queue=True)[0].cpu().numpy()
    assert np.array_equal(out, nf.batch_trafo([q], [g], 0)[0].cpu().numpy())
