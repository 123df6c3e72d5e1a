"""nfft3_batch_trafo_noalloc: the batched evaluation without device
allocation (its launch descriptors live in a static device array).  Checked
against nfft3_batch_trafo on the same inputs (bit for bit: same kernels) and
the oracle, on two calls in a row, the second with a smaller batch; plus its
two error paths (capacity of the static array, missing field grids)."""
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


def _batch(nf, spec, dtype, m, seed):
    plans, fh, raw = [], [], []
    for i, (N, M) in enumerate(spec):
        f = rand_coeffs(N, seed + i)
        x = rand_points(M, seed + 100 + i)
        p = nf.Plan(N, sigma=2.0, m=m, dtype=torch_dtype(dtype), device="cuda:0")
        p.set_points(to_dev(x))
        plans.append(p)
        fh.append(to_dev(f, dtype))
        raw.append((f, x))
    return plans, fh, raw


@pytest.mark.parametrize("dtype", ["c64", "c128"])
def test_noalloc_matches_allocating_batch_twice(nf, dtype):
    import torch
    m = 4 if dtype == "c64" else 8
    mask = 7
    spec = [((16, 16, 16), 3000), ((24, 20, 16), 1200), ((32, 32, 32), 2500), ((12, 16, 10), 1), ((16, 24, 32), 800)]
    plans, fh, raw = _batch(nf, spec, dtype, m, 300)
    for call, T in enumerate((5, 3)):          # second call: a smaller batch
        P, F = plans[:T], fh[:T]
        log(f"noalloc {dtype} call {call} T={T}")
        ref = nf.batch_trafo(P, F, mask)        # allocating entry point (makes the field grids)
        out = [torch.empty_like(r) for r in ref]
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info(0)[0]
        got = nf.batch_trafo(P, F, mask, out=out, allocate=False)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(0)[0]
        assert free1 >= free0, (free0, free1)   # no device memory taken
        for t in range(T):
            g = got[t].cpu().numpy()
            assert np.array_equal(g, ref[t].cpu().numpy()), (call, t)
            f, x = raw[t]
            l2, li = rel(g[0], oracle.ndft_trafo(f, x))
            assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (call, t, l2, li)
            if t == 0:
                D = oracle.ndft_grad(f, x)
                for d in range(3):
                    l2, li = rel(g[1 + d], D[:, d])
                    assert l2 <= tol(m, 2.0, dtype) and li <= tol(m, 2.0, dtype), (call, d, l2, li)


def test_noalloc_rejects_oversized_batch_and_missing_grids(nf):
    import torch
    # 120 plans x 4 fields x ~560-byte descriptors exceed the 256 KiB array
    plans, fh, _ = _batch(nf, [((4, 4, 4), 3)] * 120, "c64", 2, 900)
    log("noalloc capacity")
    with pytest.raises(nf.NFFT3Error) as e:
        nf.batch_trafo(plans, fh, 7, allocate=False)
    assert e.value.code == -8
    # fields without their grids (no allocating call with this mask yet)
    with pytest.raises(nf.NFFT3Error) as e:
        nf.batch_trafo(plans[:2], fh[:2], 1, allocate=False)
    assert e.value.code == -1
    # without derivative fields every plan has its grid: fine, and bit-equal
    got = nf.batch_trafo(plans[:50], fh[:50], 0, allocate=False)
    ref = nf.batch_trafo(plans[:50], fh[:50], 0)
    for g, r in zip(got, ref):
        assert np.array_equal(g.cpu().numpy(), r.cpu().numpy())
    torch.cuda.synchronize()
