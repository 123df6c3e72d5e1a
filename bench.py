"""Benchmark: type-2 NFFT points/s on one MI355X at N = 256^3, M = 1e7.

Workload: coefficients with |k|^-2 decay and random phase (N = 256^3), 1e7
points (half uniform, half in 16 Gaussian clusters of std 0.02), sigma = 2.
One step = one nfft3_trafo (deconvolve + pruned 3-D FFT on the 512^3 grid +
window sums at all points) with the points already set (nfft3_set_points is
the precomputation, timed and reported separately).  ``value`` is the FP32
form (m = 4) points/s; the FP64 form (m = 8) is timed on the same inputs and
reported beside it.  Errors are measured against the FP64 direct-sum oracle
on a seeded sample of the points, which is also the CPU baseline.

    python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
# vector FMA peak without packed FP32 (the build disables packed FP32 ops):
# 256 CUs x 4 SIMDs x 16 lanes x 2 flops x 2.4 GHz; FP64 runs at the same rate
VALU_PEAK_TFS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12
FP64_PEAK_TFLOPS = 78.6        # MI355X FP64 vector
FP32_PEAK_TFLOPS = 157.3       # MI355X FP32 vector (published, packed)
# LDS read rate: 256 B/clk/CU (ds_read_b128, measured) x 256 CUs x 2.4 GHz
LDS_PEAK_TBS = 256 * 256 * 2.4e9 / 1e12


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources of the window-sum kernel whose HBM traffic profiles/ records; the
# recorded traffic is reported only while these files are unchanged.
TRAFFIC_SOURCES = ["paper_1605_01244_amd/csrc/interp_dev.h", "paper_1605_01244_amd/csrc/interp.hip",
                   "paper_1605_01244_amd/csrc/internal.h"]
TRAFFIC_PROFILE = "profiles/interp_window_sums_N256_M1e7_traffic.md"


def strip_comments(src: str) -> str:
    """C++ source without comments and with whitespace collapsed (the code
    the counters depend on)."""
    import re
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"//[^\n]*", " ", src)
    return " ".join(src.split())


def kernel_sources_sha(read=None):
    """Hash of the window-sum kernel sources, comments and layout ignored.
    `read(path)` returns a file's text (default: the working tree)."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        if read is None:
            with open(os.path.join(ROOT, f)) as fp:
                text = fp.read()
        else:
            text = read(f)
        h.update(strip_comments(text).encode())
    return h.hexdigest()


def recorded_traffic(form):
    """HBM bytes per launch of the window-sum kernel from the rocprofv3
    FETCH_SIZE / WRITE_SIZE summary (copy-calibrated), or None when it is
    missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, TRAFFIC_PROFILE)
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("traffic-data:"):
            rec = json.loads(line.split(":", 1)[1])
            if rec.get("kernel_sources_sha256") != kernel_sources_sha():
                return None
            return rec.get(form, {}).get("bytes_per_launch")
    return None


def form_roofline(r, N, M, copy_gbs):
    """Roofline of the dominant kernel of one form's step (the window sums
    at N = 256^3, M = 1e7), seen three ways:
      hbm: algorithmic bytes (grid read once, n^3 elt; per point x 24 B,
           permutation 4 B, result elt) per launch / launch time;
      alu: algorithmic flops of the separable window sum, 4 [(2m)^3 + (2m)^2 +
           2m] per point (real weight x complex value = 2 FMAs per term over x,
           then y, then z), against the vector FMA peak without packed FP32
           (78.6 TFLOP/s, FP32 and FP64 alike; the published 157.3 TFLOP/s
           FP32 figure needs packed FP32 instructions, which this build
           disables) -- the published FP32 figure is reported beside it;
      lds: the (2m)^3 stencil values every point reads from LDS (elt each)
           against 256 B/clk/CU (the measured ds_read_b128 rate) x 256 CUs x
           2.4 GHz.
    `primary` is the bound that applies: HBM for the FP32 form (the window
    sums are balanced between HBM and VALU there), FP64 VALU for the FP64 form."""
    m = r["m"]
    elt = 8 if r["dtype"] == torch_complex64() else 16
    n3 = float(np.prod(r["n"]))
    W = 2 * m
    ms = r["ms_interp"]
    t = ms * 1e-3
    alg_bytes = n3 * elt + M * (24 + 4 + elt)
    gbs = alg_bytes / t / 1e9
    form = "fp32" if elt == 8 else "fp64"
    hbm = {"kernel": "interp (window sums)", "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": gbs / HBM_PEAK_GBS, "traffic": recorded_traffic(form), "alg_bytes_per_launch": alg_bytes,
           "ms_per_launch": ms, "achievable_copy_gbs": copy_gbs, "frac_of_achievable": gbs / copy_gbs}
    fpp = 4.0 * (W ** 3 + W ** 2 + W)
    tfs = M * fpp / t / 1e12
    alu = {"kernel": "interp (window sums)", "bound": "alu", "achieved": tfs, "peak": VALU_PEAK_TFS,
           "unit": "TFLOP/s", "frac": tfs / VALU_PEAK_TFS, "flops_per_point": fpp, "flops_per_launch": M * fpp,
           "peak_note": "vector FMA rate without packed FP32 (256 CUs x 64 lanes x 2 flops x 2.4 GHz)"}
    if elt == 8:
        alu["published_fp32_peak"] = FP32_PEAK_TFLOPS
        alu["frac_of_published_fp32_peak"] = tfs / FP32_PEAK_TFLOPS
    lds_bytes = M * float(W ** 3) * elt
    tbs = lds_bytes / t / 1e12
    lds = {"kernel": "interp (window sums)", "bound": "lds", "achieved": tbs, "peak": LDS_PEAK_TBS, "unit": "TB/s",
           "frac": tbs / LDS_PEAK_TBS, "bytes_per_launch": lds_bytes}
    primary = dict(hbm, alu=alu, lds=lds) if elt == 8 else dict(alu, hbm=hbm, lds=lds)
    return {"hbm": hbm, "alu": alu, "lds": lds, "primary": primary}


def torch_complex64():
    import torch
    return torch.complex64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--N", type=int, default=256)
    ap.add_argument("--M", type=int, default=10_000_000)
    ap.add_argument("--m32", type=int, default=4)
    ap.add_argument("--m64", type=int, default=8)
    ap.add_argument("--cpu-sample", type=int, default=10_000,
                    help="points of the seeded sample evaluated by the oracle (CPU baseline + error)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle (profiling runs)")
    ap.add_argument("--forms", default="fp32,fp64")
    ap.add_argument("--copy-calib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint / point-gradient / batched / autograd measurements")
    ap.add_argument("--only", choices=["batched", "autograd", "rectilinear", "gpe", "lowdim"], default=None,
                    help="run only this extra workload and print its result (profiling runs)")
    return ap.parse_args()


def cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo) and logical CPU count."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return f"{name} ({os.cpu_count()} logical CPUs)"


def median(v):
    v = sorted(v)
    n = len(v)
    return 0.5 * (v[(n - 1) // 2] + v[n // 2])


def event_times(torch, stream, fn, reps):
    """Run fn() reps times back to back on `stream`, with a HIP event before
    the first and after every call; returns (per-call ms list, total ms)."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for i in range(reps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    per = [ev[i].elapsed_time(ev[i + 1]) for i in range(reps)]
    return per, ev[0].elapsed_time(ev[-1])


def copy_bandwidth(torch, dev, stream, mib=1024, reps=5):
    """Achievable HBM bandwidth: a plain device-to-device copy of `mib` MiB
    (read + write bytes / time, HIP events)."""
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.copy_(a)
    e1.record(stream)
    torch.cuda.synchronize()
    gbs = 2.0 * a.numel() * 4 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def bench_batched(nf, torch, dev, workloads, stream):
    """64 coefficient sets of N in {64, 96, 128}^3 with lognormal point
    counts, each with its three derivative fields: one nfft3_batch_trafo per
    form (one launch per FFT stage and axis length plus one window-sum launch,
    each over all transforms of the batch: 256 in FP32, whose derivative
    fields are spectral; 64 in FP64, whose window sums also form the
    derivative fields), and the same batch as one work-queue launch
    (nfft3_batch_trafo_queue, `queue_ms_per_batch`), timed with HIP events."""
    t0 = time.time()
    sets = workloads.batched_sets(64)
    log(f"batched inputs generated in {time.time() - t0:.1f}s")
    res = {"workload": "64 sets, N in {64,96,128}^3, M_t lognormal in [1e4,1e6] (total "
                       f"{sum(s[2].shape[0] for s in sets)}), field + 3 derivative fields each, sigma=2"}
    for form, dt, m in (("fp32", torch.complex64, 4), ("fp64", torch.complex128, 8)):
        plans, fh = [], []
        for N, f, x in sets:
            p = nf.Plan((N, N, N), m=m, dtype=dt, device=dev)
            p.set_points(torch.from_numpy(x).to(dev))
            plans.append(p)
            fh.append(torch.from_numpy(f).to(dev).to(dt))
        nf.batch_trafo(plans, fh, 7)
        torch.cuda.synchronize()
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            outs = nf.batch_trafo(plans, fh, 7)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        qouts = nf.batch_trafo(plans, fh, 7, queue=True)
        torch.cuda.synchronize()
        same = all(torch.equal(a, b) for a, b in zip(outs, qouts))
        e0.record(stream)
        for _ in range(reps):
            qouts = nf.batch_trafo(plans, fh, 7, queue=True)
        e1.record(stream)
        torch.cuda.synchronize()
        qms = e0.elapsed_time(e1) / reps
        evals = 4 * sum(p.M for p in plans)
        res[form] = {"m": m, "ms_per_batch": ms, "point_evaluations_per_s": evals / (ms * 1e-3),
                     "queue_ms_per_batch": qms, "queue_equals_launches": bool(same)}
        log(f"batched {form}: {ms:.2f} ms per batch of 64 sets x 4 fields ({evals / ms * 1e3:.3e} evaluations/s); "
            f"one work-queue launch {qms:.2f} ms (bit-equal: {same})")
        del qouts
        for p in plans:
            p.close()
        del plans, fh, outs
        torch.cuda.empty_cache()
    return res


def bench_rgrid(nf, torch, dev, workloads, stream):
    """Evaluation at a rectilinear grid (Sec. 2.1) on the matrix cores: the
    paper's 64^3 coefficients at a 64^3 grid, and 256^3 power-law
    coefficients at a nonuniform 321^3 grid; per form the median event time
    of nfft3_rgrid_eval and its rate against the dense MFMA peak of its dtype
    (algorithmic flops 8 (N0 N1 N2 M2 + N0 N1 M1 M2 + N0 M0 M1 M2), the
    conventional count of four real products per complex multiply-add; the
    kernel issues three (Gauss's form), so `issued_frac` reports 6/8 of that
    rate, the matrix cores' own utilisation)."""
    res = {}
    r = np.random.default_rng(16)
    for name, N, M in (("64^3->64^3", (64, 64, 64), (64, 64, 64)), ("256^3->321^3", (256, 256, 256), (321, 321, 321))):
        fh = workloads.powerlaw_coeffs(N, 301) if N[0] == 256 else (
            np.random.default_rng(13).standard_normal(N) + 1j * np.random.default_rng(14).standard_normal(N))
        ys = [torch.from_numpy(np.sort(r.uniform(-0.5, 0.5, size=m))).to(dev) for m in M]
        flops = 8.0 * (N[0] * N[1] * N[2] * M[2] + N[0] * N[1] * M[1] * M[2] + N[0] * M[0] * M[1] * M[2])
        entry = {"N": list(N), "M": list(M), "flops": flops}
        for form, dt, peak in (("fp64", torch.complex128, FP64_PEAK_TFLOPS), ("fp32", torch.complex64, FP32_PEAK_TFLOPS)):
            g = nf.RectGrid(N, M, dtype=dt, device=dev)
            g.set_axes(*ys)
            fd = torch.from_numpy(fh).to(dev).to(dt)
            out = torch.empty(M, dtype=dt, device=dev)
            g.eval(fd, out=out)
            ms = median(event_times(torch, stream, lambda: g.eval(fd, out=out), 10)[0])
            tfs = flops / (ms * 1e-3) / 1e12
            entry[form] = {"ms": ms, "tflops": tfs, "peak_tflops": peak, "frac": tfs / peak,
                           "issued_frac": 0.75 * tfs / peak,
                           "points_per_s": M[0] * M[1] * M[2] / (ms * 1e-3)}
            log(f"rectilinear {name} {form}: {ms:.3f} ms, {tfs:.1f} TFLOP/s ({tfs / peak:.2f} of MFMA peak)")
            g.close()
            del out, fd
        res[name] = entry
        torch.cuda.empty_cache()
    return res


def bench_lowdim(nf, torch, dev, workloads, stream):
    """One- and two-dimensional plans (Appendix B's infft / infft2): N = 1024
    and 1024^2 |k|^-2 coefficients at M = 1e7 uniform points; per form the
    median event time of nfft3_trafo, its stages, and the window sums' HBM
    rate (algorithmic bytes: the grid once, 28 B per point for its sorted
    coordinates and index, the result)."""
    res = {}
    M = 10_000_000
    for d, N in ((1, 1024), (2, 1024)):
        fh, x = workloads.lowdim_case(d, N, M)
        xd = torch.from_numpy(x).to(dev)
        name = f"{d}-D N={N}^{d}" if d > 1 else f"1-D N={N}"
        entry = {"N": [N] * d, "M": M}
        for form, dt, m in (("fp64", torch.complex128, 8), ("fp32", torch.complex64, 4)):
            plan = nf.Plan((N,) * d, m=m, dtype=dt, device=dev)
            plan.set_points(xd)
            fd = torch.from_numpy(fh).to(dev).to(dt)
            out = torch.empty(M, dtype=dt, device=dev)
            plan.trafo(fd, out=out)
            ms = median(event_times(torch, stream, lambda: plan.trafo(fd, out=out), 10)[0])
            ms_grid = median(event_times(torch, stream, lambda: plan.stage_grid(fd), 10)[0])
            ms_interp = median(event_times(torch, stream, lambda: plan.stage_interp(out), 10)[0])
            elt = 16 if form == "fp64" else 8
            alg = float(np.prod(plan.n)) * elt + M * (28 + elt)
            gbs = alg / (ms_interp * 1e-3) / 1e9
            entry[form] = {"m": m, "ms": ms, "points_per_s": M / (ms * 1e-3), "ms_grid_stage": ms_grid,
                           "ms_interp_stage": ms_interp, "interp_gbs": gbs, "interp_hbm_frac": gbs / HBM_PEAK_GBS}
            log(f"{name} {form}: {ms:.3f} ms ({M / ms * 1e3:.3e} pts/s), grid {ms_grid:.3f} ms, "
                f"window sums {ms_interp:.3f} ms ({gbs:.0f} GB/s)")
            plan.close()
            del out, fd
        res[name] = entry
        del xd
        torch.cuda.empty_cache()
    return res


def bench_gpe_tube(nf, torch, dev, workloads, stream):
    """The paper's pipeline of Sec. 5 on its grid: Strang steps of the GPE
    (N = 80^3 on [-20, 60)^3, tau = 0.1, 200 steps to T = 20) from two
    straight vortices, then the state's coefficients and the evaluation
    within vortex tubes (rho <= 0.2, then 0.05) on the physical domain.
    Times from HIP events; FP64 and FP32."""
    N, a, b = 80, -20.0, 60.0
    psi0 = workloads.gpe_two_vortices(N, a, b)
    res = {"workload": "GPE Strang splitting, 80^3 on [-20,60)^3, tau=0.1, 200 steps; then vortex-tube "
                       "evaluation rho <= 0.2, 0.05 of the final state"}
    A3, B3 = [a] * 3, [b] * 3
    for form, dt, m in (("fp64", torch.complex128, 8), ("fp32", torch.complex64, 4)):
        g = nf.GPE((N, N, N), A3, B3, dtype=dt, device=dev)
        g.set_state(torch.from_numpy(psi0).to(dev).to(dt))
        g.step(0.1, 2)
        g.set_state(torch.from_numpy(psi0).to(dev).to(dt))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        g.step(0.1, 200)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        ph = g.coeffs()
        plan = nf.Plan((N, N, N), m=m, dtype=dt, device=dev)
        plan.tube_refine(ph, A3, B3, [0.2, 0.05])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pts, rho = plan.tube_refine(ph, A3, B3, [0.2, 0.05])
        torch.cuda.synchronize()
        t_tube = time.perf_counter() - t0
        res[form] = {"m": m, "gpe_ms_per_step": ms / 200, "gpe_ms_total": ms, "tube_ms": t_tube * 1e3,
                     "tube_points": int(pts.shape[0])}
        log(f"gpe {form}: {ms / 200:.3f} ms per step; tube refinement {t_tube * 1e3:.1f} ms, "
            f"{pts.shape[0]} points")
        plan.close()
        g.close()
        torch.cuda.empty_cache()
    return res


def bench_autograd(nf, torch, dev, workloads):
    """Differentiation form: N = 128^3, M = 1e6 clustered points; forward
    (set_points + trafo) and backward (adjoint + point gradient) of
    L = sum Re(conj(w) f), wall time per step on the device clock."""
    fhat, x, w = workloads.clustered_grad_case(128, 1_000_000)
    res = {"workload": "N=128^3, M=1e6 points in 16 clusters std 0.02, L = sum Re(conj(w) f)"}
    for form, dt, m in (("fp32", torch.complex64, 4), ("fp64", torch.complex128, 8)):
        plan = nf.Plan(fhat.shape, m=m, dtype=dt, device=dev)
        fh = torch.from_numpy(fhat).to(dev).to(dt).requires_grad_(True)
        xd = torch.from_numpy(x).to(dev).requires_grad_(True)
        wd = torch.from_numpy(w).to(dev).to(dt)

        def step():
            fh.grad = None
            xd.grad = None
            f = nf.type2(fh, xd, plan)
            (torch.conj(wd) * f).real.sum().backward()

        step()
        torch.cuda.synchronize()
        reps = 3
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            step()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[form] = {"m": m, "ms_forward_backward": ms}
        log(f"autograd {form}: {ms:.2f} ms per forward+backward")
        plan.close()
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    import paper_1605_01244_amd as nf
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.only:
        stream = torch.cuda.current_stream(dev)
        if args.only == "batched":
            res = bench_batched(nf, torch, dev, workloads, stream)
        elif args.only == "rectilinear":
            res = bench_rgrid(nf, torch, dev, workloads, stream)
        elif args.only == "gpe":
            res = bench_gpe_tube(nf, torch, dev, workloads, stream)
        elif args.only == "lowdim":
            res = bench_lowdim(nf, torch, dev, workloads, stream)
        else:
            res = bench_autograd(nf, torch, dev, workloads)
        print(json.dumps({args.only: res}), flush=True)
        return
    t0 = time.time()
    N, M = args.N, args.M
    fh, x = workloads.powerlaw_mixed_case(N, M)
    log(f"inputs generated in {time.time() - t0:.1f}s: N={N}^3 M={M}")
    x_d = torch.from_numpy(x).to(dev)
    fh64 = torch.from_numpy(fh).to(dev)
    fh32 = fh64.to(torch.complex64)
    sample = workloads.sample_indices(M, 10_000, 306)[: max(0, args.cpu_sample)]

    if args.copy_calib:
        a = torch.empty(args.copy_calib * (1 << 20) // 4, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    stream = torch.cuda.current_stream(dev)
    copy_gbs = copy_bandwidth(torch, dev, stream)
    log(f"device copy: {copy_gbs:.0f} GB/s")
    results = {}
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    for form in forms:
        m = args.m32 if form == "fp32" else args.m64
        dt = torch.complex64 if form == "fp32" else torch.complex128
        fhd = fh32 if form == "fp32" else fh64
        plan = nf.Plan((N, N, N), sigma=2.0, m=m, dtype=dt, device=dev)
        # precomputation
        torch.cuda.synchronize()
        ts = time.perf_counter()
        plan.set_points(x_d)
        torch.cuda.synchronize()
        t_set = time.perf_counter() - ts
        # a repeated call (buffers already allocated): the cost when points change
        ts = time.perf_counter()
        plan.set_points(x_d)
        torch.cuda.synchronize()
        t_set2 = time.perf_counter() - ts
        out = torch.empty(M, dtype=dt, device=dev)
        for _ in range(args.warmup):
            plan.trafo(fhd, out=out)
        torch.cuda.synchronize()
        # timed region: K whole steps, one event between consecutive steps
        w0 = time.perf_counter()
        step_ms, total_ms = event_times(torch, stream, lambda: plan.trafo(fhd, out=out), args.steps)
        wall = time.perf_counter() - w0
        ms_step = median(step_ms)
        # per-stage launch durations (HIP events on the plan's stream)
        ms_grid = median(event_times(torch, stream, lambda: plan.stage_grid(fhd), args.steps)[0])
        ms_interp = median(event_times(torch, stream, lambda: plan.stage_interp(out=out), args.steps)[0])
        extra = {}
        if not args.no_extras:
            # adjoint (type-1: spread + adjoint FFT passes + truncate) and the
            # point gradient on the same plan and points
            G = out.clone()
            adj = torch.empty_like(fhd)
            reps = max(3, args.steps // 2)
            plan.adjoint(G, out=adj)
            ms_adj = median(event_times(torch, stream, lambda: plan.adjoint(G, out=adj), reps)[0])
            ms_spread = median(event_times(torch, stream, lambda: plan.stage_spread(G), reps)[0])
            plan.grad_points(fhd, G)
            ms_gx = median(event_times(torch, stream, lambda: plan.grad_points(fhd, G), reps)[0])
            extra = {"adjoint_ms": ms_adj, "spread_stage_ms": ms_spread, "grad_points_ms": ms_gx}
            del G, adj
        f = out[torch.from_numpy(sample).to(dev)].cpu().numpy() if len(sample) else None
        results[form] = dict(m=m, dtype=dt, ms_step=ms_step, ms_step_mean=total_ms / args.steps, wall_s=wall, t_set=t_set, t_set2=t_set2, ms_grid=ms_grid,
                             ms_interp=ms_interp, f_sample=f, n=plan.n, tuning=plan.tuning(), extra=extra)
        log(f"{form} m={m}: {ms_step:.3f} ms/step ({M / ms_step * 1e3:.3e} pts/s); grid stage {ms_grid:.3f} ms, "
            f"interp stage {ms_interp:.3f} ms; set_points {t_set * 1e3:.1f} ms")
        plan.close()
        del plan
        torch.cuda.empty_cache()

    extras = {}
    if not args.no_extras:
        del x_d, fh32, fh64
        torch.cuda.empty_cache()
        extras["batched"] = bench_batched(nf, torch, dev, workloads, stream)
        extras["autograd"] = bench_autograd(nf, torch, dev, workloads)
        extras["rectilinear"] = bench_rgrid(nf, torch, dev, workloads, stream)
        extras["gpe_tube"] = bench_gpe_tube(nf, torch, dev, workloads, stream)
        extras["lowdim"] = bench_lowdim(nf, torch, dev, workloads, stream)

    # CPU baseline = the oracle on the seeded sample (also the error reference)
    cpu = None
    errs = {}
    if not args.no_cpu and len(sample):
        import oracle
        threads = oracle.default_threads()
        tc = time.perf_counter()
        ref = oracle.ndft_trafo(fh, x[sample], threads=threads)
        t_cpu = time.perf_counter() - tc
        # single-thread rate on the first 300 points of the same sample
        n1 = min(300, len(sample))
        t1 = time.perf_counter()
        oracle.ndft_trafo(fh, x[sample[:n1]], threads=1)
        t1 = time.perf_counter() - t1
        cpu = {"value": len(sample) / t_cpu, "unit": "points/s", "cores": threads, "kind": "oracle",
               "sample": f"{len(sample)} seeded points (seed 306) of the 1e7, direct FP64 sum over all "
                         f"{N}^3 coefficients, {t_cpu:.1f} s wall",
               "single_thread_value": n1 / t1, "single_thread_sample": f"first {n1} points of the sample",
               "cpu_model": cpu_model()}
        for form, r in results.items():
            errs[form] = oracle.rel_errors(r["f_sample"], ref)
        log(f"oracle: {len(sample)} points in {t_cpu:.1f}s on {threads} threads; errors {errs}")

    main_form = "fp32" if "fp32" in results else forms[0]
    r = results[main_form]
    rooflines = {form: form_roofline(rr, N, M, copy_gbs) for form, rr in results.items()}
    line = {
        "metric": "NFFT points/sec at N=256^3, M=1e7 (FP32 m=4 vs FP64 m=8) at stated rel-l2 error",
        "value": M / (r["ms_step"] * 1e-3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 (f32 grid/FFT/window sums, f64 point index math)" if main_form == "fp32" else "c128",
        "data": "synthetic",
        "config": {"workload": f"type-2 NFFT, N={N}^3 |k|^-2 random-phase coefficients, M={M} points "
                               f"(50% uniform, 50% in 16 Gaussian clusters std 0.02), sigma=2, "
                               f"{main_form} m={r['m']}; points set once, step = trafo",
                   "N": N, "M": M, "sigma": 2.0, "m": r["m"], "parallelism": "single GPU"},
        "roofline": dict(rooflines[main_form]["hbm"], alu=rooflines[main_form]["alu"],
                         lds=rooflines[main_form]["lds"]),
        "cpu_baseline": cpu,
        "forms": {},
    }
    for form, rr in results.items():
        line["forms"][form] = {
            "m": rr["m"], "points_per_s": M / (rr["ms_step"] * 1e-3), "ms_per_step": rr["ms_step"],
            "ms_grid_stage": rr["ms_grid"], "ms_interp_stage": rr["ms_interp"],
            "set_points_ms": rr["t_set"] * 1e3, "set_points_repeat_ms": rr["t_set2"] * 1e3,
            "points_per_s_incl_set_points": M / ((rr["ms_step"] + rr["t_set2"] * 1e3) * 1e-3),
            "wall_s_timed": rr["wall_s"],
            "tile": rr["tuning"][0], "points_per_item": rr["tuning"][1], **rr["extra"],
            "rel_l2": errs.get(form, (None, None))[0], "rel_linf": errs.get(form, (None, None))[1],
            "ms_per_step_mean": rr["ms_step_mean"],
            "roofline": rooflines[form]["primary"],
        }
    if extras:
        line["extras"] = extras
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
