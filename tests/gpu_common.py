"""Shared helpers for the GPU tests: tolerances, device transfers, plans."""
from __future__ import annotations

import math

import numpy as np

from oracle import nfft_steps as ns


def tol(m: int, sigma: float, dtype: str) -> float:
    """Gate on rel-l2 and rel-linf against the direct-sum oracle.

    FP64: the Kaiser-Bessel error estimate E(m, sigma), floored at 1e-12
    (m = 8, sigma = 2 gives 4e-14, so the gate is 1e-12).
    FP32: E(m, sigma) plus single-precision rounding of the grid, FFT and
    window sums (~5e-7), floored at 2e-6 (m = 4, sigma = 2 gives 1.7e-6).
    """
    e = ns.pst_error_bound(m, sigma)
    if dtype == "c128":
        return max(e, 1e-12)
    return max(e + 5e-7, 2e-6)


def torch_dtype(dtype: str):
    import torch
    return torch.complex128 if dtype == "c128" else torch.complex64


def to_dev(a: np.ndarray, dtype: str | None = None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(torch_dtype(dtype))
    return t.to("cuda:0")


def phi0(m: int, sigma: float) -> float:
    return float(ns.kb_phi(np.array([0.0]), m, sigma)[0])


def rel(got, ref):
    got = np.asarray(got).reshape(-1)
    ref = np.asarray(ref).reshape(-1)
    d = got - ref
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.max(np.abs(d)) / np.max(np.abs(ref))))


def log(msg: str) -> None:
    print(msg, flush=True)


def stage_tol(m: int, dtype: str, sigma: float = 2.0) -> float:
    """Gate of a stage against its numpy statement (both sides rounded).

    FP64: the window phi(t) = sinh(b sqrt(m^2 - t^2)) / ... grows like
    exp(b sqrt(m^2 - t^2)), so a rounding eps in t moves it by a relative
    b*m*eps at worst, in the reference's closed form and in the fitted
    polynomials alike; three such factors per term: 3 b m eps, floored at
    1e-14.  FP32: single-precision rounding of weights and sums, 1e-6."""
    if dtype == "c64":
        return 1e-6
    b = np.pi * (2.0 - 1.0 / sigma)
    return max(1e-14, 3.0 * b * m * np.finfo(np.float64).eps)


def rand_coeffs(N, seed):
    r = np.random.default_rng(seed)
    return r.standard_normal(tuple(N)) + 1j * r.standard_normal(tuple(N))


def rand_points(M, seed):
    return np.random.default_rng(seed).uniform(-0.5, 0.5, size=(int(M), 3))


def dot_tol(dtype: str) -> float:
    return 1e-12 if dtype == "c128" else 2e-5


__all__ = ["tol", "torch_dtype", "to_dev", "phi0", "rel", "log", "rand_coeffs", "rand_points",
           "dot_tol", "math"]
