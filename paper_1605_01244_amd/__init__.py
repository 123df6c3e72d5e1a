"""MI355X (gfx950) nonequispaced FFT in one, two and three dimensions.

Python binding of ``libnfft3.so`` (C ABI in ``include/nfft3.h``).  This
module only marshals arguments: every step of the computation -- point
binning, deconvolution, FFT, window sums, adjoint spreading, point
gradients -- runs in the library's HIP kernels.  PyTorch provides device
memory and the current HIP stream; there is no CPU path.

    plan = Plan((256, 256, 256), sigma=2.0, m=4, dtype=torch.complex64)
    plan.set_points(x)               # (M, 3) float64 on the GPU
    f = plan.trafo(fhat)             # f_j = sum_k fhat_k exp(-2 pi i k.x_j)
    fhat_adj = plan.adjoint(f)       # sum_j f_j exp(+2 pi i k.x_j)
    f = type2(fhat, x, plan)         # differentiable in fhat and x

The evaluated sum is the NFFT problem of Sec. 2.2.1 of Caliari & Zuccher
(arXiv:1605.01244): frequencies k_d = -N_d/2 .. N_d/2-1 stored at array index
k_d + N_d/2 (C order), points in the unit box [-1/2, 1/2)^3 (folded
periodically).
"""
from __future__ import annotations

import ctypes
import math
from typing import Sequence

import torch  # noqa: F401  (loads the HIP runtime the library binds to)

from ._lib import NFFT3_C64, NFFT3_C128, NFFT3Error, check, lib

__all__ = ["Plan", "RectGrid", "GPE", "type2", "batch_trafo", "infft", "infft2", "infft3", "deconv_factors",
           "window_poly", "NFFT3Error"]

_DT = {torch.complex64: NFFT3_C64, torch.complex128: NFFT3_C128}


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """An NFFT plan: coefficient sizes N (1, 2 or 3 axes: the one-, two- and
    three-dimensional series), oversampling sigma, window half-width m,
    precision dtype (torch.complex64 or torch.complex128).  Points are
    (M, len(N)) float64 arrays."""

    def __init__(self, N: Sequence[int], sigma: float = 2.0, m: int = 8,
                 dtype: torch.dtype = torch.complex128, device=None):
        if dtype not in _DT:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("Plan needs a GPU device")
        self.N = tuple(int(v) for v in N)
        self.dim = len(self.N)
        if self.dim not in (1, 2, 3):
            raise ValueError("N must have 1, 2 or 3 entries")
        self.sigma = float(sigma)
        self.m = int(m)
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        Narr = (ctypes.c_int64 * self.dim)(*self.N)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(lib.nfft3_plan_nd(ctypes.byref(self._h), self.dim, Narr, self.sigma, self.m, _DT[dtype],
                                    ctypes.c_void_p(stream)), "nfft3_plan_nd")
        n = (ctypes.c_int64 * 3)()
        check(lib.nfft3_get_info(self._h, n, None), "nfft3_get_info")
        self.n = tuple(int(v) for v in n)[3 - self.dim:]
        self.M = 0
        self.epoch = 0

    # -- helpers -------------------------------------------------------
    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.nfft3_set_stream(self._h, ctypes.c_void_p(s)), "nfft3_set_stream")

    def _coeffs(self, fhat: torch.Tensor) -> torch.Tensor:
        if fhat.shape != self.N:
            raise ValueError(f"coefficients must have shape {self.N}, got {tuple(fhat.shape)}")
        if fhat.dtype != self.dtype or fhat.device != self.device:
            raise TypeError(f"coefficients must be {self.dtype} on {self.device}")
        return fhat.contiguous()

    def _values(self, f: torch.Tensor, count: int = 1) -> torch.Tensor:
        if f.dtype != self.dtype or f.device != self.device:
            raise TypeError(f"values must be {self.dtype} on {self.device}")
        if f.numel() != count * self.M:
            raise ValueError(f"expected {count * self.M} values, got {f.numel()}")
        return f.contiguous()

    @staticmethod
    def _out(out: torch.Tensor) -> torch.Tensor:
        # the library writes a dense block at the tensor's first address
        if not out.is_contiguous():
            raise ValueError("out must be a contiguous tensor")
        return out

    def _points(self, x: torch.Tensor) -> torch.Tensor:
        if x.dim() != 2 or x.shape[1] != self.dim:
            raise ValueError(f"points must have shape (M, {self.dim})")
        if x.dtype != torch.float64 or x.device != self.device:
            raise TypeError("points must be float64 on the plan's device")
        return x.contiguous()

    def close(self):
        if self._h:
            lib.nfft3_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- the C ABI ---------------------------------------------------------
    def set_points(self, x: torch.Tensor) -> None:
        """x: (M, dim) float64 on the plan's device."""
        x = self._points(x)
        self._bind_stream()
        self.epoch += 1
        self.M = 0
        check(lib.nfft3_set_points(self._h, x.shape[0], _ptr(x)), "nfft3_set_points")
        self.M = int(x.shape[0])

    def set_points_if_changed(self, x: torch.Tensor) -> bool:
        """set_points(x) unless the plan's sorted points are exactly those of
        x (nfft3_points_unchanged compares every folded coordinate on the
        device, so writes that bypass the tensor's version counter, such as
        through .data, are seen).  Returns True if the points were sorted."""
        x = self._points(x)
        if self.M == x.shape[0]:
            xc = x
            same = ctypes.c_int(0)
            self._bind_stream()
            check(lib.nfft3_points_unchanged(self._h, xc.shape[0], _ptr(xc), ctypes.byref(same)),
                  "nfft3_points_unchanged")
            if same.value:
                return False
        self.set_points(x)
        return True

    def trafo(self, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        fhat = self._coeffs(fhat)
        if out is None:
            out = torch.empty(self.M, dtype=self.dtype, device=self.device)
        self._values(self._out(out))
        self._bind_stream()
        check(lib.nfft3_trafo(self._h, _ptr(fhat), _ptr(out)), "nfft3_trafo")
        return out

    def trafo_fields(self, fhat: torch.Tensor, deriv_mask: int | None = None) -> torch.Tensor:
        """(1 + popcount(mask), M): the field and its derivative fields (bit
        d of the mask = the plan's axis d; default all axes)."""
        fhat = self._coeffs(fhat)
        if deriv_mask is None:
            deriv_mask = (1 << self.dim) - 1
        k = 1 + bin(deriv_mask & 7).count("1")
        out = torch.empty((k, self.M), dtype=self.dtype, device=self.device)
        self._bind_stream()
        check(lib.nfft3_trafo_fields(self._h, _ptr(fhat), _ptr(out), int(deriv_mask)), "nfft3_trafo_fields")
        return out

    def adjoint(self, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        f = self._values(f)
        if out is None:
            out = torch.empty(self.N, dtype=self.dtype, device=self.device)
        self._coeffs(self._out(out))
        self._bind_stream()
        check(lib.nfft3_adjoint(self._h, _ptr(f), _ptr(out)), "nfft3_adjoint")
        return out

    def grad_points(self, fhat: torch.Tensor, G: torch.Tensor) -> torch.Tensor:
        """(M, dim) float64: Re(conj(G_j) d f_j / d x_{j,d})."""
        fhat = self._coeffs(fhat)
        G = self._values(G)
        out = torch.empty((self.M, self.dim), dtype=torch.float64, device=self.device)
        self._bind_stream()
        check(lib.nfft3_grad_points(self._h, _ptr(fhat), _ptr(G), _ptr(out)), "nfft3_grad_points")
        return out

    # -- the series on a physical domain (eq. (fs)) and vortex tubes ---------
    def _domain(self, a, b):
        a, b = [float(v) for v in a], [float(v) for v in b]
        if len(a) != self.dim or len(b) != self.dim:
            raise ValueError(f"a and b must have {self.dim} entries")
        return (ctypes.c_double * self.dim)(*a), (ctypes.c_double * self.dim)(*b)

    def infft3(self, psihat: torch.Tensor, a, b, xi: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """psi(xi) = sum_k psihat_k prod_d exp(2 pi i k_d (xi_d - a_d)/(b_d - a_d)) / sqrt(b_d - a_d)
        at the (M, dim) float64 points xi of the domain prod [a_d, b_d) (for
        dim 1 and 2 the paper's infft and infft2); the plan's points become
        the mapped xi."""
        psihat = self._coeffs(psihat)
        xi = self._points(xi)
        M = int(xi.shape[0])
        if out is None:
            out = torch.empty(M, dtype=self.dtype, device=self.device)
        elif out.numel() != M or out.dtype != self.dtype or out.device != self.device:
            raise ValueError(f"out must hold {M} {self.dtype} values on {self.device}")
        self._out(out)
        A, B = self._domain(a, b)
        self._bind_stream()
        self.epoch += 1
        self.M = 0
        check(lib.nfft3_infft3(self._h, A, B, _ptr(psihat), M, _ptr(xi), _ptr(out)), "nfft3_infft3")
        self.M = M
        return out

    infft = infft3      # any number of axes: the paper's infft / infft2 / infft3

    def tube_refine(self, psihat: torch.Tensor, a, b, rhobar: Sequence[float], cap: int | None = None):
        """Evaluation within vortex tubes (Sec. 4.3): returns (points (K, 3)
        float64, rho (K,) float64) of the last refined set."""
        psihat = self._coeffs(psihat)
        A, B = self._domain(a, b)
        L = len(rhobar)
        rb = (ctypes.c_double * max(L, 1))(*[float(v) for v in rhobar])
        count = ctypes.c_int64(0)
        self._bind_stream()
        if cap is None:
            n = math.prod(self.N)
            cap = n if L == 0 else 0        # first pass sizes the output
        pts = torch.empty((max(cap, 1), 3), dtype=torch.float64, device=self.device)
        rho = torch.empty(max(cap, 1), dtype=torch.float64, device=self.device)
        self.epoch += 1
        self.M = 0
        code = lib.nfft3_tube_refine(self._h, A, B, _ptr(psihat), L, rb, int(cap), _ptr(pts), _ptr(rho),
                                     ctypes.byref(count))
        if code == -8:                      # capacity: size the output and run again
            cap = int(count.value)
            pts = torch.empty((max(cap, 1), 3), dtype=torch.float64, device=self.device)
            rho = torch.empty(max(cap, 1), dtype=torch.float64, device=self.device)
            code = lib.nfft3_tube_refine(self._h, A, B, _ptr(psihat), L, rb, int(cap), _ptr(pts), _ptr(rho),
                                         ctypes.byref(count))
        check(code, "nfft3_tube_refine")
        K = int(count.value)
        self.M = K
        return pts[:K], rho[:K]

    # -- binning tuning ------------------------------------------------------
    def set_tuning(self, tile: int = 0, items: int = 0) -> None:
        """Tile edge (8/16/32 cells) and points per work item (256/512) of the
        window sums; 0 keeps a value.  A change drops the points."""
        check(lib.nfft3_set_tuning(self._h, int(tile), int(items)), "nfft3_set_tuning")
        M = ctypes.c_int64()
        check(lib.nfft3_get_info(self._h, None, ctypes.byref(M)), "nfft3_get_info")
        if int(M.value) != self.M:      # the points were dropped
            self.M = int(M.value)
            self.epoch += 1

    def tuning(self):
        t, i = ctypes.c_int(), ctypes.c_int()
        check(lib.nfft3_get_tuning(self._h, ctypes.byref(t), ctypes.byref(i)), "nfft3_get_tuning")
        return int(t.value), int(i.value)

    def autotune(self, x: torch.Tensor, fhat: torch.Tensor, reps: int = 3):
        """Time trafo for every binning candidate on these points and
        coefficients, keep the fastest (points stay set).  Returns (tile, items)."""
        x = self._points(x)
        fhat = self._coeffs(fhat)
        out = torch.empty(x.shape[0], dtype=self.dtype, device=self.device)
        t, i = ctypes.c_int(), ctypes.c_int()
        self._bind_stream()
        self.epoch += 1
        self.M = 0
        check(lib.nfft3_autotune(self._h, x.shape[0], _ptr(x), _ptr(fhat), _ptr(out), int(reps),
                                 ctypes.byref(t), ctypes.byref(i)), "nfft3_autotune")
        self.M = int(x.shape[0])
        return int(t.value), int(i.value)

    # -- stage access (tests, benchmarks) ------------------------------------
    def stage_grid(self, fhat: torch.Tensor, deriv_axis: int = -1) -> None:
        fhat = self._coeffs(fhat)
        self._bind_stream()
        check(lib.nfft3_stage_grid(self._h, _ptr(fhat), int(deriv_axis)), "nfft3_stage_grid")

    def stage_interp(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.M, dtype=self.dtype, device=self.device)
        self._values(self._out(out))
        self._bind_stream()
        check(lib.nfft3_stage_interp(self._h, _ptr(out)), "nfft3_stage_interp")
        return out

    def stage_spread(self, f: torch.Tensor) -> None:
        f = self._values(f)
        self._bind_stream()
        check(lib.nfft3_stage_spread(self._h, _ptr(f)), "nfft3_stage_spread")

    def grid(self) -> torch.Tensor:
        out = torch.empty(self.n, dtype=self.dtype, device=self.device)
        self._bind_stream()
        check(lib.nfft3_grid_copy(self._h, _ptr(out), 0), "nfft3_grid_copy")
        return out

    def load_grid(self, g: torch.Tensor) -> None:
        if tuple(g.shape) != self.n or g.dtype != self.dtype or g.device != self.device:
            raise ValueError("grid must match the plan's oversampled size, dtype and device")
        g = g.contiguous()
        self._bind_stream()
        check(lib.nfft3_grid_copy(self._h, _ptr(g), 1), "nfft3_grid_copy")


class GPE:
    """Strang splitting of the Gross-Pitaevskii equation (Sec. 3.1) on the
    regular grid of the periodic domain prod [a_d, b_d): state psi (N0, N1,
    N2) complex on the device; step(tau, n); coeffs() gives the trapezoidal
    coefficients of the state for Plan.infft3 / tube_refine."""

    def __init__(self, N: Sequence[int], a, b, dtype: torch.dtype = torch.complex128, device=None):
        if dtype not in _DT:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.N = tuple(int(v) for v in N)
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        A = (ctypes.c_double * 3)(*[float(v) for v in a])
        B = (ctypes.c_double * 3)(*[float(v) for v in b])
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(lib.nfft3_gpe_create(ctypes.byref(self._h), (ctypes.c_int64 * 3)(*self.N), A, B, _DT[dtype],
                                       ctypes.c_void_p(stream)), "nfft3_gpe_create")

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.nfft3_gpe_set_stream(self._h, ctypes.c_void_p(s)), "nfft3_gpe_set_stream")

    def _grid(self, t: torch.Tensor) -> torch.Tensor:
        if tuple(t.shape) != self.N or t.dtype != self.dtype or t.device != self.device:
            raise ValueError(f"state must be {self.N} {self.dtype} on {self.device}")
        return t.contiguous()

    def set_state(self, psi: torch.Tensor) -> None:
        psi = self._grid(psi)
        self._bind_stream()
        check(lib.nfft3_gpe_set_state(self._h, _ptr(psi)), "nfft3_gpe_set_state")
        torch.cuda.current_stream(self.device).synchronize()

    def state(self) -> torch.Tensor:
        out = torch.empty(self.N, dtype=self.dtype, device=self.device)
        self._bind_stream()
        check(lib.nfft3_gpe_get_state(self._h, _ptr(out)), "nfft3_gpe_get_state")
        return out

    def step(self, tau: float, nsteps: int = 1) -> None:
        self._bind_stream()
        check(lib.nfft3_gpe_step(self._h, float(tau), int(nsteps)), "nfft3_gpe_step")

    def coeffs(self) -> torch.Tensor:
        out = torch.empty(self.N, dtype=self.dtype, device=self.device)
        self._bind_stream()
        check(lib.nfft3_gpe_coeffs(self._h, _ptr(out)), "nfft3_gpe_coeffs")
        return out

    def close(self):
        if self._h:
            lib.nfft3_gpe_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class RectGrid:
    """The series at a rectilinear grid y0 x y1 x y2 (Sec. 2.1), exact up to
    rounding: F[i0, i1, i2] = sum_k fhat_k exp(-2 pi i (k0 y0[i0] + k1 y1[i1]
    + k2 y2[i2])), computed as three complex matrix products on the matrix
    cores.  N: coefficient sizes; M: grid points per axis (1, 2 or 3 axes:
    with two, the double matrix product of the paper's igridft2; with one,
    the matrix-vector product E psihat)."""

    def __init__(self, N: Sequence[int], M: Sequence[int], dtype: torch.dtype = torch.complex128, device=None):
        if dtype not in _DT:
            raise TypeError("dtype must be torch.complex64 or torch.complex128")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        if self.device.type != "cuda":
            raise ValueError("RectGrid needs a GPU device")
        self.N = tuple(int(v) for v in N)
        self.M = tuple(int(v) for v in M)
        self.dim = len(self.N)
        if self.dim not in (1, 2, 3) or len(self.M) != self.dim:
            raise ValueError("N and M must have the same length, 1, 2 or 3")
        self.dtype = dtype
        self._h = ctypes.c_void_p()
        pad = (1,) * (3 - self.dim)      # leading unit axes
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device).cuda_stream
            check(lib.nfft3_rgrid_plan(ctypes.byref(self._h), (ctypes.c_int64 * 3)(*(pad + self.N)),
                                       (ctypes.c_int64 * 3)(*(pad + self.M)), _DT[dtype], ctypes.c_void_p(stream)),
                  "nfft3_rgrid_plan")
        self._axes = None

    def _bind_stream(self):
        s = torch.cuda.current_stream(self.device).cuda_stream
        check(lib.nfft3_rgrid_set_stream(self._h, ctypes.c_void_p(s)), "nfft3_rgrid_set_stream")

    def set_axes(self, *ys: torch.Tensor) -> None:
        """Grid coordinates per axis: one float64 vector of M_d values on the
        device per axis."""
        if len(ys) != self.dim:
            raise ValueError(f"expected {self.dim} coordinate vectors")
        ys = list(ys)
        for d, y in enumerate(ys):
            if y.dtype != torch.float64 or y.device != self.device or y.numel() != self.M[d]:
                raise ValueError(f"y{d} must be {self.M[d]} float64 values on {self.device}")
            ys[d] = y.contiguous()
        ptrs = [ctypes.c_void_p()] * (3 - self.dim) + [_ptr(y) for y in ys]   # unit axes: NULL
        self._bind_stream()
        check(lib.nfft3_rgrid_set_axes(self._h, *ptrs), "nfft3_rgrid_set_axes")
        self._axes = ys

    def eval(self, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if tuple(fhat.shape) != self.N or fhat.dtype != self.dtype or fhat.device != self.device:
            raise ValueError(f"coefficients must be {self.N} {self.dtype} on {self.device}")
        fhat = fhat.contiguous()
        if out is None:
            out = torch.empty(self.M, dtype=self.dtype, device=self.device)
        elif tuple(out.shape) != self.M or out.dtype != self.dtype or out.device != self.device:
            raise ValueError(f"out must be {self.M} {self.dtype} on {self.device}")
        Plan._out(out)
        self._bind_stream()
        check(lib.nfft3_rgrid_eval(self._h, _ptr(fhat), _ptr(out)), "nfft3_rgrid_eval")
        return out

    def close(self):
        if self._h:
            lib.nfft3_rgrid_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_trafo(plans: Sequence[Plan], fhats: Sequence[torch.Tensor], deriv_mask: int = 0,
                out: Sequence[torch.Tensor] | None = None, allocate: bool = True, queue: bool = False):
    """Evaluate every plan's coefficients (and derivative fields) together:
    per stage one launch per transform length over all (plan, field) pairs
    of that length (the window sums: one launch).  Returns a list of
    (1 + popcount(mask), M_t) tensors (`out`, when given: contiguous tensors
    of those shapes).  allocate=False calls nfft3_batch_trafo_noalloc, which
    allocates no device memory (the plans must already hold their field
    grids); queue=True calls nfft3_batch_trafo_queue, the whole batch as one
    work-queue launch (same results)."""
    T = len(plans)
    if T != len(fhats):
        raise ValueError("one coefficient array per plan")
    k = 1 + bin(deriv_mask & 7).count("1")
    fh = [p._coeffs(f) for p, f in zip(plans, fhats)]
    if out is None:
        outs = [torch.empty((k, p.M), dtype=p.dtype, device=p.device) for p in plans]
    else:
        outs = list(out)
        if len(outs) != T:
            raise ValueError("one output tensor per plan")
        for p, o in zip(plans, outs):
            if tuple(o.shape) != (k, p.M) or o.dtype != p.dtype or o.device != p.device:
                raise ValueError(f"output must be ({k}, {p.M}) {p.dtype} on {p.device}")
            Plan._out(o)
    if T == 0:
        return outs
    plans[0]._bind_stream()
    H = (ctypes.c_void_p * T)(*[p._h.value for p in plans])
    F = (ctypes.c_void_p * T)(*[f.data_ptr() for f in fh])
    O = (ctypes.c_void_p * T)(*[o.data_ptr() for o in outs])
    if queue:
        if not allocate:
            raise ValueError("the work-queue form allocates its descriptor buffer")
        check(lib.nfft3_batch_trafo_queue(T, H, F, O, int(deriv_mask)), "nfft3_batch_trafo_queue")
    elif allocate:
        check(lib.nfft3_batch_trafo(T, H, F, O, int(deriv_mask)), "nfft3_batch_trafo")
    else:
        check(lib.nfft3_batch_trafo_noalloc(T, H, F, O, int(deriv_mask)), "nfft3_batch_trafo_noalloc")
    return outs


class _Type2(torch.autograd.Function):
    """f = A(x) fhat.  Backward: grad_fhat = A^H G (adjoint spreading),
    grad_x[j, d] = Re(conj(G_j) d f_j/d x_{j,d}) (window derivative)."""

    @staticmethod
    def forward(ctx, fhat, x, plan):
        # the sort is the precomputation: redo it only for new or modified points
        plan.set_points_if_changed(x.detach())
        ctx.plan = plan
        ctx.epoch = plan.epoch
        ctx.save_for_backward(fhat, x)
        return plan.trafo(fhat.detach())

    @staticmethod
    def backward(ctx, G):
        fhat, x = ctx.saved_tensors
        plan = ctx.plan
        if plan.epoch != ctx.epoch:      # points were replaced since forward
            plan.set_points(x.detach())
            ctx.epoch = plan.epoch
        G = G.contiguous()
        gf = plan.adjoint(G) if ctx.needs_input_grad[0] else None
        gx = plan.grad_points(fhat.detach(), G) if ctx.needs_input_grad[1] else None
        return gf, gx, None


def _infft_call(psihat: torch.Tensor, a, b, xi: torch.Tensor, dim: int, m: int, sigma: float) -> torch.Tensor:
    if psihat.dim() != dim:
        raise ValueError(f"coefficients must have {dim} axes")
    plan = Plan(tuple(psihat.shape), sigma=sigma, m=m, dtype=psihat.dtype, device=psihat.device)
    try:
        return plan.infft3(psihat, a, b, xi.reshape(-1, dim))
    finally:
        plan.close()


def infft(psihat: torch.Tensor, a: float, b: float, xi: torch.Tensor, m: int = 8, sigma: float = 2.0):
    """The one-dimensional series on [a, b) at the points xi (Appendix B's
    infft): psi(xi) = sum_k psihat_k exp(2 pi i k (xi - a)/(b - a)) / sqrt(b - a),
    k = -N/2 .. N/2-1.  Makes a plan for the call."""
    return _infft_call(psihat, [a], [b], xi, 1, m, sigma)


def infft2(psihat: torch.Tensor, a, b, xi: torch.Tensor, m: int = 8, sigma: float = 2.0):
    """The two-dimensional series on [a0, b0) x [a1, b1) at the (M, 2)
    points xi (Appendix B's infft2).  Makes a plan for the call."""
    return _infft_call(psihat, a, b, xi, 2, m, sigma)


def infft3(psihat: torch.Tensor, a, b, xi: torch.Tensor, m: int = 8, sigma: float = 2.0):
    """The three-dimensional series of eq. (fs) at the (M, 3) points xi.
    Makes a plan for the call (Plan.infft3 reuses one)."""
    return _infft_call(psihat, a, b, xi, 3, m, sigma)


def type2(fhat: torch.Tensor, x: torch.Tensor, plan: Plan) -> torch.Tensor:
    """Differentiable type-2 NFFT: f_j = sum_k fhat_k exp(-2 pi i k.x_j)."""
    return _Type2.apply(fhat, x, plan)


# -- host-only helpers (no GPU needed) ----------------------------------------

def deconv_factors(Nd: int, sigma: float, m: int):
    import numpy as np
    out = np.zeros(int(Nd), dtype=np.float64)
    check(lib.nfft3_deconv_factors(int(Nd), float(sigma), int(m),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "nfft3_deconv_factors")
    return out


def window_poly(m: int, sigma: float, dtype: torch.dtype = torch.complex128, cap_deg: int = 24):
    """(2m, deg+1) monomial coefficients in y = 2f - 1 of the window pieces."""
    import numpy as np
    buf = np.zeros(2 * int(m) * (cap_deg + 1), dtype=np.float64)
    deg = ctypes.c_int(0)
    check(lib.nfft3_window_poly(int(m), float(sigma), _DT[dtype], int(cap_deg),
                                buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(deg)),
          "nfft3_window_poly")
    d = deg.value
    return buf[: 2 * int(m) * (d + 1)].reshape(2 * int(m), d + 1)
