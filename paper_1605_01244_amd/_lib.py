"""ctypes loader for libnfft3.so (the C ABI declared in include/nfft3.h).

The library is built in-tree by ``python paper_1605_01244_amd/csrc/build.py``.
There is no fallback: if the shared library is missing or does not load,
importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libnfft3.so")

NFFT3_C64 = 0
NFFT3_C128 = 1

STATUS = {
    0: "NFFT3_OK",
    -1: "NFFT3_ERR_INVALID_ARG",
    -2: "NFFT3_ERR_DTYPE",
    -3: "NFFT3_ERR_OOM",
    -4: "NFFT3_ERR_NO_POINTS",
    -5: "NFFT3_ERR_NONFINITE",
    -6: "NFFT3_ERR_HIP",
    -7: "NFFT3_ERR_NULL",
    -8: "NFFT3_ERR_CAPACITY",
    -9: "NFFT3_ERR_TIMEOUT",
}


class NFFT3Error(RuntimeError):
    def __init__(self, code: int, where: str, detail: str = ""):
        self.code = code
        name = STATUS.get(code, str(code))
        msg = f"{where}: {name}"
        if detail:
            msg += f" ({detail})"
        super().__init__(msg)


def _load() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1605_01244_amd/csrc/build.py`")
    lib = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    i64p = ctypes.POINTER(ctypes.c_int64)
    dp = ctypes.POINTER(ctypes.c_double)
    ci = ctypes.c_int
    sig = {
        "nfft3_plan": ([ctypes.POINTER(vp), i64p, ctypes.c_double, ci, ci, vp], ci),
        "nfft3_plan_nd": ([ctypes.POINTER(vp), ci, i64p, ctypes.c_double, ci, ci, vp], ci),
        "nfft3_set_stream": ([vp, vp], ci),
        "nfft3_set_points": ([vp, i64, vp], ci),
        "nfft3_points_unchanged": ([vp, i64, vp, ctypes.POINTER(ci)], ci),
        "nfft3_trafo": ([vp, vp, vp], ci),
        "nfft3_adjoint": ([vp, vp, vp], ci),
        "nfft3_grad_points": ([vp, vp, vp, vp], ci),
        "nfft3_trafo_fields": ([vp, vp, vp, ci], ci),
        "nfft3_batch_trafo": ([ci, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ci], ci),
        "nfft3_batch_trafo_noalloc": ([ci, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ci], ci),
        "nfft3_batch_trafo_queue": ([ci, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), ci], ci),
        "nfft3_infft3": ([vp, dp, dp, vp, i64, vp, vp], ci),
        "nfft3_tube_refine": ([vp, dp, dp, vp, ci, dp, i64, vp, vp, i64p], ci),
        "nfft3_gpe_create": ([ctypes.POINTER(vp), i64p, dp, dp, ci, vp], ci),
        "nfft3_gpe_set_stream": ([vp, vp], ci),
        "nfft3_gpe_set_state": ([vp, vp], ci),
        "nfft3_gpe_get_state": ([vp, vp], ci),
        "nfft3_gpe_step": ([vp, ctypes.c_double, ci], ci),
        "nfft3_gpe_coeffs": ([vp, vp], ci),
        "nfft3_gpe_destroy": ([vp], ci),
        "nfft3_rgrid_plan": ([ctypes.POINTER(vp), i64p, i64p, ci, vp], ci),
        "nfft3_rgrid_set_stream": ([vp, vp], ci),
        "nfft3_rgrid_set_axes": ([vp, vp, vp, vp], ci),
        "nfft3_rgrid_eval": ([vp, vp, vp], ci),
        "nfft3_rgrid_destroy": ([vp], ci),
        "nfft3_set_tuning": ([vp, ci, ci], ci),
        "nfft3_get_tuning": ([vp, ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
        "nfft3_autotune": ([vp, i64, vp, vp, vp, ci, ctypes.POINTER(ci), ctypes.POINTER(ci)], ci),
        "nfft3_destroy": ([vp], ci),
        "nfft3_strerror": ([ci], ctypes.c_char_p),
        "nfft3_last_hip_error": ([], ctypes.c_char_p),
        "nfft3_get_info": ([vp, i64p, i64p], ci),
        "nfft3_stage_grid": ([vp, vp, ci], ci),
        "nfft3_stage_interp": ([vp, vp], ci),
        "nfft3_stage_spread": ([vp, vp], ci),
        "nfft3_grid_copy": ([vp, vp, ci], ci),
        "nfft3_deconv_factors": ([i64, ctypes.c_double, ci, dp], ci),
        "nfft3_window_poly": ([ci, ctypes.c_double, ci, ci, dp, ctypes.POINTER(ci)], ci),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


lib = _load()


def check(code: int, where: str) -> None:
    if code != 0:
        detail = ""
        if code == -6:
            detail = lib.nfft3_last_hip_error().decode(errors="replace")
        raise NFFT3Error(code, where, detail)
