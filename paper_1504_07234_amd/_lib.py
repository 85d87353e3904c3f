"""ctypes declarations of the C ABI in include/mlba.h.

Loading fails loudly when the library has not been built: there is no
fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmlba.so")

# status codes
OK, WARN_DIVERGED, EINVAL, EUNSUPPORTED, EHIP, ENOMEM = 0, 1, -1, -2, -3, -4
# boundary models / preconditioners / schedules
BC_RECT, BC_REFLECT, BC_PERIODIC, BC_ZERO, BC_ANTIREFLECT = 0, 1, 2, 3, 4
PRECOND_BCCB, PRECOND_DCT, PRECOND_NONE, PRECOND_AR = 0, 1, 2, 3
ALPHA_CONST, ALPHA_GEOMETRIC, ALPHA_TABLE, ALPHA_NS = 0, 1, 2, 3
METHOD_MLBA, METHOD_ALG4, METHOD_ALG2 = 0, 1, 2
BLUR_DIRECT, BLUR_FFT = 0, 1
STATE_EXPLICIT, STATE_IMPLICIT = 0, 1

c_int, c_double, c_size_t, c_void_p = ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_void_p
c_dbl_p = ctypes.POINTER(ctypes.c_double)
c_int_p = ctypes.POINTER(ctypes.c_int)


class AlphaSchedule(ctypes.Structure):
    _fields_ = [("kind", c_int), ("alpha0", c_double), ("ratio", c_double), ("alpha_floor", c_double),
                ("table", c_dbl_p), ("table_len", c_int), ("ns_q", c_double), ("ns_rho", c_double)]


class Stop(ctypes.Structure):
    _fields_ = [("noise_norm", c_double), ("gamma", c_double), ("check_every", c_int)]


class BatchTuning(ctypes.Structure):
    _fields_ = [("conv_rows", c_int * 2), ("fft_rows_cap", c_int), ("fft_cols_cap", c_int),
                ("conv_ms", (c_double * 2) * 2), ("rows_ms", c_double * 4), ("cols_ms", c_double * 6)]


class Params(ctypes.Structure):
    _fields_ = [("alpha", AlphaSchedule), ("mu", c_dbl_p), ("n_mu", c_int), ("delta", c_double),
                ("delta_table", c_dbl_p), ("iters", c_int), ("k0", c_int),
                ("stop", ctypes.POINTER(Stop)), ("state", c_int), ("method", c_int), ("alpha_out", c_dbl_p),
                ("pcg_max", c_int), ("pcg_tol", c_double), ("pcg_steps_out", c_int_p),
                ("delta_out", c_dbl_p), ("delta_table_len", c_int)]


# name -> (restype, argtypes); every symbol declared in include/mlba.h
SIGNATURES = {
    "mlba_status_string": (ctypes.c_char_p, [c_int]),
    "mlba_last_hip_error": (c_int, []),
    "mlba_version": (c_int, []),
    "mlba_plan_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int, c_int, c_int, c_int, c_void_p, c_void_p]),
    "mlba_plan_set_psf": (c_int, [c_void_p, c_void_p, c_void_p]),
    "mlba_plan_destroy": (c_int, [c_void_p]),
    "mlba_plan_set_blur": (c_int, [c_void_p, c_int, c_void_p]),
    "mlba_plan_autotune": (c_int, [c_void_p, c_int, c_dbl_p, c_void_p]),
    "mlba_plan_dims": (c_int, [c_void_p, c_int_p, c_int_p, c_int_p, c_int_p]),
    "mlba_plan_opnorm": (c_int, [c_void_p, c_double, c_int, c_dbl_p, c_void_p]),
    "mlba_apply_A": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlba_residual": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlba_apply_At": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlba_apply_P": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p]),
    "mlba_apply_CtP": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_void_p]),
    "mlba_framelet_analysis": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlba_analysis_update": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlba_framelet_synthesis": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "mlba_threshold_synthesis": (c_int, [c_void_p, c_void_p, c_dbl_p, c_int, c_double, c_void_p, c_void_p]),
    "mlba_shrink_synthesis": (c_int, [c_void_p, c_void_p, c_dbl_p, c_int, c_double, c_void_p, c_void_p]),
    "mlba_soft_threshold": (c_int, [c_void_p, c_void_p, c_int, c_size_t, c_dbl_p, c_int, c_double, c_void_p]),
    "mlba_apply_P_static": (c_int, [c_void_p, c_int, c_int, c_int, c_void_p, c_void_p, c_double, c_void_p]),
    "mlba_restore": (c_int, [c_void_p, c_void_p, ctypes.POINTER(Params), c_void_p, c_void_p, c_dbl_p, c_int_p,
                             c_void_p]),
    "mlba_batch_create": (c_int, [ctypes.POINTER(c_void_p), c_int, ctypes.POINTER(c_void_p), c_int, c_void_p]),
    "mlba_batch_destroy": (c_int, [c_void_p]),
    "mlba_batch_restore": (c_int, [c_void_p, ctypes.POINTER(c_void_p), c_dbl_p, c_dbl_p, c_int, c_dbl_p, c_int,
                                   ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_dbl_p, c_int, c_int,
                                   c_void_p]),
    "mlba_batch_autotune": (c_int, [c_void_p, c_int, ctypes.POINTER(BatchTuning), c_void_p]),
    "mlba_batch_set_tiles": (c_int, [c_void_p, ctypes.POINTER(BatchTuning), c_void_p]),
    "mlba_unrolled_create": (c_int, [ctypes.POINTER(c_void_p), c_int, ctypes.POINTER(c_void_p), c_int, c_int,
                                     c_void_p]),
    "mlba_unrolled_destroy": (c_int, [c_void_p]),
    "mlba_unrolled_dims": (c_int, [c_void_p, c_int_p, ctypes.POINTER(c_size_t)]),
    "mlba_unrolled_forward": (c_int, [c_void_p, ctypes.POINTER(c_void_p), c_double, c_dbl_p, c_int, c_double,
                                      ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_void_p]),
    "mlba_unrolled_backward": (c_int, [c_void_p, ctypes.POINTER(c_void_p), c_double, c_dbl_p, c_int, c_double,
                                       ctypes.POINTER(c_void_p), ctypes.POINTER(c_void_p), c_void_p, c_void_p,
                                       c_void_p, ctypes.POINTER(c_void_p), c_void_p]),
    "mlba_profile_begin": (c_int, [c_void_p, c_int]),
    "mlba_profile_end": (c_int, [c_void_p, c_dbl_p, c_int_p, c_int_p]),
    "mlba_profile_kernels": (c_int, [c_void_p, c_dbl_p, c_int_p]),
    "mlba_profile_every": (c_int, [c_void_p, c_int]),
}

PHASES = ("synthesis", "blur", "precond", "blur_t", "analysis")
# MLBA_KERNEL_* in order
KERNELS = ("synthesis_level", "lowpass_level", "shrink_synthesis", "conv_blur", "conv_blur_t", "fold_reflect",
           "reduce", "fft_rows_fwd", "fft_cols", "fft_rows_inv", "fc_rows_fwd", "fc_cols", "fc_rows_inv",
           "fc_residual_precond_rows", "precond_rows_fc_fwd", "analysis_level", "other")

_lib = None


def load() -> ctypes.CDLL:
    """Load libmlba.so and declare every entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1504_07234_amd.build` "
                           "(or __graft_entry__.build()); there is no fallback implementation")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class MLBAError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.mlba_status_string(status).decode()
        if status == EHIP:
            msg += f" (hipError {lib.mlba_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")
        self.status = status


def check(status: int, where: str) -> int:
    if status < 0:
        raise MLBAError(status, where)
    return status
