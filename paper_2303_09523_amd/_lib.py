"""ctypes binding of libokrig.so (the C ABI declared in include/okrig.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# OKRIG_LIB names another build of the same library (the host-sanitizer test
# loads an instrumented one); there is no other library and no fallback.
LIB_PATH = os.environ.get("OKRIG_LIB") or os.path.join(HERE, "libokrig.so")

OKR_OK = 0
STATUS_NAMES = {0: "OKR_OK", 1: "OKR_E_INVALID_ARG", 2: "OKR_E_SHAPE", 3: "OKR_E_NONFINITE",
                4: "OKR_E_DEVICE", 5: "OKR_E_OOM", 6: "OKR_E_UNSUPPORTED",
                7: "OKR_E_NOT_CONVERGED", 8: "OKR_E_CAPACITY"}
MODELS = {"spherical": 0, "exponential": 1, "gaussian": 2}
PHASES = ["place", "tables", "select", "bucket", "solve", "fallback", "plain", "loso", "pattern",
          "mesh", "edge_shear", "edge_thin", "edge_trace"]
PRECISIONS = {"fp32": 0, "mixed_fp16": 1, "mixed_bf16": 2, "fp64": 3}
ALGOS = {"batched": 0, "plain": 1, "pattern": 2}

EXPORTED = ["okr_plan_create", "okr_execute", "okr_select", "okr_loso_forward",
            "okr_loso_backward", "okr_stats_get", "okr_plan_destroy", "okr_status_string",
            "okr_plan_last_error", "okr_version", "okr_abi_sizes", "okr_plan_set_profiling",
            "okr_plan_set_graph", "okr_plan_autotune", "okr_plan_get_tuning",
            "okr_krige_points", "okr_marching_cubes", "okr_execute_noalloc",
            "okr_edge_postpass", "okr_edge_filters"]


class Variogram(C.Structure):
    _fields_ = [("model", C.c_int32), ("nugget", C.c_double), ("sill", C.c_double),
                ("range", C.c_double)]


class Problem(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nslices", C.c_int32),
                ("upsample", C.c_int32), ("radius", C.c_int32), ("min_points", C.c_int32),
                ("precision", C.c_int32), ("algo", C.c_int32), ("refine_tol", C.c_double),
                ("refine_max", C.c_int32), ("strict", C.c_int32), ("drift", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_systems", C.c_int64), ("n_kriged", C.c_int64), ("bucket", C.c_int64 * 128),
                ("n_floor_filled", C.c_int64), ("n_refined", C.c_int64),
                ("n_fp64_fallback", C.c_int64), ("n_nonpositive_pivot", C.c_int64),
                ("max_kappa_est", C.c_double), ("phase_ms", C.c_double * 13),
                ("phase_calls", C.c_int64 * 13), ("n_not_converged", C.c_int64),
                ("n_refine_unconverged", C.c_int64), ("kappa_window", C.c_double),
                ("direct_fp64", C.c_int32)]


class OkrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    """Load libokrig.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run paper_2303_09523_amd.build.build() "
                          "(hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    P, VP = C.POINTER, C.c_void_p
    sig = {
        "okr_plan_create": (C.c_int32, [P(Problem), VP, P(VP)]),
        "okr_execute": (C.c_int32, [VP, P(Variogram), VP, VP, VP, VP, VP]),
        "okr_select": (C.c_int32, [VP, VP, VP, VP]),
        "okr_loso_forward": (C.c_int32, [VP, P(Variogram), VP, VP, VP]),
        "okr_loso_backward": (C.c_int32, [VP, VP]),
        "okr_stats_get": (C.c_int32, [VP, P(Stats)]),
        "okr_plan_destroy": (C.c_int32, [VP]),
        "okr_status_string": (C.c_char_p, [C.c_int32]),
        "okr_plan_last_error": (C.c_char_p, [VP]),
        "okr_version": (C.c_int32, []),
        "okr_abi_sizes": (C.c_int32, [P(C.c_int64)]),
        "okr_plan_set_profiling": (C.c_int32, [VP, C.c_int32]),
        "okr_plan_set_graph": (C.c_int32, [VP, C.c_int32]),
        "okr_krige_points": (C.c_int32, [VP, P(Variogram), C.c_int64, VP, VP, VP, VP, VP, VP,
                                         VP, VP]),
        "okr_plan_autotune": (C.c_int32, [VP, P(Variogram), VP, VP, VP, VP]),
        "okr_marching_cubes": (C.c_int32, [VP, VP, C.c_float, VP, VP, C.c_int64,
                                           P(C.c_int64)]),
        "okr_plan_get_tuning": (C.c_int32, [VP, P(C.c_int32), P(C.c_int32), P(C.c_double),
                                            P(C.c_int32)]),
        "okr_execute_noalloc": (C.c_int32, [P(Problem), VP, P(Variogram), VP, VP, VP, VP, VP,
                                            VP]),
        "okr_edge_postpass": (C.c_int32, [VP, VP, VP, C.c_double, VP, VP, VP]),
        "okr_edge_filters": (C.c_int32, [VP, VP]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    sizes = (C.c_int64 * 3)()
    if lib.okr_abi_sizes(sizes) != OKR_OK or list(sizes) != [C.sizeof(Problem), C.sizeof(Variogram),
                                                            C.sizeof(Stats)]:
        raise ImportError(f"okrig ABI mismatch: library {list(sizes)} vs binding "
                          f"{[C.sizeof(Problem), C.sizeof(Variogram), C.sizeof(Stats)]}")
    _lib = lib
    return lib


def check(status: int, plan=None):
    if status != OKR_OK:
        lib = load()
        msg = lib.okr_plan_last_error(plan).decode() if plan else \
            lib.okr_status_string(status).decode()
        raise OkrError(status, msg)
