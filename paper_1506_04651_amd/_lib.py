"""ctypes binding of librd (include/rd.h).  Argument marshalling only: every
step of the reaction substep runs in the library's HIP kernels.  If the
library has not been built, importing the functions below raises: there is
no CPU fallback."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librd.so")

OREGONATOR, KINETICS, NAGUMO, LINEAR, ROBERTSON, BYTECODE = 1, 2, 3, 4, 5, 6
JAC_ANALYTIC, JAC_FD = 0, 1
FP64, MIXED = 0, 1
PERSISTENT, ONE_LAUNCH = 0, 1
NSTATS = 9
STAT_NAMES = ("status", "nstep", "naccept", "nreject", "nfev", "njac", "ndec",
              "nsol", "nnewt")
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "ETOOBIG", -5: "ECLOSED",
          -6: "ENOTFOUND"}


class RdModel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("m", ctypes.c_int32),
                ("params", ctypes.POINTER(ctypes.c_double)), ("n_params", ctypes.c_int64)]


class RdOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("schedule", ctypes.c_int32),
                ("tol_transform", ctypes.c_int32), ("max_steps", ctypes.c_int32),
                ("newton_max", ctypes.c_int32), ("fixed_steps", ctypes.c_int32),
                ("h0", ctypes.c_double), ("h_min", ctypes.c_double),
                ("variant", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("order", ctypes.c_int32), ("jacobian", ctypes.c_int32),
                ("h_cells", ctypes.c_void_p), ("session_streams", ctypes.c_int32)]


class RdGrid(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("h", ctypes.c_double),
                ("diff", ctypes.POINTER(ctypes.c_double))]


class RdMraParams(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("levels", ctypes.c_int32), ("eps", ctypes.c_double),
                ("scale", ctypes.POINTER(ctypes.c_double)), ("refine", ctypes.c_int32)]


class RdRequestInfo(ctypes.Structure):
    _fields_ = [("done", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_failed", ctypes.c_int64), ("n_cells", ctypes.c_int64),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_done_ns", ctypes.c_uint64), ("batch_id", ctypes.c_int64),
                ("kernel_start_ms", ctypes.c_double), ("kernel_end_ms", ctypes.c_double),
                ("stream", ctypes.c_int32), ("deferred", ctypes.c_int32)]


# name -> (restype, argtypes); every symbol include/rd.h declares
SIGNATURES = {
    "rd_default_options": (None, [ctypes.POINTER(RdOptions)]),
    "rd_reaction_step": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                          ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                          ctypes.POINTER(RdModel)]),
    "rd_reaction_step_ex": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                             ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                             ctypes.POINTER(RdModel), ctypes.POINTER(RdOptions),
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32]),
    "rd_reaction_step_noalloc": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int64,
                                                  ctypes.c_int32, ctypes.c_double,
                                                  ctypes.c_double, ctypes.c_double,
                                                  ctypes.POINTER(RdModel),
                                                  ctypes.POINTER(RdOptions), ctypes.c_void_p,
                                                  ctypes.c_void_p, ctypes.c_int32]),
    "rd_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "rd_session_create": (ctypes.c_int32, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                           ctypes.c_size_t, ctypes.POINTER(RdOptions)]),
    "rd_submit": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.POINTER(RdModel), ctypes.c_void_p,
                                   ctypes.POINTER(ctypes.c_uint64)]),
    "rd_submit_ex": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.POINTER(RdModel), ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "rd_poll": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.POINTER(RdRequestInfo)]),
    "rd_wait": (ctypes.c_int32, [ctypes.c_void_p, ctypes.c_uint64,
                                 ctypes.POINTER(RdRequestInfo)]),
    "rd_request_bytes": (ctypes.c_size_t, [ctypes.c_int64, ctypes.c_int32, ctypes.c_int32]),
    "rd_session_destroy": (ctypes.c_int32, [ctypes.c_void_p]),
    "rd_last_error": (ctypes.c_char_p, []),
    "rd_variant_count": (ctypes.c_int32, [ctypes.c_int32] * 4),
    "rd_variant_name": (ctypes.c_char_p, [ctypes.c_int32] * 5),
    "rd_set_default_variant": (ctypes.c_int32, [ctypes.c_int32] * 5),
    "rd_variant_lanes": (ctypes.c_int32, [ctypes.c_int32] * 5),
    "rd_persistent_grid": (ctypes.c_int32, [ctypes.c_int32] * 4 + [ctypes.c_int64]),
    "rd_last_kernel_ms": (ctypes.c_double, []),
    "rd_diffusion_step": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int32,
                                           ctypes.POINTER(RdGrid), ctypes.c_double,
                                           ctypes.c_int32, ctypes.c_void_p]),
    "rd_mra_leaves": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(RdMraParams),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "rd_mra_reconstruct": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.POINTER(RdMraParams),
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "rd_mra_adapt": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.POINTER(RdMraParams),
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_int64), ctypes.c_void_p]),
    "rd_strang_step": (ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(RdGrid),
                                        ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                        ctypes.POINTER(RdModel), ctypes.POINTER(RdOptions),
                                        ctypes.c_void_p, ctypes.c_void_p]),
}

_lib = None


def load():
    """Load librd.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built: run `python -m paper_1506_04651_amd.build`"
                          " (the reaction step has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().rd_last_error().decode()


def default_options() -> RdOptions:
    o = RdOptions()
    load().rd_default_options(ctypes.byref(o))
    return o
