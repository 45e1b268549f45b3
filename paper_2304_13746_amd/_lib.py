"""ctypes binding of libmhd.so (the C ABI in include/mhd.h).

Argument marshalling only: every step of the method runs in the HIP kernels of
libmhd.so.  Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# MHD_LIB selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MHD_LIB") or os.path.join(HERE, "libmhd.so")

MHD_OK = 0
MHD_ERR_INVALID_ARG = -1
MHD_ERR_WORKSPACE = -2
MHD_ERR_HIP = -3
MHD_ERR_NONPHYSICAL = -4
MHD_ERR_UNSUPPORTED = -5

MHD_FP64, MHD_FP32 = 0, 1
MHD_HLLD, MHD_HLL, MHD_HLLC = 0, 1, 2
MHD_EMF_EC, MHD_EMF_E0, MHD_EMF_ARITH, MHD_EMF_UCT_HLL, MHD_EMF_UCT_HLLD = 0, 1, 2, 3, 4
MHD_PLM, MHD_LIMO3, MHD_PPM = 0, 1, 2
MHD_CT_FACE, MHD_CT_VECPOT = 0, 1
MHD_RK2, MHD_EULER, MHD_RK3 = 0, 1, 2
TILE_16x16, TILE_24x8, TILE_18x11 = 1, 2, 3

EXPORTED = ("mhd_workspace_bytes", "mhd_create", "mhd_set_state", "mhd_step", "mhd_get_state",
            "mhd_get_stage_output", "mhd_get_diagnostics", "mhd_get_diagnostics_noalloc",
            "mhd_step_batch", "mhd_set_launch",
            "mhd_get_launch", "mhd_tune", "mhd_destroy", "mhd_status_string")


class Params(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("lx", C.c_double), ("ly", C.c_double), ("lz", C.c_double),
                ("gamma", C.c_double), ("cfl", C.c_double),
                ("precision", C.c_int), ("riemann", C.c_int), ("emf", C.c_int),
                ("integrator", C.c_int),
                ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
                ("stream", C.c_void_p), ("tile", C.c_int), ("zchunk", C.c_int),
                ("recon", C.c_int), ("ct", C.c_int), ("b0", C.c_double * 3)]


class StateView(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in ("rho", "mx", "my", "mz", "en", "bx", "by", "bz",
                                           "ax", "ay", "az")]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("mom", C.c_double * 3), ("energy", C.c_double),
                ("bflux", C.c_double * 3), ("divb_max", C.c_double), ("divb_rms", C.c_double),
                ("status", C.c_uint)]


class TuneResult(C.Structure):
    _fields_ = [("tile", C.c_int), ("zchunk_cap", C.c_int), ("best_ms", C.c_float),
                ("default_ms", C.c_float), ("candidates", C.c_int)]


class MHDError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {status_string(code)} ({code})")


_lib = None


def lib():
    """Load libmhd.so; raises if it is missing (build with __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python -m paper_2304_13746_amd.build")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.mhd_workspace_bytes.argtypes = [P(Params)]
        L.mhd_workspace_bytes.restype = C.c_size_t
        L.mhd_create.argtypes = [P(Params), P(C.c_void_p)]
        L.mhd_set_state.argtypes = [C.c_void_p, P(StateView), C.c_double, C.c_double]
        L.mhd_step.argtypes = [C.c_void_p, C.c_int, C.c_double]
        L.mhd_get_state.argtypes = [C.c_void_p, P(StateView), P(C.c_double), P(C.c_double)]
        L.mhd_get_stage_output.argtypes = [C.c_void_p, C.c_int, P(StateView)]
        L.mhd_get_diagnostics.argtypes = [C.c_void_p, P(Diag)]
        L.mhd_get_diagnostics_noalloc.argtypes = [C.c_void_p, P(Diag)]
        L.mhd_step_batch.argtypes = [P(C.c_void_p), P(C.c_int), C.c_int, C.c_void_p]
        L.mhd_set_launch.argtypes = [C.c_void_p, C.c_int, C.c_int]
        L.mhd_get_launch.argtypes = [C.c_void_p, P(C.c_int), P(C.c_int)]
        L.mhd_tune.argtypes = [P(C.c_void_p), C.c_int, C.c_int, C.c_void_p, P(TuneResult)]
        L.mhd_destroy.argtypes = [C.c_void_p]
        L.mhd_status_string.argtypes = [C.c_int]
        L.mhd_status_string.restype = C.c_char_p
        for name in EXPORTED:
            if name != "mhd_workspace_bytes" and name != "mhd_status_string":
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def status_string(code: int) -> str:
    try:
        return lib().mhd_status_string(int(code)).decode()
    except ImportError:
        return "libmhd not loaded"


def check(rc: int, what: str):
    if rc != MHD_OK:
        raise MHDError(rc, what)
    return rc
