"""ctypes binding of libidw.so (argument marshalling only; every computation runs in the
library's HIP kernels).  The library is built in-tree by ``paper_1402_4986_amd.build``;
loading fails loudly when it is missing."""
from __future__ import annotations

import ctypes
import os
import threading

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libidw.so")

IDW_OK, IDW_EINVAL, IDW_EDEVICE, IDW_ENOMEM, IDW_EUNSUPPORTED, IDW_EWORKSPACE = range(6)
SOA, AOS, AOAS, HYBRID, SOAOS = range(5)
FP32, FP64, FP32_KAHAN = 0, 1, 2
EXCLUDE_SELF, NEED_DZ, NEED_DP, NEED_DQ, NEED_DX = 0x1, 0x2, 0x4, 0x8, 0x10

LAYOUT_CODES = {"soa": SOA, "aos": AOS, "aoas": AOAS, "hybrid": HYBRID, "soaos": SOAOS}
PRECISION_CODES = {"f32": FP32, "f64": FP64, "f32_kahan": FP32_KAHAN}

EXPORTED = ("idw_version", "idw_last_error", "idw_record_bytes", "idw_workspace_size",
            "idw_forward", "idw_backward", "idw_timing_enable", "idw_timing_read", "idw_batched_plan_create",
            "idw_batched_plan_workspace", "idw_batched", "idw_batched_plan_destroy", "idw_batched_plan_params",
            "idw_batched_defaults", "idw_forward_noalloc")
T_FWD_SWEEP, T_BWD_QUERY, T_BWD_DATA, T_BWD_FUSED = 0, 1, 2, 3


class IdwPoints(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p * 4), ("n", ctypes.c_int64), ("dim", ctypes.c_int32),
                ("layout", ctypes.c_int32)]


class IdwConfig(ctypes.Structure):
    _fields_ = [("queries_per_lane", ctypes.c_int32), ("split", ctypes.c_int32),
                ("batch_chunk", ctypes.c_int32), ("batch_workgroups", ctypes.c_int32),
                ("separate_adjoint", ctypes.c_int32), ("near_search", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 2)]


class IdwInstance(ctypes.Structure):
    _fields_ = [("data", IdwPoints), ("query", IdwPoints), ("p", ctypes.c_double),
                ("out_z", ctypes.c_void_p), ("out_den", ctypes.c_void_p)]


class IDWError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libidw status {code}: {msg}")
        self.code = code


_lock = threading.Lock()
_lib = None


def load(path: str | None = None):
    """Load libidw.so (once) and declare its prototypes.  Raises if it is not built."""
    global _lib
    with _lock:
        if _lib is not None and path is None:
            return _lib
        p = path or LIB_PATH
        if not os.path.exists(p):
            raise ImportError(f"{p} is not built: run `python -m paper_1402_4986_amd.build`")
        lib = ctypes.CDLL(p)
        P = ctypes.POINTER
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        lib.idw_version.restype = ctypes.c_char_p
        lib.idw_version.argtypes = []
        lib.idw_last_error.restype = ctypes.c_char_p
        lib.idw_last_error.argtypes = []
        lib.idw_record_bytes.restype = ctypes.c_int
        lib.idw_record_bytes.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P(sz)]
        lib.idw_workspace_size.restype = ctypes.c_int
        lib.idw_workspace_size.argtypes = [P(IdwPoints), P(IdwPoints), ctypes.c_int32, ctypes.c_uint32, P(IdwConfig),
                                           P(sz)]
        lib.idw_forward.restype = ctypes.c_int
        lib.idw_forward.argtypes = [P(IdwPoints), P(IdwPoints), ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                    vp, vp, vp, sz, vp, P(IdwConfig)]
        lib.idw_forward_noalloc.restype = ctypes.c_int
        lib.idw_forward_noalloc.argtypes = [P(IdwPoints), P(IdwPoints), ctypes.c_double, ctypes.c_int32,
                                            ctypes.c_uint32, vp, vp, vp, P(IdwConfig)]
        lib.idw_backward.restype = ctypes.c_int
        lib.idw_backward.argtypes = [P(IdwPoints), P(IdwPoints), ctypes.c_double, ctypes.c_int32, ctypes.c_uint32,
                                     vp, vp, vp, vp, vp, vp, vp, vp, sz, vp, P(IdwConfig)]
        lib.idw_timing_enable.restype = ctypes.c_int
        lib.idw_timing_enable.argtypes = [ctypes.c_int32]
        lib.idw_timing_read.restype = ctypes.c_int
        lib.idw_timing_read.argtypes = [ctypes.c_int32, P(ctypes.c_double), P(ctypes.c_int64)]
        lib.idw_batched_plan_create.restype = ctypes.c_int
        lib.idw_batched_plan_create.argtypes = [P(IdwInstance), ctypes.c_int32, ctypes.c_int32, P(IdwConfig),
                                                P(vp)]
        lib.idw_batched_plan_workspace.restype = ctypes.c_int
        lib.idw_batched_plan_workspace.argtypes = [vp, P(sz)]
        lib.idw_batched.restype = ctypes.c_int
        lib.idw_batched.argtypes = [vp, vp, sz, vp]
        lib.idw_batched_plan_destroy.restype = None
        lib.idw_batched_plan_destroy.argtypes = [vp]
        lib.idw_batched_plan_params.restype = ctypes.c_int
        lib.idw_batched_plan_params.argtypes = [vp, P(ctypes.c_int64), P(ctypes.c_int32)]
        lib.idw_batched_defaults.restype = ctypes.c_int
        lib.idw_batched_defaults.argtypes = [P(ctypes.c_int64), P(ctypes.c_int32)]
        if path is None:
            _lib = lib
        return lib


def check(code: int) -> None:
    if code != IDW_OK:
        raise IDWError(code, load().idw_last_error().decode(errors="replace"))
