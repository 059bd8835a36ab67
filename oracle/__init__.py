"""FP64 CPU oracle for Shepard IDW (Section 2.1, Eq. 1).

TEST INFRASTRUCTURE ONLY: the test-suite, the smoke check and the CPU-baseline leg of
the benchmark may import this package; the product library never does.  It shares no
code with the HIP path: the arithmetic lives in ``idw_oracle.c`` (plain single-threaded
FP64 loops) and in ``exact.py`` (exact / 60-digit brute force for tiny inputs).

Parity pins (each listed with its test in ``tests/test_oracle_*.py``): constant and
linear fields on symmetric stencils, exact-hit reproduction, weights summing to one, the
two-point closed form, the p -> 0 and large-p limits, permutation invariance, exact
rational / 60-digit brute force on 8-point inputs, high-precision finite differences
of the forward for every gradient, and leave-one-out against explicit deletion.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "idw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2, no fast-math, no OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load_library(path: str):
    """Loads an oracle library built from idw_oracle.c (or, in the mutation tests, from a
    copy of it with a planted mistake) and declares its prototypes."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int64)
    lib.idw_oracle_forward.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, ctypes.c_int64, dp,
                                       ctypes.c_double, ip, dp, dp, dp, ip]
    lib.idw_oracle_forward.restype = ctypes.c_int
    lib.idw_oracle_backward.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, ctypes.c_int64, dp,
                                        ctypes.c_double, ip, dp, dp, dp, dp, dp, dp, dp, dp, dp]
    lib.idw_oracle_backward.restype = ctypes.c_int
    lib.idw_oracle_backward_x.argtypes = [ctypes.c_int64, ctypes.c_int, dp, dp, ctypes.c_int64, dp,
                                          ctypes.c_double, ip, dp, dp, dp]
    lib.idw_oracle_backward_x.restype = ctypes.c_int
    return lib


def compile_source(src: str, out: str) -> str:
    """Builds a shared library from a C source file with the oracle's flags."""
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", out, src, "-lm"])
    return out


def _load(lib=None):
    global _lib
    if lib is not None:
        return lib
    with _lock:
        if _lib is None:
            build()
            _lib = load_library(_LIB_PATH)
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if a is not None else None


def _prep(x, z, q, self_index):
    x = np.ascontiguousarray(x, dtype=np.float64)
    z = np.ascontiguousarray(z, dtype=np.float64).reshape(-1)
    q = np.ascontiguousarray(q, dtype=np.float64)
    if x.ndim != 2 or q.ndim != 2 or x.shape[1] != q.shape[1] or x.shape[0] != z.shape[0]:
        raise ValueError("oracle: x [n,dim], z [n], q [m,dim] expected")
    si = None
    if self_index is not None:
        si = np.ascontiguousarray(self_index, dtype=np.int64).reshape(-1)
        if si.shape[0] != q.shape[0]:
            raise ValueError("oracle: self_index must have one entry per query")
    return x, z, q, si


def forward(x, z, q, p, self_index=None, lib=None):
    """Eq. 1 over every data point.  Returns dict(Z, D, S, H) of numpy arrays.

    x: [n, dim] data coordinates, z: [n] data values, q: [m, dim] queries, p > 0.
    self_index: optional [m] data index left out per query (leave-one-out).
    lib: an alternative library from load_library (default: the built oracle).
    """
    lib = _load(lib)
    x, z, q, si = _prep(x, z, q, self_index)
    m = q.shape[0]
    Z = np.empty(m)
    D = np.empty(m)
    S = np.empty(m)
    H = np.empty(m, dtype=np.int64)
    rc = lib.idw_oracle_forward(x.shape[0], x.shape[1], _d(x), _d(z), m, _d(q), float(p), _i(si),
                                _d(Z), _d(D), _d(S), _i(H))
    if rc != 0:
        raise ValueError("oracle forward: invalid arguments")
    return {"Z": Z, "D": D, "S": S, "H": H}


def backward(x, z, q, p, g, self_index=None, lib=None):
    """Analytic adjoint of Eq. 1.

    Returns dict(dz, dp, dq, dz_scale, dp_scale, dq_scale, dp_cond, dq_cond): the *_scale
    entries are the sums of absolute terms; dp_cond / dq_cond the uncentred sums that
    measure how far a relative perturbation of the values moves dp / dq.
    """
    lib = _load(lib)
    x, z, q, si = _prep(x, z, q, self_index)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    n, dim = x.shape
    m = q.shape[0]
    if g.shape[0] != m:
        raise ValueError("oracle backward: g must be [m]")
    dz = np.empty(n)
    dzs = np.empty(n)
    dp = np.empty(1)
    dps = np.empty(1)
    dq = np.empty((m, dim))
    dqs = np.empty(m)
    dpc = np.empty(1)
    dqc = np.empty(m)
    rc = lib.idw_oracle_backward(n, dim, _d(x), _d(z), m, _d(q), float(p), _i(si), _d(g), _d(dz), _d(dp),
                                 _d(dq), _d(dzs), _d(dps), _d(dqs), _d(dpc), _d(dqc))
    if rc != 0:
        raise ValueError("oracle backward: invalid arguments")
    return {"dz": dz, "dp": float(dp[0]), "dq": dq, "dz_scale": dzs, "dp_scale": float(dps[0]),
            "dq_scale": dqs, "dp_cond": float(dpc[0]), "dq_cond": dqc}


def backward_x(x, z, q, p, g, self_index=None, lib=None):
    """Adjoint with respect to the data coordinates: dict(dx [n, dim], dx_cond [n]).

    dx_cond is the uncentred sum (|z_j| + |Z_i| in place of z_j - Z_i) that bounds how far
    a relative perturbation of the values moves each row of dx.
    """
    lib = _load(lib)
    x, z, q, si = _prep(x, z, q, self_index)
    g = np.ascontiguousarray(g, dtype=np.float64).reshape(-1)
    n, dim = x.shape
    if g.shape[0] != q.shape[0]:
        raise ValueError("oracle backward_x: g must be [m]")
    dx = np.empty((n, dim))
    dxc = np.empty(n)
    rc = lib.idw_oracle_backward_x(n, dim, _d(x), _d(z), q.shape[0], _d(q), float(p), _i(si), _d(g),
                                   _d(dx), _d(dxc))
    if rc != 0:
        raise ValueError("oracle backward_x: invalid arguments")
    return {"dx": dx, "dx_cond": dxc}


def loo_loss(x, z, p, idx=None):
    """Leave-one-out mean squared error of Eq. 1 at the data points listed in idx."""
    x = np.asarray(x, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    idx = np.arange(x.shape[0]) if idx is None else np.asarray(idx, dtype=np.int64)
    r = forward(x, z, x[idx], p, self_index=idx)
    return float(np.mean((r["Z"] - z[idx]) ** 2))
