"""The forward entry point that allocates nothing (idw_forward_noalloc): its workspace is the
library's static device scratch.  Checked against idw_forward on the same inputs, bit for
bit (the same kernels and launch configuration), on two calls in a row, the second with
smaller inputs, so that what the first call left in the scratch cannot leak into the second;
sizes above the scratch are rejected."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, points, rand_case, scaled_err
from paper_1402_4986_amd import _lib, api

pytestmark = pytest.mark.gpu


def _noalloc(d, qq, p, prec, exclude_self=False):
    lib = _lib.load()
    m = qq.n
    Z = torch.empty(m, dtype=torch.float32 if prec != "f64" else torch.float64, device="cuda")
    D = torch.empty(m, dtype=torch.float64, device="cuda")
    dc, qc = d.c(), qq.c()
    flags = _lib.EXCLUDE_SELF if exclude_self else 0
    _lib.check(lib.idw_forward_noalloc(ctypes.byref(dc), ctypes.byref(qc), float(p), _lib.PRECISION_CODES[prec],
                                       flags, Z.data_ptr(), D.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream, None))
    return Z, D


@pytest.mark.parametrize("prec,p", [("f32", 2.0), ("f32", 8.0), ("f64", 1.7), ("f32_kahan", 2.5)])
def test_noalloc_forward_matches_idw_forward_twice(prec, p):
    for k, (n, m) in enumerate([(200000, 70000), (30000, 5000)]):
        x, z, q = rand_case(900 + k, n, m, 2, "f64" if prec == "f64" else "f32")
        q[:3] = x[:3]                              # exact hits: the FP64 fix-up uses the scratch too
        print(f"noalloc prec={prec} p={p} n={n} m={m}", flush=True)
        d, qq = points(x, z, q, "aoas", prec)
        Z0, D0 = api.forward(d, qq, p, prec)
        Z1, D1 = _noalloc(d, qq, p, prec)
        torch.cuda.synchronize()
        assert torch.equal(Z0, Z1)
        assert torch.equal(D0, D1)
        idx = np.arange(0, m, max(1, m // 300))
        ref = oracle.forward(x, z, q[idx], p)
        assert np.max(scaled_err(Z1.cpu().numpy().astype(np.float64)[idx], ref)) <= TOL[prec]


def test_noalloc_leave_one_out():
    x, z, _ = rand_case(910, 5000, 1, 2, "f32")
    d, qq = points(x, z, x, "hybrid", "f32")
    Z0, _ = api.forward(d, qq, 1.5, "f32", exclude_self=True)
    Z1, _ = _noalloc(d, qq, 1.5, "f32", exclude_self=True)
    torch.cuda.synchronize()
    assert torch.equal(Z0, Z1)
