"""The forward entry point that allocates nothing (idw_forward_noalloc): its workspace is the
library's static device scratch.  Checked against idw_forward on the same inputs on two calls
in a row, the second with smaller inputs, so that what the first call left in the scratch
cannot leak into the second:
  * with a data split given in the configuration, bit for bit (the same kernels and launch);
  * with the default configuration, where the first size's default split would need more
    partial sums than the scratch holds and the entry point takes a smaller one, within the
    FP32 / FP64 tolerance of idw_forward and of the oracle;
sizes above the scratch are rejected."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import TOL, points, rand_case, scaled_err
from paper_1402_4986_amd import _lib, api

pytestmark = pytest.mark.gpu

SCRATCH = 64 << 20


def _noalloc(d, qq, p, prec, exclude_self=False, split=0):
    lib = _lib.load()
    m = qq.n
    Z = torch.empty(m, dtype=torch.float32 if prec != "f64" else torch.float64, device="cuda")
    D = torch.empty(m, dtype=torch.float64, device="cuda")
    dc, qc = d.c(), qq.c()
    flags = _lib.EXCLUDE_SELF if exclude_self else 0
    cfg = _lib.IdwConfig()
    cfg.split = split
    _lib.check(lib.idw_forward_noalloc(ctypes.byref(dc), ctypes.byref(qc), float(p), _lib.PRECISION_CODES[prec],
                                       flags, Z.data_ptr(), D.data_ptr(),
                                       torch.cuda.current_stream().cuda_stream, ctypes.byref(cfg)))
    return Z, D


def _fwd_bytes(d, qq, prec, split=0):
    lib = _lib.load()
    dc, qc = d.c(), qq.c()
    cfg = _lib.IdwConfig()
    cfg.split = split
    b = ctypes.c_size_t()
    _lib.check(lib.idw_workspace_size(ctypes.byref(dc), ctypes.byref(qc), _lib.PRECISION_CODES[prec], 0,
                                      ctypes.byref(cfg), ctypes.byref(b)))
    return b.value


@pytest.mark.parametrize("prec,p", [("f32", 2.0), ("f32", 8.0), ("f64", 1.7), ("f32_kahan", 2.5)])
def test_noalloc_forward_matches_idw_forward_twice(prec, p):
    tol = TOL["f64" if prec == "f64" else "f32"]
    for k, (n, m) in enumerate([(200000, 70000), (30000, 5000)]):
        x, z, q = rand_case(900 + k, n, m, 2, "f64" if prec == "f64" else "f32")
        q[:3] = x[:3]                              # exact hits: the FP64 fix-up uses the scratch too
        d, qq = points(x, z, q, "aoas", prec)
        if k == 0:
            # the default split's partials exceed the scratch here: the entry point splits less
            assert _fwd_bytes(d, qq, prec) > SCRATCH and _fwd_bytes(d, qq, prec, split=4) <= SCRATCH
        print(f"noalloc prec={prec} p={p} n={n} m={m}, split 4", flush=True)
        Z0, D0 = api.forward(d, qq, p, prec, split=4)
        Z1, D1 = _noalloc(d, qq, p, prec, split=4)
        torch.cuda.synchronize()
        assert torch.equal(Z0, Z1)
        assert torch.equal(D0, D1)
        print(f"noalloc prec={prec} p={p} n={n} m={m}, default split", flush=True)
        Z0, D0 = api.forward(d, qq, p, prec)
        Z1, D1 = _noalloc(d, qq, p, prec)
        torch.cuda.synchronize()
        z0, z1 = Z0.cpu().numpy().astype(np.float64), Z1.cpu().numpy().astype(np.float64)
        # both within tol S of Eq. 1, and S <= max|z|
        assert np.max(np.abs(z1 - z0)) <= 2 * tol * np.max(np.abs(z))
        np.testing.assert_array_equal(z1[:3], z0[:3])
        d0, d1 = D0.cpu().numpy(), D1.cpu().numpy()
        fin = np.isfinite(d0)
        assert np.array_equal(fin, np.isfinite(d1))
        np.testing.assert_allclose(d1[fin], d0[fin], rtol=2 * tol)
        idx = np.arange(0, m, max(1, m // 300))
        ref = oracle.forward(x, z, q[idx], p)
        assert np.max(scaled_err(z1[idx], ref)) <= tol


def test_noalloc_leave_one_out():
    x, z, _ = rand_case(910, 5000, 1, 2, "f32")
    d, qq = points(x, z, x, "hybrid", "f32")
    Z0, _ = api.forward(d, qq, 1.5, "f32", exclude_self=True)
    Z1, _ = _noalloc(d, qq, 1.5, "f32", exclude_self=True)
    torch.cuda.synchronize()
    assert torch.equal(Z0, Z1)
