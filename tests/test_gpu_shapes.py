"""Launch shapes against the oracle: sizes chosen around the decompositions the library picks.

The forward cuts the data into chunks (at least 4 tiles of 512 points, or 1 tile where 4
would leave fewer than 2048 workgroups) for about 16384 workgroups; the fused adjoint cuts it
into ranges of at most 32K points (at least one tile) for about 8192 workgroups over
1,024-query blocks (512 in FP64).  These cases put the last chunk or range down to a few
points, give many ranges to a single query block, sit just
above and below the 32K range size and the 65,536-point grid threshold, and hand the fused
adjoint one-point and one-tile data sets.  Forward, and adjoint (dz, dp, dq, and dx for the
fused FP32 sweep), against the FP64 oracle at the usual tolerances.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, TOL, dp_errors, dq_errors, points, rand_case, scaled_err
from paper_1402_4986_amd import api

pytestmark = pytest.mark.gpu

SHAPES = [
    (1, 700),        # one data point: one range of one point
    (513, 1),        # one query: one block, ranges of a tile and one point
    (2049, 3001),    # last forward chunk of one point
    (32767, 300),    # just below the 32K range size
    (33000, 700),    # 65 one-tile ranges, the last of 232 points
    (65537, 260),    # grid threshold, ragged everything
]


def _tol_checks(prec, x, z, q, p, Z, dz, dp, dq, dx, g):
    ref = oracle.forward(x, z, q, p)
    assert np.max(scaled_err(Z, ref)) <= TOL[prec]
    refb = oracle.backward(x, z, q, p, g)
    tol = GTOL[prec]
    e = np.abs(dz - refb["dz"]) / np.maximum(refb["dz_scale"], 1e-300)
    assert np.max(e) <= tol, f"dz err {np.max(e):.3e}"
    ec, es = dp_errors(dp, refb)
    assert ec <= tol and es <= tol, (dp, refb["dp"])
    ec, es = dq_errors(dq, refb)
    assert np.max(ec) <= tol and (es.size == 0 or np.max(es) <= tol)
    if dx is not None:
        refx = oracle.backward_x(x, z, q, p, g)
        ex = np.max(np.abs(dx - refx["dx"]), axis=1) / np.maximum(refx["dx_cond"], 1e-300)
        assert np.max(ex) <= tol, f"dx err {np.max(ex):.3e}"


@pytest.mark.parametrize("n,m", SHAPES)
@pytest.mark.parametrize("prec,dim,p", [("f32", 2, 2.0), ("f32", 3, 1.5), ("f32", 2, 8.0), ("f64", 2, 2.0),
                                        ("f64", 3, 1.7)])
def test_awkward_sizes_match_oracle(n, m, prec, dim, p):
    x, z, q = rand_case(700 + n % 97 + m % 89, n, m, dim, prec)
    g = np.random.default_rng(n + m).normal(size=m)
    t = np.float32 if prec == "f32" else np.float64
    g = g.astype(t).astype(np.float64)
    print(f"shape n={n} m={m} prec={prec} dim={dim} p={p}", flush=True)
    d, qq = points(x, z, q, "aoas", prec)
    Zt, Dt = api.forward(d, qq, p, prec)
    gt = torch.tensor(g, dtype=torch.float32 if prec == "f32" else torch.float64, device="cuda")
    need_dx = prec == "f32" and p < 6
    r = api.backward(d, qq, p, gt, Zt, Dt, prec, need_dx=need_dx)
    torch.cuda.synchronize()
    cv = lambda a: a.cpu().numpy().astype(np.float64)
    dx = cv(r[3]) if need_dx else None
    _tol_checks(prec, x, z, q, p, cv(Zt), cv(r[0]), float(r[1]), cv(r[2]), dx, g)
