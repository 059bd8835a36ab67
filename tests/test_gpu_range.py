"""GPU parity at the edges of the floating-point range: large exponents p and large |values|.

Eq. 1 is scale-free in the weights, but the FP32 sweeps hold raw weights and weighted sums.
For large p a nearby point's weight (d^-p) exceeds the FP32 range, and for large |z| the
weighted sums do; then the threshold (1e-6 extent)^-p itself can exceed the FP64 range.
Such queries must be routed to the FP64 recomputation, in the forward and in the adjoint,
and agree with the FP64 oracle like any other query.  Every case asserts first that the
oracle's own result is finite, so that the comparison is meaningful.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, TOL, gpu_forward, points, rand_case, scaled_err
from paper_1402_4986_amd import api, batched, workloads

pytestmark = pytest.mark.gpu


def _backward(x, z, q, p, layout, prec, g):
    d, qq = points(x, z, q, layout, prec)
    Z, D = api.forward(d, qq, p, prec)
    t = torch.float32 if prec == "f32" else torch.float64
    dz, dp, dq = api.backward(d, qq, p, torch.as_tensor(g, dtype=t, device="cuda"), Z, D, prec)
    torch.cuda.synchronize()
    return dz.cpu().numpy().astype(np.float64), float(dp), dq.cpu().numpy().astype(np.float64)


# At large p most weight ratios w_ij / D_i are far below FLT_MIN, and so are many dz_j:
# an FP32 output can only hold such a value to the subnormal spacing 2^-149, which is
# added to the FP32 bound as an absolute floor (dp is returned in FP64).  From p = 6 on the
# FP32 adjoint uses relative weights, in which a weight below FLT_MIN of its query's scale
# may be flushed to zero: each query then moves a dz_j by at most |g_i| 2^-126 (its
# relative denominator is at least 1), so the FP32 floor grows by 2^-126 sum |g|.
FLOOR = {"f32": 2.0 ** -149, "f64": 0.0}


def _floor(prec, g, p):
    rel = prec == "f32" and p >= 6.0
    return FLOOR[prec] + (2.0 ** -126 * float(np.sum(np.abs(g))) if rel else 0.0)


def _check_grad(got, ref, prec, g, p):
    dz, dp, dq = got
    tol, fl = GTOL[prec], _floor(prec, g, p)
    assert np.all(np.isfinite(dz)) and np.isfinite(dp) and np.all(np.isfinite(dq))
    e = np.abs(dz - ref["dz"]) - tol * ref["dz_scale"]
    assert np.max(e) <= fl, f"dz err {np.max(e):.3e} above the bound"
    assert abs(dp - ref["dp"]) <= tol * ref["dp_cond"], f"dp {dp} vs {ref['dp']}"
    e = np.max(np.abs(dq - ref["dq"]), axis=1) - tol * ref["dq_cond"]
    assert np.max(e) <= fl, f"dq err {np.max(e):.3e} above the bound"


def _case(seed, prec, zscale=1.0):
    x, z, q = rand_case(seed, 3000, 1000, 2, prec)
    q[:8] = x[:8]                                   # exact hits
    t = np.float32 if prec == "f32" else np.float64
    z = (z * zscale).astype(t).astype(np.float64)
    g = np.random.default_rng(seed + 1).normal(size=len(q)).astype(t).astype(np.float64)
    return x, z, q, g


# p = 56: (1e-6 extent)^-p is beyond the FP64 range and every FP32 weight of a point
# closer than about 0.2 of the extent overflows; the FP64 weights of this case stay finite.
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("p", [12.0, 56.0])
def test_large_exponent_forward_and_adjoint(prec, p):
    x, z, q, g = _case(61, prec)
    print(f"case prec={prec} p={p}", flush=True)
    ref = oracle.forward(x, z, q, p)
    assert np.all(np.isfinite(ref["Z"])) and np.all(np.isfinite(ref["D"][8:]))
    for layout in ("aoas", "soa"):
        Z, _ = gpu_forward(x, z, q, p, layout, prec)
        assert np.all(np.isfinite(Z))
        assert np.max(scaled_err(Z, ref)) <= TOL[prec]
        assert np.array_equal(Z[:8], ref["Z"][:8])
    gref = oracle.backward(x, z, q, p, g)
    _check_grad(_backward(x, z, q, p, "hybrid", prec, g), gref, prec, g, p)


# |z| up to about 3e20 and 3e34: the FP32 weighted sums of a query near a data point
# exceed the FP32 range unless the query is recomputed in FP64.
@pytest.mark.parametrize("zscale", [1e20, 1e34])
@pytest.mark.parametrize("p", [2.0, 3.0])
def test_large_values_forward_and_adjoint(zscale, p):
    x, z, q, g = _case(62, "f32", zscale)
    print(f"case zscale={zscale:g} p={p}", flush=True)
    ref = oracle.forward(x, z, q, p)
    assert np.all(np.isfinite(ref["Z"]))
    Z, _ = gpu_forward(x, z, q, p, "aoas", "f32")
    assert np.all(np.isfinite(Z))
    assert np.max(scaled_err(Z, ref)) <= TOL["f32"]
    gref = oracle.backward(x, z, q, p, g)
    _check_grad(_backward(x, z, q, p, "aoas", "f32", g), gref, "f32", g, p)


def test_batched_large_exponent_and_values():
    # One batch holding an ordinary instance, a p = 56 instance and a |z| ~ 1e34 instance.
    cases, insts = [], []
    for k, (p, zs) in enumerate([(2.0, 1.0), (56.0, 1.0), (2.0, 1e34)]):
        x, z, q, _ = _case(70 + k, "f32", zs)
        cases.append((x, z, q, p))
        insts.append(dict(data=torch.tensor(workloads.pack_data(x, z, "aoas", "f32")[0], device="cuda"),
                          query=torch.tensor(workloads.pack_query(q, "aoas", "f32")[0], device="cuda"),
                          dim=2, p=p, out_z=torch.empty(len(q), dtype=torch.float32, device="cuda")))
    plan = batched.BatchedPlan(insts, tuning={})
    plan.run()
    torch.cuda.synchronize()
    for (x, z, q, p), inst in zip(cases, insts):
        ref = oracle.forward(x, z, q, p)
        Zg = inst["out_z"].cpu().numpy().astype(np.float64)
        assert np.all(np.isfinite(Zg))
        assert np.max(scaled_err(Zg, ref)) <= TOL["f32"], p
    plan.close()


# The FP64 sweeps take a general-p weight as 2^(e nh) from an exponent table times a
# mantissa table entry and a short series.  Coordinates are scaled by a power of two (the
# extent into [1/2, 1)) before the sweeps, in FP64 as in FP32, so factors of 1e-90 and 1e90
# only move the reported denominators by s^p; without that scale, the adjoint's factor
# w / r^2 = d^(-p-2) would leave the FP64 range at 1e-90 and p = 2.9 (about 1e441), and at
# 1e-40 the sweeps' r^2 would sit hundreds of binades from 1, far into the exponent table.
# p near 64 stresses the series.  The forward, the dz-only adjoint (the data sweep), the
# dz + dq adjoint (fused, w / r^2 from the tables) and dq alone (the query sweep) run
# through those weights; few queries may take the FP64 fix-up.
#
# At 2^-299 (about 1e-90) the oracle itself, which computes in the caller's units, cannot
# form w / r^2: there the expected values come from the oracle on the unscaled coordinates
# and the scale law of Eq. 1, exact for a power of two c: Z and dz do not change, D takes
# the factor c^-p, dq the factor 1/c, and dp does not change (the shift of ln r2 by 2 ln c
# multiplies sum_j w_ij (z_j - Z_i) = 0).
@pytest.mark.parametrize("scale,p", [(2.0 ** -299, 2.9), (1e-40, 2.9), (1.0, 0.37), (1.0, 17.9), (1.0, 63.5),
                                     (1e90, 1.3)])
def test_f64_general_p_across_scales(scale, p):
    x1, z, q1 = rand_case(71, 3000, 1000, 2, "f64")
    q1[:4] = x1[:4]                                 # exact hits
    x, q = x1 * scale, q1 * scale
    g = np.random.default_rng(72).normal(size=len(q))
    law = scale == 2.0 ** -299
    print(f"case scale={scale:g} p={p} ({'scale law' if law else 'direct'})", flush=True)
    if law:
        ref = oracle.forward(x1, z, q1, p)
        ref = dict(ref, D=ref["D"] * scale ** -p)
        gref = oracle.backward(x1, z, q1, p, g)
        gref = dict(gref, dq=gref["dq"] / scale, dq_cond=gref["dq_cond"] / scale)
    else:
        ref = oracle.forward(x, z, q, p)
        gref = oracle.backward(x, z, q, p, g)
    assert np.all(np.isfinite(ref["Z"])) and np.all(np.isfinite(ref["D"][4:]))
    assert np.all(np.isfinite(gref["dq"])) and np.all(np.isfinite(gref["dq_cond"]))
    d, qq = points(x, z, q, "aoas", "f64")
    ws = api.workspace(d, qq, "f64")
    Z, D = api.forward(d, qq, p, "f64", ws=ws)
    torch.cuda.synchronize()
    nf = int(ws[256:260].view(torch.int32).item())
    assert nf <= 4 + len(q) // 100, f"{nf} queries took the FP64 fix-up"
    assert np.max(scaled_err(Z.cpu().numpy(), ref)) <= TOL["f64"]
    np.testing.assert_allclose(D.cpu().numpy()[4:], ref["D"][4:], rtol=1e-12)
    dz, _, _ = api.backward(d, qq, p, torch.as_tensor(g, device="cuda"), Z, D, "f64", ws=ws,
                            need_dp=False, need_dq=False)
    e = np.abs(dz.cpu().numpy() - gref["dz"]) / gref["dz_scale"]
    assert np.max(e) <= GTOL["f64"], f"dz err {np.max(e):.3e}"
    dz, _, dq = api.backward(d, qq, p, torch.as_tensor(g, device="cuda"), Z, D, "f64", ws=ws,
                             need_dp=False)
    assert np.all(np.isfinite(dq.cpu().numpy()))
    e = np.abs(dz.cpu().numpy() - gref["dz"]) / gref["dz_scale"]
    assert np.max(e) <= GTOL["f64"], f"dz (with dq) err {np.max(e):.3e}"
    e = np.max(np.abs(dq.cpu().numpy() - gref["dq"])[4:], axis=1) / gref["dq_cond"][4:]
    assert np.max(e) <= GTOL["f64"], f"dq err {np.max(e):.3e}"      # rows 0-3: exact hits
    _, _, dq = api.backward(d, qq, p, torch.as_tensor(g, device="cuda"), Z, D, "f64", ws=ws,
                            need_dz=False, need_dp=False)    # the query sweep alone
    e = np.max(np.abs(dq.cpu().numpy() - gref["dq"])[4:], axis=1) / gref["dq_cond"][4:]
    assert np.max(e) <= GTOL["f64"], f"dq (alone) err {np.max(e):.3e}"
    _, dp, _ = api.backward(d, qq, p, torch.as_tensor(g, device="cuda"), Z, D, "f64", ws=ws,
                            need_dz=False, need_dq=False)    # dp: the log2 / exp2 route
    assert abs(float(dp) - gref["dp"]) <= GTOL["f64"] * gref["dp_cond"], (float(dp), gref["dp"])


# Small exponents: every weight is close to 1 whatever the distance, so a record that is not
# data but reaches the denominator (the padding after the last data point of a tile) would
# move Z by about its weight over n.  At p = 0.05 and n = 8 the padding of one tile would
# add about 6e-5 relative to D.  Coordinates of about 1e118 place the data beyond 2^390:
# only the power-of-two scale keeps it apart from any far padding coordinate.
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("n", [8, 1000])
@pytest.mark.parametrize("p", [0.05, 0.1])
@pytest.mark.parametrize("scale", [1.0, 1e118])
def test_small_exponent_few_points_and_far_coordinates(prec, n, p, scale):
    if prec == "f32" and scale != 1.0:
        pytest.skip("1e118 is beyond the FP32 range")
    x, z, q = rand_case(80 + n, n, 300, 2, prec)
    x, q = x * scale, q * scale
    q[:2] = x[:2]                                   # exact hits
    print(f"case prec={prec} n={n} p={p} scale={scale:g}", flush=True)
    ref = oracle.forward(x, z, q, p)
    assert np.all(np.isfinite(ref["Z"])) and np.all(np.isfinite(ref["D"][2:]))
    for layout in ("aoas", "soa"):
        Z, D = gpu_forward(x, z, q, p, layout, prec)
        assert np.max(scaled_err(Z, ref)) <= TOL[prec]
        np.testing.assert_allclose(D[2:], ref["D"][2:], rtol=10 * TOL[prec])
        assert np.array_equal(Z[:2], ref["Z"][:2].astype(np.float32 if prec == "f32" else np.float64))
    g = np.random.default_rng(81).normal(size=len(q))
    if prec == "f32":
        g = g.astype(np.float32).astype(np.float64)
    gref = oracle.backward(x, z, q, p, g)
    _check_grad(_backward(x, z, q, p, "hybrid", prec, g), gref, prec, g, p)
