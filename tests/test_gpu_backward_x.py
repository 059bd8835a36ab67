"""GPU parity of the gradient with respect to the data coordinates (IDW_NEED_DX) against
the FP64 oracle, element by element:

    dL/dx_j = sum_i g_i (p / D_i)(w_ij / r2_ij)(z_j - Z_i)(q_i - x_j)

It comes from the fused FP32 adjoint sweep (default), from the data-direction sweep that
also yields dz (FP64, or FP32 with the separate sweeps), and from the FP64 fix-up for
queries at or near a data point.  The tolerance is that of dq: FP32 1e-5 and FP64 1e-12
of each row's uncentred condition scale (|z_j| + |Z_i| in place of z_j - Z_i), plus, for
FP32 outputs, the subnormal spacing 2^-149 as an absolute floor.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, points, rand_case
from paper_1402_4986_amd import api

pytestmark = pytest.mark.gpu

FLOOR = {"f32": 2.0 ** -149, "f64": 0.0}


def _run(x, z, q, p, layout, prec, g, exclude_self=False, separate=False, need=(True, True, True)):
    d, qq = points(x, z, q, layout, prec)
    Z, D = api.forward(d, qq, p, prec, exclude_self=exclude_self)
    t = torch.float32 if prec == "f32" else torch.float64
    gt = torch.as_tensor(g, dtype=t, device="cuda")
    dz, dp, dq, dx = api.backward(d, qq, p, gt, Z, D, prec, need_dz=need[0], need_dp=need[1], need_dq=need[2],
                                  exclude_self=exclude_self, separate=separate, need_dx=True)
    torch.cuda.synchronize()
    cv = lambda a: None if a is None else a.cpu().numpy().astype(np.float64)
    return cv(dz), (None if dp is None else float(dp)), cv(dq), cv(dx)


def _check_dx(dx, ref, prec):
    assert np.all(np.isfinite(dx))
    e = np.max(np.abs(dx - ref["dx"]), axis=1) - GTOL[prec] * ref["dx_cond"]
    assert np.max(e) <= FLOOR[prec], f"dx err {np.max(e):.3e} above the bound"


def _g(seed, m, prec):
    g = np.random.default_rng(seed).normal(size=m)
    return g.astype(np.float32).astype(np.float64) if prec == "f32" else g


@pytest.mark.parametrize("layout", ["hybrid", "aoas", "soa"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [1.0, 2.0, 2.5, 3.0])
def test_dx_matches_oracle_small(layout, prec, dim, p):
    x, z, q = rand_case(400 + dim, 2100, 777, dim, prec)
    g = _g(8, len(q), prec)
    print(f"case layout={layout} prec={prec} dim={dim} p={p}", flush=True)
    dz, dp, dq, dx = _run(x, z, q, p, layout, prec, g)
    _check_dx(dx, oracle.backward_x(x, z, q, p, g), prec)
    # the other gradients of the same call are unchanged by the request
    ref = oracle.backward(x, z, q, p, g)
    assert np.max(np.abs(dz - ref["dz"]) / ref["dz_scale"]) <= GTOL[prec]
    assert abs(dp - ref["dp"]) <= GTOL[prec] * ref["dp_cond"]


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [1.5, 2.0])
def test_dx_separate_fp32_sweeps(dim, p):
    x, z, q = rand_case(410 + dim, 2500, 1300, dim)
    g = _g(9, len(q), "f32")
    print(f"case separate dim={dim} p={p}", flush=True)
    _, _, _, dx = _run(x, z, q, p, "aoas", "f32", g, separate=True)
    _check_dx(dx, oracle.backward_x(x, z, q, p, g), "f32")


@pytest.mark.parametrize("need", [(False, False, False), (True, False, False), (False, True, False)])
def test_dx_alone_or_with_some_gradients(need):
    x, z, q = rand_case(420, 1900, 900, 2)
    g = _g(10, len(q), "f32")
    dz, dp, dq, dx = _run(x, z, q, 2.0, "hybrid", "f32", g, need=need)
    assert (dz is None) != need[0] and (dp is None) != need[1] and (dq is None) != need[2]
    _check_dx(dx, oracle.backward_x(x, z, q, 2.0, g), "f32")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_dx_hits_and_near_coincident_queries(prec):
    x, z, q = rand_case(430, 1800, 400, 2, prec)
    x[5] = x[4]
    q[:20] = x[:20]                  # exact hits (no dx contribution), a duplicate pair
    q[20:30] = x[200:210] + 3e-7     # near-coincident: FP64 fix-up
    t = np.float32 if prec == "f32" else np.float64
    q = q.astype(t).astype(np.float64)
    g = _g(11, len(q), prec)
    _, _, _, dx = _run(x, z, q, 2.0, "aoas", prec, g)
    _check_dx(dx, oracle.backward_x(x, z, q, 2.0, g), prec)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_dx_leave_one_out(prec):
    x, z, _ = rand_case(440, 3000, 1, 2, prec)
    g = _g(12, len(x), prec)
    _, _, _, dx = _run(x, z, x, 1.7, "hybrid", prec, g, exclude_self=True)
    _check_dx(dx, oracle.backward_x(x, z, x, 1.7, g, self_index=np.arange(len(x))), prec)


def test_dx_and_dq_cancel_on_the_gpu():
    # Z depends on q - x only: sum_j dx_j = -sum_i dq_i (FP64 path, no hits).
    x, z, q = rand_case(450, 2000, 800, 3, "f64")
    g = _g(13, len(q), "f64")
    _, _, dq, dx = _run(x, z, q, 2.0, "aoas", "f64", g)
    ref = oracle.backward_x(x, z, q, 2.0, g)
    scale = np.sum(ref["dx_cond"])
    np.testing.assert_allclose(dx.sum(axis=0), -dq.sum(axis=0), rtol=0, atol=1e-12 * scale)


def test_fused_dx_accumulates_over_query_blocks():
    # As for dz: 1,000,000 data points in 31 ranges, 600,000 queries in 586 blocks folded by
    # 265 groups; the upstream gradient is non-zero on 150 queries only, so the oracle needs
    # just those queries.
    x, z, q = rand_case(460, 1000000, 600000, 2)
    r = np.random.default_rng(461)
    sel = np.sort(r.choice(len(q), size=150, replace=False))
    g = np.zeros(len(q))
    g[sel] = r.normal(size=150).astype(np.float32)
    print("fused dx, n=1e6 m=6e5", flush=True)
    _, _, _, dx = _run(x, z, q, 2.0, "soa", "f32", g)
    _check_dx(dx, oracle.backward_x(x, z, q[sel], 2.0, g[sel]), "f32")


def test_autograd_reaches_data_coordinates():
    x, z, q = rand_case(470, 1500, 600, 2)
    g = _g(14, len(q), "f32")
    X = torch.tensor(x, dtype=torch.float32, device="cuda", requires_grad=True)
    V = torch.tensor(z, dtype=torch.float32, device="cuda", requires_grad=True)
    Q = torch.tensor(q, dtype=torch.float32, device="cuda", requires_grad=True)
    p = torch.tensor(2.0, dtype=torch.float64, device="cuda", requires_grad=True)
    Z = api.interpolate(X, V, Q, p)
    (Z.double() * torch.tensor(g, device="cuda")).sum().backward()
    _check_dx(X.grad.cpu().numpy().astype(np.float64), oracle.backward_x(x, z, q, 2.0, g), "f32")
    ref = oracle.backward(x, z, q, 2.0, g)
    e = np.max(np.abs(Q.grad.cpu().numpy() - ref["dq"]), axis=1) / ref["dq_cond"]
    assert np.max(e) <= GTOL["f32"]


def test_gradcheck_fp64_with_data_coordinates():
    r = np.random.default_rng(480)
    X = torch.tensor(r.random((40, 2)), dtype=torch.float64, device="cuda", requires_grad=True)
    V = torch.tensor(r.normal(size=40), dtype=torch.float64, device="cuda", requires_grad=True)
    Q = torch.tensor(r.random((12, 2)), dtype=torch.float64, device="cuda", requires_grad=True)
    p = torch.tensor(1.8, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda a, b, c, d: api.interpolate(a, b, c, d), (X, V, Q, p),
                                    eps=1e-6, atol=1e-7, rtol=1e-6)


def test_dx_degenerate_sizes():
    # No queries: every gradient is zero.  One data point: Z is that point's value for every
    # query, so its position has no gradient.
    x, z, q = rand_case(490, 500, 0, 2)
    d, qq = points(x, z, np.zeros((0, 2)), "aoas", "f32")
    dz, dp, dq, dx = api.backward(d, qq, 2.0, torch.zeros(0, device="cuda"), torch.zeros(0, device="cuda"),
                                  torch.zeros(0, dtype=torch.float64, device="cuda"), "f32", need_dx=True)
    torch.cuda.synchronize()
    assert torch.all(dz == 0) and float(dp) == 0.0 and torch.all(dx == 0) and dq.numel() == 0
    x1, z1, q1 = rand_case(491, 1, 300, 3)
    g = _g(15, 300, "f32")
    _, _, _, dx1 = _run(x1, z1, q1, 2.0, "hybrid", "f32", g)
    assert np.all(dx1 == 0.0)
