"""Gradient workload (2-D FP32, n = m = 131,072, p = 1.5): the MSE-against-held-out-target
loss, its adjoint and the leave-one-out fit of p, checked against the FP64 oracle.

The oracle cannot afford all 1.7e10 pairs of every gradient sum, so:
  * dq (per query) is compared on 2,048 sampled queries of the full-size launch;
  * dz and dp (sums over queries) are compared on the same sampled query subset, run
    through the library as its own (smaller) query set;
  * along the 50-step Adam fit of p on a 4,096-point subsample, dL/dp of the leave-one-out
    loss matches the oracle's analytic gradient and a central difference of its loss;
    the full-size fit lowers the loss.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, points
from paper_1402_4986_amd import api, workloads

pytestmark = pytest.mark.gpu


def _data():
    cfg = workloads.WORKLOADS["plain2d_grad_f32_128k"]
    x, z, q, t = workloads.plain2d(cfg["n"], cfg["m"], "f32", cfg=cfg["cfg"])
    return x, z, q, t, cfg["p"]


def _check_grad(got, ref, prec):
    dz, dp, dq = got
    tol = GTOL[prec]
    if dz is not None:
        assert np.max(np.abs(dz - ref["dz"]) / np.maximum(ref["dz_scale"], 1e-300)) <= tol
    if dp is not None:
        assert abs(dp - ref["dp"]) <= tol * ref["dp_cond"]
    if dq is not None:
        e = np.max(np.abs(dq - ref["dq"]), axis=1) / np.maximum(ref["dq_cond"], 1e-300)
        assert np.max(e) <= tol


def test_full_size_mse_adjoint_sampled():
    x, z, q, t, p = _data()
    d, qq = points(x, z, q, "hybrid", "f32")
    Z, D = api.forward(d, qq, p, "f32")
    Zh = Z.cpu().numpy().astype(np.float64)
    g = (2.0 / len(q)) * (Zh - t)                      # dL/dZ of the mean squared error
    g32 = g.astype(np.float32).astype(np.float64)
    gt = torch.tensor(g32, dtype=torch.float32, device="cuda")
    print("full-size backward n=m=131072", flush=True)
    dz, dp, dq = api.backward(d, qq, p, gt, Z, D, "f32")
    torch.cuda.synchronize()
    assert torch.all(torch.isfinite(dz)) and torch.isfinite(dp) and torch.all(torch.isfinite(dq))
    idx = np.sort(np.random.default_rng(3).choice(len(q), size=2048, replace=False))
    ref = oracle.backward(x, z, q[idx], p, g32[idx])
    e = np.max(np.abs(dq.cpu().numpy()[idx] - ref["dq"]), axis=1) / ref["dq_cond"]
    assert np.max(e) <= GTOL["f32"]
    # the same sampled queries as their own query set: dz and dp sums
    ds, qs = points(x, z, q[idx], "hybrid", "f32")
    Zs, Ds = api.forward(ds, qs, p, "f32")
    gs = torch.tensor(g32[idx], dtype=torch.float32, device="cuda")
    a, b, c = api.backward(ds, qs, p, gs, Zs, Ds, "f32")
    torch.cuda.synchronize()
    _check_grad((a.cpu().numpy().astype(np.float64), float(b), c.cpu().numpy().astype(np.float64)), ref, "f32")


def test_loo_fit_gradient_matches_oracle_and_finite_differences():
    # 50 Adam steps on the leave-one-out loss of a 4,096-point subsample; at the start,
    # middle and end of the fit the GPU dL/dp is checked against the oracle's analytic
    # gradient and a central difference of the oracle's loss.
    x, z, _, _, p0 = _data()
    sub = np.random.default_rng(4).choice(len(x), size=4096, replace=False)
    xs, zs = x[sub], z[sub]
    X = torch.tensor(xs, dtype=torch.float32, device="cuda")
    Zt = torch.tensor(zs, dtype=torch.float32, device="cuda")
    p_fit, hist = api.fit_p_loo(X, Zt, p0=p0, steps=50, lr=0.05)
    print(f"fitted p {p_fit:.4f}", flush=True)
    assert hist[-1][1] < hist[0][1] and p_fit > p0  # the LOO optimum of this field lies above 1.5
    idx = np.arange(len(xs))
    for pv in (hist[0][0], hist[25][0], p_fit):
        pt = torch.tensor(pv, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = api.loo_loss(X, Zt, pt)
        loss.backward()
        gpu_dp = float(pt.grad)
        r = oracle.forward(xs, zs, xs, pv, self_index=idx)
        g = 2.0 * (r["Z"] - zs) / len(xs)
        ref = oracle.backward(xs, zs, xs, pv, g, self_index=idx)
        h = 1e-4
        fd = (oracle.loo_loss(xs, zs, pv + h) - oracle.loo_loss(xs, zs, pv - h)) / (2 * h)
        assert ref["dp"] == pytest.approx(fd, rel=1e-5, abs=1e-9)
        assert abs(gpu_dp - ref["dp"]) <= 1e-4 * abs(ref["dp"]) + GTOL["f32"] * ref["dp_cond"], (pv, gpu_dp, ref["dp"])
        assert float(loss.detach()) == pytest.approx(oracle.loo_loss(xs, zs, pv), rel=1e-4)


def test_full_size_loo_fit_lowers_the_loss():
    x, z, _, _, p0 = _data()
    X = torch.tensor(x, dtype=torch.float32, device="cuda")
    Zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    print("full-size LOO fit, 50 steps", flush=True)
    p_fit, hist = api.fit_p_loo(X, Zt, p0=p0, steps=50, lr=0.05)
    assert hist[-1][1] < hist[0][1]
    assert 0.05 <= p_fit <= 6.0
