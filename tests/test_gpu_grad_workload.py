"""Gradient workload (2-D FP32, n = m = 131,072, p = 1.5): the MSE-against-held-out-target
loss, its adjoint and the leave-one-out fit of p, checked against the FP64 oracle.

The oracle cannot afford all 1.7e10 pairs of every gradient sum, so:
  * dq (per query) is compared on 2,048 sampled queries of the full-size launch;
  * dz and dp (sums over queries) are compared on a second full-size launch whose upstream
    gradient is kept on those 2,048 queries only, so that the oracle's sums over them are
    exact;
  * the leave-one-out fit of p on a 4,096-point subsample ends within one grid step of the
    minimum of the oracle's loss scanned over p in [0.5, 6], and along it dL/dp matches the
    oracle's analytic gradient (itself checked against a central difference of its loss);
  * the full-size fit lowers the loss and ends at a stationary point of it.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, dp_errors, dq_errors, points
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
        ec, es = dp_errors(dp, ref)
        assert ec <= tol and es <= tol
    if dq is not None:
        ec, es = dq_errors(dq, ref)
        assert np.max(ec) <= tol and (es.size == 0 or np.max(es) <= tol)


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
    _check_grad((None, None, dq.cpu().numpy().astype(np.float64)[idx]), ref, "f32")
    # dz and dp of the full-size launch: the same launch with the upstream gradient kept on
    # the sampled queries only (zero elsewhere), so that their sums over queries are the
    # oracle's sums over those queries
    gs = np.zeros(len(q))
    gs[idx] = g32[idx]
    a, b, c = api.backward(d, qq, p, torch.tensor(gs, dtype=torch.float32, device="cuda"), Z, D, "f32")
    torch.cuda.synchronize()
    ch = c.cpu().numpy().astype(np.float64)
    _check_grad((a.cpu().numpy().astype(np.float64), float(b), ch[idx]), ref, "f32")
    assert np.all(ch[np.setdiff1d(np.arange(len(q)), idx)] == 0.0)


def _loo_scan(xs, zs, grid):
    """The oracle's leave-one-out loss at every p of the grid (one thread per value)."""
    import concurrent.futures as cf
    with cf.ThreadPoolExecutor(16) as ex:
        return np.array(list(ex.map(lambda pv: oracle.loo_loss(xs, zs, pv), grid)))


def test_loo_fit_reaches_the_oracle_minimum_and_its_gradient_matches():
    # The leave-one-out fit of p on a 4,096-point subsample (at most 50 evaluations of the
    # loss and its gradient).  Pinned against the oracle: its loss scanned over p in
    # [0.5, 6] (step 0.1) has its minimum within one grid step of the fitted p, and the loss
    # at the fitted p is at most the scan's minimum (1e-4 relative).  At the start, middle
    # and end of the fit the GPU dL/dp is checked against the oracle's analytic gradient
    # for the same upstream gradient (the GPU's own 2 (Z - z) / n, in FP32 as autograd
    # hands it down), and the oracle's gradient against a central difference of its loss.
    x, z, _, _, p0 = _data()
    sub = np.random.default_rng(4).choice(len(x), size=4096, replace=False)
    xs, zs = x[sub], z[sub]
    X = torch.tensor(xs, dtype=torch.float32, device="cuda")
    Zt = torch.tensor(zs, dtype=torch.float32, device="cuda")
    p_fit, hist = api.fit_p_loo(X, Zt, p0=p0, steps=50)
    print(f"fitted p {p_fit:.4f} after {len(hist)} evaluations", flush=True)
    assert len(hist) <= 50 and hist[-1][1] < hist[0][1]
    grid = np.round(np.arange(0.5, 6.0 + 1e-9, 0.1), 10)
    scan = _loo_scan(xs, zs, grid)
    k = int(np.argmin(scan))
    assert 0 < k < len(grid) - 1, "the scan's minimum lies inside [0.5, 6]"
    assert abs(p_fit - grid[k]) <= 0.1 + 1e-12, (p_fit, grid[k])
    assert oracle.loo_loss(xs, zs, p_fit) <= scan[k] * (1 + 1e-4)
    idx = np.arange(len(xs))
    for pv in (hist[0][0], hist[len(hist) // 2][0], p_fit):
        pt = torch.tensor(pv, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = api.loo_loss(X, Zt, pt)
        loss.backward()
        gpu_dp = float(pt.grad)
        Zg = api.IDWFunction.apply(X, Zt, X, pt.detach(), True).cpu().numpy().astype(np.float64)
        g_gpu = (2.0 * (Zg - zs) / len(xs)).astype(np.float32).astype(np.float64)
        ref = oracle.backward(xs, zs, xs, pv, g_gpu, self_index=idx)
        assert abs(gpu_dp - ref["dp"]) <= GTOL["f32"] * ref["dp_cond"], (pv, gpu_dp, ref["dp"])
        r = oracle.forward(xs, zs, xs, pv, self_index=idx)
        exact = oracle.backward(xs, zs, xs, pv, 2.0 * (r["Z"] - zs) / len(xs), self_index=idx)
        h = 1e-4
        fd = (oracle.loo_loss(xs, zs, pv + h) - oracle.loo_loss(xs, zs, pv - h)) / (2 * h)
        assert exact["dp"] == pytest.approx(fd, rel=1e-5, abs=1e-9)
        # the loss from Z within 1e-5 S of the oracle's: |L - L_o| <= mean(2 e |Z_o - z| + e^2)
        # with e = 1e-5 S the largest error the forward's tolerance allows per query
        e = GTOL["f32"] * r["S"]
        bound = np.mean(2.0 * e * np.abs(r["Z"] - zs) + e * e)
        assert abs(float(loss.detach()) - np.mean((r["Z"] - zs) ** 2)) <= bound


def test_full_size_loo_fit_reaches_a_stationary_point():
    # The leave-one-out fit on all 131,072 points: the loss goes down, and at the fitted p
    # the GPU gradient has fallen below a hundredth of its value at p0 (the oracle cannot
    # scan this size).
    x, z, _, _, p0 = _data()
    X = torch.tensor(x, dtype=torch.float32, device="cuda")
    Zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    print("full-size LOO fit, at most 50 evaluations", flush=True)
    p_fit, hist = api.fit_p_loo(X, Zt, p0=p0, steps=50)
    assert hist[-1][1] < hist[0][1] and len(hist) <= 50
    assert 0.05 < p_fit < 6.0

    def grad_at(pv):
        pt = torch.tensor(pv, dtype=torch.float64, device="cuda", requires_grad=True)
        api.loo_loss(X, Zt, pt).backward()
        return float(pt.grad)

    assert abs(grad_at(p_fit)) <= 1e-2 * abs(grad_at(p0)), p_fit
