"""GPU adjoint parity: dz, dp and dq from idw_backward against the FP64 oracle's analytic
gradient (itself pinned by 80-digit finite differences in test_oracle_grad.py), element
by element.

Tolerances (the workload states none for gradients; these follow the forward's): 1e-5
for the FP32 path and 1e-12 for the FP64 path, relative to each sum's condition scale.
dz_j = sum_i g_i w_ij / D_i has positive weights: its scale is sum_i |g_i| w_ij / D_i.
dp and dq are sums centred on Z_i (factor z_j - Z_i).  Close to a data point that factor
is tiny, and a relative perturbation e of the values (the FP32 rounding of z and Z, or
FP64 rounding at near-coincident points) moves the sum by about e times the uncentred
sum, with |z_j| + |Z_i| in place of |z_j - Z_i|: that uncentred sum is their scale.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, TOL, dp_errors, dq_errors, points, rand_case
from paper_1402_4986_amd import api

pytestmark = pytest.mark.gpu


def _run(x, z, q, p, layout, prec, g, exclude_self=False, need=(True, True, True)):
    d, qq = points(x, z, q, layout, prec)
    Z, D = api.forward(d, qq, p, prec, exclude_self=exclude_self)
    t = torch.float32 if prec == "f32" else torch.float64
    gt = torch.as_tensor(g, dtype=t, device="cuda")
    dz, dp, dq = api.backward(d, qq, p, gt, Z, D, prec, need_dz=need[0], need_dp=need[1], need_dq=need[2],
                              exclude_self=exclude_self)
    torch.cuda.synchronize()
    cv = lambda a: None if a is None else a.cpu().numpy().astype(np.float64)
    return cv(dz), (None if dp is None else float(dp)), cv(dq)


def _check(got, ref, prec):
    dz, dp, dq = got
    tol = GTOL[prec]
    if dz is not None:
        e = np.abs(dz - ref["dz"]) / np.maximum(ref["dz_scale"], 1e-300)
        assert np.max(e) <= tol, f"dz err {np.max(e):.3e}"
    if dp is not None:
        ec, es = dp_errors(dp, ref)
        assert ec <= tol and es <= tol, f"dp {dp} vs {ref['dp']}"
    if dq is not None:
        ec, es = dq_errors(dq, ref)
        assert np.max(ec) <= tol, f"dq err {np.max(ec):.3e}"
        # well-conditioned rows are held to their own (centred) absolute-term sum as well
        assert es.size == 0 or np.max(es) <= tol, f"dq err (centred scale) {np.max(es):.3e}"


@pytest.mark.parametrize("layout", ["hybrid", "aoas", "soa"])
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [1.0, 1.5, 2.0, 2.5, 3.0])
def test_backward_matches_oracle_small(layout, prec, dim, p):
    x, z, q = rand_case(200 + dim, 2100, 777, dim, prec)
    g = np.random.default_rng(5).normal(size=len(q))
    if prec == "f32":
        g = g.astype(np.float32).astype(np.float64)
    print(f"case layout={layout} prec={prec} dim={dim} p={p}", flush=True)
    got = _run(x, z, q, p, layout, prec, g)
    ref = oracle.backward(x, z, q, p, g)
    _check(got, ref, prec)


@pytest.mark.parametrize("need", [(True, False, False), (False, True, False), (False, False, True)])
def test_backward_single_gradients(need):
    x, z, q = rand_case(21, 1500, 900, 2)
    g = np.random.default_rng(6).normal(size=len(q)).astype(np.float32).astype(np.float64)
    got = _run(x, z, q, 2.0, "hybrid", "f32", g, need=need)
    assert (got[0] is None) != need[0] and (got[1] is None) != need[1] and (got[2] is None) != need[2]
    _check(got, oracle.backward(x, z, q, 2.0, g), "f32")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_backward_hits_and_near_coincident_queries(prec):
    x, z, q = rand_case(22, 1800, 400, 2, prec)
    x[5] = x[4]
    q[:20] = x[:20]                  # exact hits, q[4], q[5] on a duplicate pair
    q[20:30] = x[200:210] + 3e-7     # near-coincident: FP64 fix-up
    t = np.float32 if prec == "f32" else np.float64
    q = q.astype(t).astype(np.float64)
    g = np.random.default_rng(7).normal(size=len(q)).astype(t).astype(np.float64)
    got = _run(x, z, q, 2.0, "aoas", prec, g)
    ref = oracle.backward(x, z, q, 2.0, g)
    _check(got, ref, prec)
    np.testing.assert_array_equal(got[2][:20], 0.0)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_backward_leave_one_out(prec):
    x, z, _ = rand_case(23, 2300, 1, 2, prec)
    g = np.random.default_rng(8).normal(size=len(x)).astype(np.float32).astype(np.float64)
    got = _run(x, z, x, 1.5, "hybrid", prec, g, exclude_self=True)
    ref = oracle.backward(x, z, x, 1.5, g, self_index=np.arange(len(x)))
    _check(got, ref, prec)


def test_value_gradient_conserves_the_upstream_sum():
    x, z, q = rand_case(24, 3000, 2000, 3, "f64")
    g = np.random.default_rng(9).normal(size=len(q))
    dz, _, _ = _run(x, z, q, 2.5, "aoas", "f64", g, need=(True, False, False))
    assert abs(dz.sum() - g.sum()) <= 1e-11 * np.abs(g).sum()


def test_zero_queries_gives_zero_gradients():
    x, z, q = rand_case(25, 100, 0, 2)
    d, qq = points(x, z, q.reshape(0, 2), "hybrid", "f32")
    Z, D = api.forward(d, qq, 2.0, "f32")
    dz, dp, dq = api.backward(d, qq, 2.0, torch.zeros(0, device="cuda"), Z, D, "f32")
    torch.cuda.synchronize()
    assert torch.all(dz == 0) and float(dp) == 0.0 and dq.shape == (0, 2)


def test_autograd_function_gradcheck_fp64():
    r = np.random.default_rng(26)
    X = torch.tensor(r.random((40, 2)), device="cuda")
    z = torch.tensor(r.normal(size=40), device="cuda", requires_grad=True)
    Q = torch.tensor(r.random((7, 2)), device="cuda", requires_grad=True)
    p = torch.tensor(1.7, dtype=torch.float64, device="cuda", requires_grad=True)
    f = lambda z_, Q_, p_: api.IDWFunction.apply(X, z_, Q_, p_)
    assert torch.autograd.gradcheck(f, (z, Q, p), eps=1e-6, atol=1e-7, rtol=1e-5)


def test_loo_fit_reduces_the_loss():
    x, z, _ = rand_case(27, 4096, 1, 2, "f32")
    X = torch.tensor(x, dtype=torch.float32, device="cuda")
    zt = torch.tensor(z, dtype=torch.float32, device="cuda")
    for method in ("adam", "lbfgs"):
        p, hist = api.fit_p_loo(X, zt, p0=1.5, steps=20, lr=0.1, method=method)
        assert hist[-1][1] < hist[0][1] and len(hist) <= 20
        # the loss at the fitted p agrees with the oracle's leave-one-out loss, within what
        # the forward's tolerance (1e-5 S per query) allows: mean(2 e |Z - z| + e^2)
        r = oracle.forward(x, z, x, p, self_index=np.arange(len(x)))
        e = 1e-5 * r["S"]
        got = float(api.loo_loss(X, zt, torch.tensor(p, dtype=torch.float64, device="cuda")))
        assert abs(got - np.mean((r["Z"] - z) ** 2)) <= np.mean(2 * e * np.abs(r["Z"] - z) + e * e)


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fixup_split_over_data_chunks(prec):
    # Few flagged queries against many data points: the FP64 fix-up cuts each flagged
    # query's data range into chunks swept by separate workgroups and merged in order.
    x, z, q = rand_case(28, 200000, 300, 2, prec)
    q[:3] = x[[5, 77, 1234]]                 # exact hits
    q[3:6] = x[[9, 99, 999]] + 3e-7          # near-coincident
    t = np.float32 if prec == "f32" else np.float64
    q = q.astype(t).astype(np.float64)
    d, qq = points(x, z, q, "soa", prec)
    Z, D = api.forward(d, qq, 2.0, prec)
    Zh = Z.cpu().numpy().astype(np.float64)
    ref = oracle.forward(x, z, q, 2.0)
    assert np.all(ref["H"][:3] == 1)
    np.testing.assert_array_equal(Zh[:3], ref["Z"][:3].astype(t).astype(np.float64))
    near = np.abs(Zh[3:6] - ref["Z"][3:6]) / ref["S"][3:6]
    assert np.max(near) <= (6e-8 if prec == "f32" else 1e-14)
    assert np.max(np.abs(Zh - ref["Z"]) / ref["S"]) <= TOL[prec]
    g = np.random.default_rng(29).normal(size=len(q)).astype(t).astype(np.float64)
    got = _run(x, z, q, 2.0, "soa", prec, g)
    _check(got, oracle.backward(x, z, q, 2.0, g), prec)


@pytest.mark.parametrize("separate", [False, True])
@pytest.mark.parametrize("dim,p", [(2, 2.0), (3, 2.5), (2, 1.0), (3, 3.0)])
def test_fused_and_separate_adjoint_sweeps(separate, dim, p):
    # FP32 dz with dp/dq runs as one fused sweep by default; the separate query-direction
    # and data-direction sweeps stay available.  Both against the oracle.
    x, z, q = rand_case(30 + dim, 2100, 1537, dim)
    g = np.random.default_rng(31).normal(size=len(q)).astype(np.float32).astype(np.float64)
    d, qq = points(x, z, q, "aoas", "f32")
    Z, D = api.forward(d, qq, p, "f32")
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    dz, dp, dq = api.backward(d, qq, p, gt, Z, D, "f32", separate=separate)
    torch.cuda.synchronize()
    got = (dz.cpu().numpy().astype(np.float64), float(dp), dq.cpu().numpy().astype(np.float64))
    _check(got, oracle.backward(x, z, q, p, g), "f32")


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_fused_adjoint_accumulates_over_query_blocks(prec):
    # 1,000,000 data points in 31 ranges and 600,000 queries: in FP32, 586 blocks of 1,024
    # queries on 265 workgroup groups; in FP64, 1,172 blocks of 512 on the same 265 groups.
    # Each group folds two or three (FP64: four or five) query blocks into its dz row.  The
    # upstream gradient is non-zero on 150 scattered queries only, so the oracle needs just
    # those queries for the exact dz, dp and dq.
    t = np.float32 if prec == "f32" else np.float64
    x, z, q = rand_case(32, 1000000, 600000, 2, prec)
    r = np.random.default_rng(33)
    sel = np.sort(r.choice(len(q), size=150, replace=False))
    g = np.zeros(len(q))
    g[sel] = r.normal(size=150).astype(t)
    print(f"fused fold prec={prec}", flush=True)
    d, qq = points(x, z, q, "soa", prec)
    Z, D = api.forward(d, qq, 2.0, prec)
    gt = torch.tensor(g, dtype=torch.float32 if prec == "f32" else torch.float64, device="cuda")
    dz, dp, dq = api.backward(d, qq, 2.0, gt, Z, D, prec)
    torch.cuda.synchronize()
    ref = oracle.backward(x, z, q[sel], 2.0, g[sel])
    dqh = dq.cpu().numpy().astype(np.float64)
    got = (dz.cpu().numpy().astype(np.float64), float(dp), dqh[sel])
    _check(got, ref, prec)
    rest = np.setdiff1d(np.arange(len(q)), sel)
    assert np.all(dqh[rest] == 0.0)
