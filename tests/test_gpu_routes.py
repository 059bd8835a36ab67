"""Query routes at small p.  The near-coincidence test on the denominator, above
(1e-6 extent)^-p, is only a candidate test: for p near 1 and large n the many moderate
weights of a query add up past it with no data point anywhere near (n E[1/d] ~ 3n at p = 1
in the unit square).  Candidates are settled by their nearest distance; these cases check
that queries routed either way agree with the oracle, in the forward, the adjoint, leave-
one-out and the batched form (which must stay bit-identical to idw_forward)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import GTOL, TOL, gpu_forward, points, rand_case, scaled_err
from paper_1402_4986_amd import api, batched, workloads

pytestmark = pytest.mark.gpu


def _case(seed, n, m, dim, prec="f32"):
    x, z, q = rand_case(seed, n, m, dim, prec)
    q[:4] = x[:4]                                         # exact hits
    q[4:8] = x[100:104] + 3e-8                            # within 1e-6 of the extent
    q[8:12] = x[200:204] + 3e-5                           # close, but not near-coincident
    t = np.float32 if prec == "f32" else np.float64
    return x, z, q.astype(t).astype(np.float64)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("p", [1.0, 0.6])
def test_small_p_forward_and_adjoint(prec, p):
    # 400,000 points: at p = 1 the denominators of nearly all queries pass 1e6.
    x, z, q = _case(800, 400000, 300, 2, prec)
    print(f"case prec={prec} p={p}", flush=True)
    ref = oracle.forward(x, z, q, p)
    assert np.median(ref["D"][12:]) > (1e-6) ** -p         # most queries are candidates
    Z, D = gpu_forward(x, z, q, p, "aoas", prec)
    assert np.max(scaled_err(Z, ref)) <= TOL[prec]
    np.testing.assert_array_equal(Z[:4], ref["Z"][:4].astype(np.float32 if prec == "f32" else np.float64))
    g = np.random.default_rng(801).normal(size=len(q))
    if prec == "f32":
        g = g.astype(np.float32).astype(np.float64)
    d, qq = points(x, z, q, "aoas", prec)
    t = torch.float32 if prec == "f32" else torch.float64
    Zt, Dt = api.forward(d, qq, p, prec)
    dz, dp, dq = api.backward(d, qq, p, torch.as_tensor(g, dtype=t, device="cuda"), Zt, Dt, prec)
    torch.cuda.synchronize()
    rb = oracle.backward(x, z, q, p, g)
    tol = GTOL[prec]
    assert np.max(np.abs(dz.cpu().numpy() - rb["dz"]) / rb["dz_scale"]) <= tol
    assert abs(float(dp) - rb["dp"]) <= tol * rb["dp_cond"]
    e = np.max(np.abs(dq.cpu().numpy() - rb["dq"]), axis=1) / np.maximum(rb["dq_cond"], 1e-300)
    assert np.max(e) <= tol


def test_small_p_leave_one_out():
    # Every query is a candidate and a data point itself; the self pair must not count as
    # a near point (it is left out), and the result must match explicit leave-one-out.
    x, z, _ = rand_case(810, 8000, 1, 2)
    Z, _ = gpu_forward(x, z, x, 0.5, "hybrid", "f32", exclude_self=True)
    ref = oracle.forward(x, z, x, 0.5, self_index=np.arange(len(x)))
    assert np.median(ref["D"]) > (1e-6) ** -0.5
    assert np.max(scaled_err(Z, ref)) <= TOL["f32"]


def test_small_p_batched_matches_forward():
    cases = []
    for k, (n, m, dim) in enumerate([(300000, 700, 2), (200000, 500, 3)]):
        x, z, q = _case(820 + k, n, m, dim)
        cases.append((x, z, q, dim))
    insts = []
    for x, z, q, dim in cases:
        insts.append(dict(data=torch.tensor(workloads.pack_data(x, z, "aoas", "f32")[0], device="cuda"),
                          query=torch.tensor(workloads.pack_query(q, "aoas", "f32")[0], device="cuda"),
                          dim=dim, p=1.0, out_z=torch.empty(len(q), dtype=torch.float32, device="cuda")))
    plan = batched.BatchedPlan(insts, chunk=1 << 30, tuning={})
    plan.run()
    torch.cuda.synchronize()
    for (x, z, q, dim), inst in zip(cases, insts):
        got = inst["out_z"].cpu().numpy().astype(np.float64)
        Zs, _ = gpu_forward(x, z, q, 1.0, "aoas", "f32", split=1)
        np.testing.assert_array_equal(got, Zs)
        ref = oracle.forward(x, z, q, 1.0)
        assert np.max(scaled_err(got, ref)) <= TOL["f32"]
    plan.close()
