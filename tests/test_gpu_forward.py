"""GPU forward parity against the FP64 oracle (element by element), through the C ABI.

Tolerances (stated by the workload definition): FP32 path 1e-5 and FP64 path 1e-12,
relative to the summation scale S_i = sum_j w_ij |z_j| / sum_j w_ij (>= |Z_i|), so that
queries where Z crosses zero are measured against the conditioning of their sum.
"""
import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import (GTOL, PLAIN_TOL, TOL, dp_errors, dq_errors, gpu_forward, oracle_backward_par,
                         oracle_forward_par, plain_rel_err, points, rand_case, scaled_err)
from paper_1402_4986_amd import api, workloads

pytestmark = pytest.mark.gpu

LAYOUTS = ["soa", "aos", "aoas", "hybrid", "soaos"]


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [1.0, 2.0, 2.5, 3.0, 4.0, 1.7])
def test_forward_matches_oracle_small(layout, prec, dim, p):
    # 3000 data points = 5 full LDS tiles + a ragged one; 1337 queries = ragged query block.
    x, z, q = rand_case(100 + dim, 3000, 1337, dim, prec)
    print(f"case layout={layout} prec={prec} dim={dim} p={p}", flush=True)
    Z, D = gpu_forward(x, z, q, p, layout, prec)
    ref = oracle.forward(x, z, q, p)
    err = scaled_err(Z, ref)
    assert np.max(err) <= TOL[prec], f"max scaled err {np.max(err):.3e}"
    np.testing.assert_allclose(D, ref["D"], rtol=10 * TOL[prec])


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_exact_hits_duplicates_and_near_coincident_points(prec):
    x, z, q = rand_case(7, 2000, 600, 2, prec)
    x[11] = x[10]                       # duplicate location with a different value
    q[:50] = x[:50]                     # exact hits (q[10], q[11] hit the duplicate pair)
    q[50:60] = x[100:110] + 3e-7        # closer than 1e-6 of the extent: FP64 path
    t = np.float32 if prec == "f32" else np.float64
    q = q.astype(t).astype(np.float64)
    Z, D = gpu_forward(x, z, q, 2.0, "aoas", prec)
    ref = oracle.forward(x, z, q, 2.0)
    hits = ref["H"] > 0
    assert hits[:50].all()
    # exact hit: the data value (mean of duplicates), rounded once to the output type
    np.testing.assert_array_equal(Z[hits], ref["Z"][hits].astype(t).astype(np.float64))
    assert np.all(np.isinf(D[hits]))
    # near-coincident queries are recomputed in FP64: only the output rounding remains
    assert not hits[50:60].any()
    near = scaled_err(Z[50:60], {"Z": ref["Z"][50:60], "S": ref["S"][50:60]})
    assert np.max(near) <= (6e-8 if prec == "f32" else 1e-14)
    assert np.max(scaled_err(Z, ref)) <= TOL[prec]


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("p", [2.0, 2.5])
def test_leave_one_out_matches_oracle(prec, p):
    x, z, _ = rand_case(8, 2500, 1, 2, prec)
    x[7] = x[3]  # a duplicate: left-out point 3 still has an exact hit at 7
    d, q = points(x, z, x, "hybrid", prec)
    Z, _ = api.forward(d, q, p, prec, exclude_self=True)
    Z = Z.cpu().numpy().astype(np.float64)
    ref = oracle.forward(x, z, x, p, self_index=np.arange(len(x)))
    assert np.max(scaled_err(Z, ref)) <= TOL[prec]
    assert Z[3] == np.float64(z[7]).astype(np.float32 if prec == "f32" else np.float64)


@pytest.mark.parametrize("split", [1, 3, 7, 64])
def test_data_split_merges_to_the_same_result(split):
    x, z, q = rand_case(9, 40000, 700, 2)
    Z, _ = gpu_forward(x, z, q, 2.0, "aoas", "f32", split=split)
    ref = oracle.forward(x, z, q, 2.0)
    assert np.max(scaled_err(Z, ref)) <= TOL["f32"]


@pytest.mark.parametrize("prec,qpl", [("f32", 2), ("f32", 4), ("f32", 8), ("f64", 2), ("f64", 4)])
@pytest.mark.parametrize("dim,p", [(2, 2.0), (3, 3.0), (2, 1.7)])
def test_queries_per_lane_variants(prec, qpl, dim, p):
    # Every queries-per-lane build against the oracle (the defaults are 2 for FP64 and for
    # the FP32 weights with one transcendental, 4 otherwise), with a ragged last block.
    x, z, q = rand_case(10, 5000, 3001, dim, prec)
    Z, _ = gpu_forward(x, z, q, p, "soa", prec, queries_per_lane=qpl)
    ref = oracle.forward(x, z, q, p)
    assert np.max(scaled_err(Z, ref)) <= TOL[prec]


def test_tiny_and_degenerate_sizes():
    for n, m in [(1, 1), (1, 5), (2, 1), (511, 3), (513, 257), (1024, 1)]:
        x, z, q = rand_case(11 + n, n, m, 2)
        Z, _ = gpu_forward(x, z, q, 2.0, "aos", "f32")
        ref = oracle.forward(x, z, q, 2.0)
        assert np.max(scaled_err(Z, ref)) <= TOL["f32"], (n, m)
    # all data points at one location: extent is degenerate (taken as 1)
    x = np.full((100, 2), 0.25)
    z = np.arange(100.0)
    q = np.array([[0.25, 0.25], [0.5, 0.5], [0.0, 1.0]])
    Z, _ = gpu_forward(x, z, q, 2.0, "soa", "f32")
    assert Z[0] == np.float32(np.mean(z))
    np.testing.assert_allclose(Z[1:], np.mean(z), rtol=1e-6)


def test_determinism_permutation_and_power_of_two_scaling():
    x, z, q = rand_case(12, 6000, 2000, 2)
    Z1, D1 = gpu_forward(x, z, q, 2.0, "aoas", "f32")
    Z2, D2 = gpu_forward(x, z, q, 2.0, "aoas", "f32")
    np.testing.assert_array_equal(Z1, Z2)
    np.testing.assert_array_equal(D1, D2)
    perm = np.random.default_rng(0).permutation(len(q))
    Zp, _ = gpu_forward(x, z, q[perm], 2.0, "aoas", "f32")
    np.testing.assert_array_equal(Zp, Z1[perm])
    # coordinates times 2^5: the sweep rescales by a power of two, so Z is bit-identical
    Zs, Ds = gpu_forward(x * 32.0, z, q * 32.0, 2.0, "aoas", "f32")
    np.testing.assert_array_equal(Zs, Z1)
    np.testing.assert_allclose(Ds, D1 / 1024.0, rtol=1e-15)


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("p", [2.0, 8.0])
def test_invariances_within_tolerance(prec, p):
    # Eq. 1 is invariant under a permutation of the data points and commutes with an affine
    # map of the values, Z(a z + b) = a Z + b.  The GPU results may differ by rounding only:
    # the permuted run is held to the tolerance of the summation scale S; the mapped one to
    # the tolerance of S_a + |a| S (S_a the mapped values' scale, which can be far smaller
    # where a z + b crosses zero), plus the rounding of the mapped values themselves.
    x, z, q = rand_case(14, 5000, 1500, 2, prec)
    t = np.float32 if prec == "f32" else np.float64
    ref = oracle.forward(x, z, q, p)
    Z0, _ = gpu_forward(x, z, q, p, "aoas", prec)
    perm = np.random.default_rng(15).permutation(len(x))
    Zp, _ = gpu_forward(x[perm], z[perm], q, p, "aoas", prec)
    assert np.max(np.abs(Zp - Z0) / ref["S"]) <= 2 * TOL[prec]
    a, b = -2.5, 0.75
    za = (a * z + b).astype(t).astype(np.float64)
    Za, _ = gpu_forward(x, za, q, p, "aoas", prec)
    refa = oracle.forward(x, za, q, p)
    scale = refa["S"] + abs(a) * ref["S"]
    assert np.max(np.abs(Za - (a * Z0 + b)) / scale) <= 2 * TOL[prec] + np.finfo(t).eps


def test_large_coordinates_and_offsets():
    x, z, q = rand_case(13, 3000, 500, 2)
    Z, _ = gpu_forward(x * 1e5 + 3e5, z, q * 1e5 + 3e5, 2.0, "aoas", "f64")
    ref = oracle.forward(x * 1e5 + 3e5, z, q * 1e5 + 3e5, 2.0)
    assert np.max(scaled_err(Z, ref)) <= TOL["f64"]
    xs, qs = (x * 1e5).astype(np.float32).astype(np.float64), (q * 1e5).astype(np.float32).astype(np.float64)
    Z, _ = gpu_forward(xs, z, qs, 6.0, "aoas", "f32")
    ref = oracle.forward(xs, z, qs, 6.0)
    assert np.max(scaled_err(Z, ref)) <= TOL["f32"]


def _sample(m, k, seed):
    return np.sort(np.random.default_rng(seed).choice(m, size=k, replace=False))


@pytest.fixture(scope="module")
def plain2d_1m():
    # The benchmark's workload (1,048,576 x 1,048,576, 2-D, p = 2) and the oracle on 4,096
    # queries sampled by seed, evaluated one by one (in parallel over query slices).
    cfg = workloads.WORKLOADS["plain2d_f32_1m"]
    x, z, q, _ = workloads.plain2d(cfg["n"], cfg["m"], "f32", cfg=cfg["cfg"])
    idx = _sample(len(q), 4096, 1)
    return x, z, q, idx, oracle_forward_par(x, z, q[idx], 2.0)


@pytest.mark.parametrize("prec,layout", [("f32", l) for l in LAYOUTS] + [("f64", "aoas")])
def test_full_size_plain2d_1m_sampled(prec, layout, plain2d_1m):
    # FP32 in every record layout and FP64 (whose forward finishes in the sweep kernel at
    # this size: one data chunk), in the launch configuration of the benchmark.  Both error
    # measures: relative to the summation scale on every sampled query, and plain relative
    # error where |Z| >= 0.1 max|z|.
    x, z, q, idx, ref = plain2d_1m
    print(f"full-size plain2d prec={prec} layout={layout}", flush=True)
    Z, D = gpu_forward(x, z, q, 2.0, layout, prec)
    assert np.max(scaled_err(Z[idx], ref)) <= TOL[prec]
    pr = plain_rel_err(Z[idx], ref, z)
    assert pr.size > 1000 and np.max(pr) <= PLAIN_TOL[prec], f"plain relative error {np.max(pr):.3e}"
    np.testing.assert_allclose(D[idx], ref["D"], rtol=1e-5 if prec == "f32" else 1e-12)
    assert np.all(np.isfinite(Z))


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_full_size_plain2d_1m_adjoint_sparse_upstream(prec, plain2d_1m):
    # The full-size adjoint (dz, dp, dq) in the benchmark's launch configuration, with the
    # upstream gradient non-zero on the 4,096 sampled queries only: dz and dp are then sums
    # over those queries alone, which the oracle evaluates exactly.  Every workgroup group of
    # the fused sweep folds 4 query blocks (FP64: 8) into its dz row at this size.
    x, z, q, idx, _ = plain2d_1m
    t = np.float32 if prec == "f32" else np.float64
    g = np.zeros(len(q))
    g[idx] = np.random.default_rng(2).normal(size=len(idx)).astype(t)
    d, qq = points(x, z, q, "aoas", prec)
    print(f"full-size plain2d adjoint prec={prec}", flush=True)
    Z, D = api.forward(d, qq, 2.0, prec)
    gt = torch.tensor(g, dtype=torch.float32 if prec == "f32" else torch.float64, device="cuda")
    dz, dp, dq = api.backward(d, qq, 2.0, gt, Z, D, prec)
    torch.cuda.synchronize()
    ref = oracle_backward_par(x, z, q[idx], 2.0, g[idx])
    tol = GTOL[prec]
    dzh = dz.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(dzh - ref["dz"]) / ref["dz_scale"]) <= tol
    ec, es = dp_errors(float(dp), ref)
    assert ec <= tol and es <= tol
    dqh = dq.cpu().numpy().astype(np.float64)
    ec, es = dq_errors(dqh[idx], ref)
    assert np.max(ec) <= tol, f"dq err {np.max(ec):.3e}"
    assert es.size > 100 and np.max(es) <= tol, f"dq err (centred scale) {np.max(es):.3e}"
    rest = np.setdiff1d(np.arange(len(q)), idx)
    assert np.all(dqh[rest] == 0.0)


def test_full_size_mixture3d_hits_and_fp32_vs_fp64():
    cfg = workloads.WORKLOADS["mixture3d_p2.5_262k_1m"]
    x, z, q, hit_rows = workloads.mixture3d(cfg["n"], cfg["m"], cfg["hits"], "f32", cfg=cfg["cfg"])
    print("full-size mixture3d", flush=True)
    Z32, _ = gpu_forward(x, z, q, 2.5, "aoas", "f32")
    Z64, _ = gpu_forward(x, z, q, 2.5, "aoas", "f64")
    # every exact hit returns its data value
    ref_h = oracle.forward(x, z, q[hit_rows], 2.5)
    assert np.all(ref_h["H"] >= 1)
    np.testing.assert_array_equal(Z32[hit_rows], ref_h["Z"].astype(np.float32).astype(np.float64))
    np.testing.assert_array_equal(Z64[hit_rows], ref_h["Z"])
    idx = _sample(len(q), 4096, 2)
    ref = oracle_forward_par(x, z, q[idx], 2.5)
    assert np.max(scaled_err(Z32[idx], ref)) <= TOL["f32"]
    assert np.max(scaled_err(Z64[idx], ref)) <= TOL["f64"]
    for Zp, prec in ((Z32, "f32"), (Z64, "f64")):
        pr = plain_rel_err(Zp[idx], ref, z)
        assert pr.size > 1000 and np.max(pr) <= PLAIN_TOL[prec], f"{prec} plain relative error {np.max(pr):.3e}"
    # FP32 path against the GPU FP64 path for every query
    rel = np.abs(Z32 - Z64) / np.maximum(np.abs(Z64), 1e-3)
    assert np.max(rel) <= 1e-5


@pytest.fixture(scope="module")
def plain2d_10k():
    cfg = workloads.WORKLOADS["plain2d_f64_10k"]
    x, z, q, _ = workloads.plain2d(cfg["n"], cfg["m"], "f64", cfg=cfg["cfg"])
    return x, z, q, oracle.forward(x, z, q, 2.0)


@pytest.mark.parametrize("layout", ["soa", "aos", "aoas", "hybrid", "soaos"])
def test_full_size_plain2d_f64_10k_every_query(layout, plain2d_10k):
    # 10,240 x 10,240 FP64, p = 2: the oracle evaluates every query.
    x, z, q, ref = plain2d_10k
    Z, D = gpu_forward(x, z, q, 2.0, layout, "f64")
    assert np.max(scaled_err(Z, ref)) <= TOL["f64"]
    pr = plain_rel_err(Z, ref, z)
    assert pr.size > 2000 and np.max(pr) <= PLAIN_TOL["f64"]
    np.testing.assert_allclose(D, ref["D"], rtol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_collinear_data_and_far_offsets(dim):
    # Data on a line (every coordinate but the first constant), queries off it: the extent
    # comes from one axis only.
    r = np.random.default_rng(14)
    n, m = 2000, 400
    x = np.zeros((n, dim))
    x[:, 0] = r.random(n)
    x[:, 1:] = 0.3
    z = np.sin(4 * x[:, 0]) + r.normal(0, 0.1, n)
    q = r.random((m, dim))
    q[:5] = x[:5]
    x, z, q = (a.astype(np.float32).astype(np.float64) for a in (x, z, q))
    Z, _ = gpu_forward(x, z, q, 2.0, "aoas", "f32")
    ref = oracle.forward(x, z, q, 2.0)
    assert np.max(scaled_err(Z, ref)) <= TOL["f32"]
    # FP32 records far from the origin (offset 1e6, extent 1e3): differences of nearby
    # coordinates are exact, so the FP32 sweep keeps its accuracy without centring.
    x2 = (1e6 + 1e3 * r.random((n, dim))).astype(np.float32).astype(np.float64)
    q2 = (1e6 + 1e3 * r.random((m, dim))).astype(np.float32).astype(np.float64)
    z2 = r.normal(size=n).astype(np.float32).astype(np.float64)
    Z2, _ = gpu_forward(x2, z2, q2, 2.0, "aoas", "f32")
    ref2 = oracle.forward(x2, z2, q2, 2.0)
    assert np.max(scaled_err(Z2, ref2)) <= TOL["f32"]
