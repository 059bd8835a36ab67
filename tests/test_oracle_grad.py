"""Pins of the oracle's analytic adjoint against high-precision finite differences of
the forward (Section 2.1, Eq. 1 differentiated), plus conservation laws of the gradient.
"""
import numpy as np
import pytest

import oracle
from oracle import exact


def _case(seed, n=6, m=3, dim=2, hit=False):
    r = np.random.default_rng(3000 + seed)
    x = r.random((n, dim)).astype(np.float32).astype(np.float64)
    z = r.normal(size=n).astype(np.float32).astype(np.float64)
    q = r.random((m, dim)).astype(np.float32).astype(np.float64)
    g = r.normal(size=m)
    if hit:
        q[0] = x[2]
    return x, z, q, g


@pytest.mark.parametrize("p,dim,hit", [("2", 2, False), ("2.5", 3, False), ("1.5", 2, True), ("3", 3, True)])
def test_analytic_gradient_matches_decimal_finite_differences(p, dim, hit):
    x, z, q, g = _case(int(float(p) * 10) + dim, dim=dim, hit=hit)
    fd = exact.gradients_fd([tuple(r) for r in x], z, [tuple(r) for r in q], p, g)
    an = oracle.backward(x, z, q, float(p), g)
    np.testing.assert_allclose(an["dz"], fd["dz"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(an["dq"], np.array(fd["dq"]), rtol=1e-11, atol=1e-12)
    assert an["dp"] == pytest.approx(fd["dp"], rel=1e-11, abs=1e-13)
    ax = oracle.backward_x(x, z, q, float(p), g)
    np.testing.assert_allclose(ax["dx"], np.array(fd["dx"]), rtol=1e-11, atol=1e-12)


def test_value_gradient_sums_to_upstream_gradient():
    # Weights are normalised, so sum_j dZ_i/dz_j = 1 for every query.
    x, z, q, g = _case(21, n=80, m=30, dim=3)
    an = oracle.backward(x, z, q, 2.0, g)
    assert np.sum(an["dz"]) == pytest.approx(np.sum(g), rel=1e-13)


def test_constant_field_has_no_position_or_power_gradient():
    x, _, q, g = _case(22, n=50, m=10)
    an = oracle.backward(x, np.full(50, 0.75), q, 2.5, g)
    assert an["dp"] == pytest.approx(0.0, abs=1e-13)
    np.testing.assert_allclose(an["dq"], 0.0, atol=1e-12)


def test_hit_gradient_goes_to_the_coincident_points_only():
    x, z, q, g = _case(23, n=10, m=2)
    x[4] = x[1]
    q[0] = x[1]
    an = oracle.backward(x, z, q[:1], 2.0, g[:1])
    expect = np.zeros(10)
    expect[[1, 4]] = g[0] / 2
    np.testing.assert_allclose(an["dz"], expect, rtol=1e-15, atol=0)
    assert an["dp"] == 0.0
    np.testing.assert_array_equal(an["dq"], 0.0)


def test_scales_bound_gradients():
    x, z, q, g = _case(24, n=60, m=12, dim=2)
    an = oracle.backward(x, z, q, 2.0, g)
    assert np.all(np.abs(an["dz"]) <= an["dz_scale"] * (1 + 1e-14))
    assert abs(an["dp"]) <= an["dp_scale"] * (1 + 1e-14)
    assert np.all(np.max(np.abs(an["dq"]), axis=1) <= an["dq_scale"] * (1 + 1e-14))
    # the uncentred condition sums dominate the centred ones: |z - Z| <= |z| + |Z|
    assert np.all(an["dq_scale"] <= an["dq_cond"] * (1 + 1e-14))
    assert an["dp_scale"] <= an["dp_cond"] * (1 + 1e-14)


def test_value_scale_equals_the_value_gradient_for_nonnegative_upstream():
    # dz_scale_j = sum_i |g_i| w_ij / D_i (1/h at a hit): with every g_i >= 0 its terms are
    # those of dz_j, added in the same order, so the two are equal bit for bit.  A stray
    # factor in the scale, which would loosen every dz tolerance, fails here.
    x, z, q, g = _case(28, n=60, m=15, dim=3, hit=True)
    x[9] = x[2]                      # the hit query meets a duplicated point
    g = np.abs(g)
    an = oracle.backward(x, z, q, 2.5, g)
    np.testing.assert_array_equal(an["dz_scale"], an["dz"])


def test_centred_scales_equal_the_gradients_when_every_term_has_one_sign():
    # q at the origin, x1 = (-1/2, 0) with z1 = 1, x2 = (2, 0) with z2 = 0, g > 0.  Z lies
    # strictly between z2 and z1, so z1 - Z > 0 > z2 - Z; ln r2 is ln(1/4) < 0 for x1 and
    # ln 4 > 0 for x2; q - x is +1/2 and -2 along x and 0 along y.  Every term of the power
    # sum w ln(r2)(z - Z) is then negative and every term of the position sum
    # (w / r2)(z - Z)(q - x) positive, so the centred scales (sums of absolute terms) equal
    # |dp| and |dq_x| exactly.
    x = np.array([[-0.5, 0.0], [2.0, 0.0]])
    z = np.array([1.0, 0.0])
    q = np.array([[0.0, 0.0]])
    for p in (1.0, 2.0, 2.5):
        an = oracle.backward(x, z, q, p, np.array([0.8]))
        assert an["dp"] > 0 and an["dp_scale"] == an["dp"]
        assert an["dq"][0, 1] == 0.0
        assert an["dq_scale"][0] == abs(an["dq"][0, 0])


@pytest.mark.parametrize("p", [1.0, 2.5])
def test_condition_scales_closed_form_on_a_constant_field(p):
    # Four points at distance h around q (on the axes), every value c: Z = c, D = 4 h^-p.
    # The uncentred sums take |z_j| + |Z| = 2|c| for every term:
    #   dq_cond = |p g / D| * 4 (h^-p / h^2) 2|c| h = 2 p |g| |c| / h,
    #   dp_cond = |g / D| * 4 h^-p |ln h| 2|c|    = 2 |g| |c| |ln h|,
    #   dx_cond_j = |p g / D| (h^-p / h^2) 2|c| h = p |g| |c| / (2 h)  for each point,
    # while the centred dq and dp scales vanish (z - Z = 0).
    h, c, g = 0.375, -1.25, 0.6
    qc = np.array([0.3, -0.1])
    x = qc + np.array([[h, 0.0], [-h, 0.0], [0.0, h], [0.0, -h]])
    z = np.full(4, c)
    an = oracle.backward(x, z, qc[None, :], p, np.array([g]))
    assert an["dq_cond"][0] == pytest.approx(2 * p * abs(g) * abs(c) / h, rel=1e-14)
    assert an["dp_cond"] == pytest.approx(2 * abs(g) * abs(c) * abs(np.log(h)), rel=1e-14)
    assert an["dq_scale"][0] == 0.0 and an["dp_scale"] == 0.0
    ax = oracle.backward_x(x, z, qc[None, :], p, np.array([g]))
    np.testing.assert_allclose(ax["dx_cond"], p * abs(g) * abs(c) / (2 * h), rtol=1e-14)


def test_leave_one_out_equals_explicit_deletion():
    r = np.random.default_rng(25)
    n = 48
    x = r.random((n, 2))
    z = r.normal(size=n)
    idx = np.arange(n)
    loo = oracle.forward(x, z, x, 2.0, self_index=idx)
    g = r.normal(size=n)
    bl = oracle.backward(x, z, x, 2.0, g, self_index=idx)
    dz = np.zeros(n)
    dp = 0.0
    for i in range(n):
        keep = np.array([j for j in range(n) if j != i])
        one = oracle.forward(x[keep], z[keep], x[i:i + 1], 2.0)
        assert loo["Z"][i] == pytest.approx(one["Z"][0], rel=1e-15, abs=1e-15)
        b1 = oracle.backward(x[keep], z[keep], x[i:i + 1], 2.0, g[i:i + 1])
        dz[keep] += b1["dz"]
        dp += b1["dp"]
        np.testing.assert_allclose(bl["dq"][i], b1["dq"][0], rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(bl["dz"], dz, rtol=1e-13, atol=1e-15)
    assert bl["dp"] == pytest.approx(dp, rel=1e-12)


def test_loo_loss_of_constant_field_is_zero():
    r = np.random.default_rng(26)
    x = r.random((40, 2))
    assert oracle.loo_loss(x, np.full(40, 2.0), 1.5) == pytest.approx(0.0, abs=1e-28)


def test_data_coordinate_gradient_two_point_closed_form():
    # q at the origin, x1 = (a, 0), x2 = (-b, 0), p = 2: Z = (z1 b^2 + z2 a^2) / (a^2 + b^2),
    # so dZ/da = 2 a b^2 (z2 - z1) / (a^2 + b^2)^2 and dZ/db = 2 a^2 b (z1 - z2) / (a^2 + b^2)^2
    # (x2's x-coordinate is -b); moving either point across the line changes Z only to
    # second order.
    a, b, z1, z2 = 0.3, 0.7, 1.25, -0.5
    x = np.array([[a, 0.0], [-b, 0.0]])
    z = np.array([z1, z2])
    q = np.array([[0.0, 0.0]])
    r = oracle.backward_x(x, z, q, 2.0, np.array([1.0]))
    s2 = a * a + b * b
    np.testing.assert_allclose(r["dx"][0], [2 * a * b * b * (z2 - z1) / s2 ** 2, 0.0], rtol=1e-14, atol=1e-16)
    np.testing.assert_allclose(r["dx"][1], [-(2 * a * a * b * (z1 - z2) / s2 ** 2), 0.0], rtol=1e-14, atol=1e-16)


@pytest.mark.parametrize("hit", [False, True])
def test_data_and_query_coordinate_gradients_cancel(hit):
    # Z_i depends on the differences q_i - x_j only, so moving every point and every query
    # together changes nothing: sum_j dL/dx_j = -sum_i dL/dq_i.
    x, z, q, g = _case(25, n=70, m=25, dim=3, hit=hit)
    bx = oracle.backward_x(x, z, q, 2.5, g)
    bq = oracle.backward(x, z, q, 2.5, g)
    np.testing.assert_allclose(bx["dx"].sum(axis=0), -bq["dq"].sum(axis=0), rtol=1e-11,
                               atol=1e-13 * np.abs(bx["dx"]).sum())
    assert np.all(bx["dx_cond"] >= np.abs(bx["dx"]).max(axis=1) - 1e-15)


def test_constant_field_has_no_data_coordinate_gradient():
    x, _, q, g = _case(26, n=40, m=9)
    r = oracle.backward_x(x, np.full(40, -1.5), q, 3.0, g)
    np.testing.assert_allclose(r["dx"], 0.0, atol=1e-12)


def test_leave_one_out_data_gradient_matches_explicit_deletion():
    # With queries at the data points and point i left out of query i, dL/dx_j collects
    # from each query i != j the gradient of the interpolant built without point i.
    x, z, _, _ = _case(27, n=12, m=1, dim=2)
    g = np.random.default_rng(7).normal(size=12)
    got = oracle.backward_x(x, z, x, 1.5, g, self_index=np.arange(12))["dx"]
    want = np.zeros_like(x)
    for i in range(12):
        keep = np.array([j for j in range(12) if j != i])
        r = oracle.backward_x(x[keep], z[keep], x[i:i + 1], 1.5, g[i:i + 1])
        want[keep] += r["dx"]
    np.testing.assert_allclose(got, want, rtol=1e-13, atol=1e-15)
