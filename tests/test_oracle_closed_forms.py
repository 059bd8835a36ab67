"""Pins of the FP64 oracle against closed forms and invariants of Eq. 1 (Section 2.1).

None of these re-types the oracle's formula: each expected value follows from the
mathematics of Shepard's weighting (a constant or linear field reproduced on a symmetric
stencil, the two-point ratio, limits in p, exact hits, invariances).
"""
import numpy as np
import pytest

import oracle


def _rng(s):
    return np.random.default_rng(1000 + s)


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("p", [0.5, 1.0, 2.0, 2.5, 3.0, 6.0])
def test_constant_field_is_reproduced(dim, p):
    # Weights are normalised (Eq. 1 divides by their sum), so z == c gives Z == c.
    r = _rng(1)
    x = r.random((50, dim))
    q = r.random((20, dim))
    c = -3.25
    out = oracle.forward(x, np.full(50, c), q, p)
    assert np.all(np.abs(out["Z"] - c) <= 4e-16 * abs(c))
    assert np.all(out["H"] == 0)


@pytest.mark.parametrize("p", [1.0, 2.0, 3.7])
def test_symmetric_stencil_reproduces_linear_field_2d(p):
    # 8 points at (+-h,0), (0,+-h), (+-h,+-h) around q: opposite points carry equal
    # weights, so a linear field a + b x + c y averages to its value at q.
    h = 0.125
    qc = np.array([0.375, 0.625])
    offs = np.array([[h, 0], [-h, 0], [0, h], [0, -h], [h, h], [-h, -h], [h, -h], [-h, h]])
    x = qc + offs
    a, b, c = 0.5, -1.25, 2.0
    z = a + b * x[:, 0] + c * x[:, 1]
    out = oracle.forward(x, z, qc[None, :], p)
    assert abs(out["Z"][0] - (a + b * qc[0] + c * qc[1])) < 1e-15


@pytest.mark.parametrize("p", [2.0, 2.5])
def test_symmetric_stencil_reproduces_linear_field_3d(p):
    h = 0.25
    qc = np.array([0.5, 0.25, 0.75])
    offs = [np.eye(3)[k] * s * h for k in range(3) for s in (1, -1)]
    offs += [np.array([sx, sy, sz]) * h for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)]
    x = qc + np.array(offs)
    coef = np.array([0.75, -2.0, 1.5])
    z = 0.125 + x @ coef
    out = oracle.forward(x, z, qc[None, :], p)
    assert abs(out["Z"][0] - (0.125 + qc @ coef)) < 1e-15


def test_equidistant_points_give_the_plain_mean():
    # Four points at the same distance carry identical weights: Z is their mean, and the
    # denominator is 4 d^-p.
    qc = np.array([0.5, 0.5])
    x = qc + 0.25 * np.array([[1, 0], [-1, 0], [0, 1], [0, -1]])
    z = np.array([1.0, 2.0, 4.0, 8.0])
    out = oracle.forward(x, z, qc[None, :], 3.0)
    assert out["Z"][0] == pytest.approx(15.0 / 4.0, rel=1e-15)
    assert out["D"][0] == pytest.approx(4 * 0.25 ** -3.0, rel=1e-15)


@pytest.mark.parametrize("p", [0.7, 2.0, 3.0])
def test_two_point_closed_form(p):
    # Z = (z0 d1^p + z1 d0^p) / (d0^p + d1^p) for two data points.
    x = np.array([[0.0, 0.0], [1.0, 0.5]])
    z = np.array([1.5, -0.5])
    q = np.array([[0.3, 0.1], [0.9, 0.9], [-2.0, 3.0]])
    d0 = np.hypot(q[:, 0] - x[0, 0], q[:, 1] - x[0, 1])
    d1 = np.hypot(q[:, 0] - x[1, 0], q[:, 1] - x[1, 1])
    expect = (z[0] * d1 ** p + z[1] * d0 ** p) / (d0 ** p + d1 ** p)
    out = oracle.forward(x, z, q, p)
    np.testing.assert_allclose(out["Z"], expect, rtol=1e-14)


def test_exact_hits_return_data_values_and_duplicates_average():
    r = _rng(2)
    x = r.random((30, 2))
    z = r.normal(size=30)
    x[7] = x[3]          # duplicate location with a different value
    q = x[[0, 3, 12, 29]]
    out = oracle.forward(x, z, q, 2.0)
    assert out["Z"][0] == z[0]
    assert out["Z"][1] == (z[3] + z[7]) / 2
    assert out["Z"][2] == z[12]
    assert out["Z"][3] == z[29]
    assert list(out["H"]) == [1, 2, 1, 1]


def test_small_p_limit_is_the_mean():
    # As p -> 0 every weight tends to 1: Z tends to the arithmetic mean of z.
    r = _rng(3)
    x = r.random((40, 2))
    z = r.normal(size=40)
    q = r.random((5, 2))
    out = oracle.forward(x, z, q, 1e-9)
    np.testing.assert_allclose(out["Z"], np.mean(z), rtol=0, atol=1e-7)


def test_large_p_limit_is_the_nearest_value():
    # For large p the nearest point dominates: (d_near/d_other)^p vanishes.
    r = _rng(4)
    x = r.random((40, 2))
    z = r.normal(size=40)
    q = r.random((8, 2))
    d = np.linalg.norm(q[:, None, :] - x[None, :, :], axis=2)
    ds = np.sort(d, axis=1)
    keep = ds[:, 0] / ds[:, 1] < 0.8
    out = oracle.forward(x, z, q[keep], 200.0)
    np.testing.assert_allclose(out["Z"], z[np.argmin(d[keep], axis=1)], rtol=0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_data_permutation_invariance(dim):
    r = _rng(5)
    x = r.random((300, dim))
    z = r.normal(size=300)
    q = r.random((25, dim))
    a = oracle.forward(x, z, q, 2.5)
    perm = r.permutation(300)
    b = oracle.forward(x[perm], z[perm], q, 2.5)
    np.testing.assert_allclose(a["Z"], b["Z"], rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(a["D"], b["D"], rtol=1e-15)


def test_affine_value_map_and_power_of_two_scaling():
    r = _rng(6)
    x = r.random((200, 2))
    z = r.normal(size=200)
    q = r.random((30, 2))
    base = oracle.forward(x, z, q, 2.0)
    # Z(a z + b) = a Z(z) + b, since the weights sum to one.
    aff = oracle.forward(x, 3.0 * z - 0.5, q, 2.0)
    np.testing.assert_allclose(aff["Z"], 3.0 * base["Z"] - 0.5, rtol=1e-14, atol=1e-14)
    # Scaling every coordinate by 4 scales all weights by 4^-p: Z is unchanged, D scales.
    sc = oracle.forward(4.0 * x, z, 4.0 * q, 2.0)
    np.testing.assert_allclose(sc["Z"], base["Z"], rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(sc["D"], base["D"] / 16.0, rtol=1e-15)
    # A translation changes nothing but rounding.
    tr = oracle.forward(x + np.array([0.25, -0.5]), z, q + np.array([0.25, -0.5]), 2.0)
    np.testing.assert_allclose(tr["Z"], base["Z"], rtol=1e-12, atol=1e-12)


def test_scale_bounds_the_result():
    r = _rng(7)
    x = r.random((100, 3))
    z = r.normal(size=100)
    q = r.random((40, 3))
    out = oracle.forward(x, z, q, 2.5)
    assert np.all(np.abs(out["Z"]) <= out["S"] * (1 + 1e-15))
    assert np.all(out["S"] <= np.max(np.abs(z)) * (1 + 1e-15))
    # Eq. 1 is a convex combination: min z <= Z <= max z.
    assert np.all(out["Z"] >= z.min() - 1e-15) and np.all(out["Z"] <= z.max() + 1e-15)


def test_scale_equals_the_result_for_nonnegative_values_and_two_point_form():
    # S = sum w |z| / sum w: with every z >= 0 its sum is the numerator's, term by term, so
    # S equals Z bit for bit; at a hit it is |Z|.  On two points with values of both signs it
    # has the closed form (|z0| d1^p + |z1| d0^p) / (d0^p + d1^p).  (S is the denominator of
    # every forward tolerance, so it is pinned from above as well as below.)
    r = _rng(8)
    x = r.random((90, 2))
    z = np.abs(r.normal(size=90))
    q = r.random((30, 2))
    q[0] = x[5]
    out = oracle.forward(x, z, q, 1.7)
    np.testing.assert_array_equal(out["S"], out["Z"])
    x2 = np.array([[0.3, 0.1], [-0.2, 0.6]])
    z2 = np.array([1.5, -2.0])
    q2 = np.array([[0.05, 0.2]])
    d0, d1 = np.linalg.norm(x2 - q2, axis=1)
    for p in (1.0, 2.5):
        out = oracle.forward(x2, z2, q2, p)
        want = (abs(z2[0]) * d1 ** p + abs(z2[1]) * d0 ** p) / (d0 ** p + d1 ** p)
        assert out["S"][0] == pytest.approx(want, rel=1e-14)


def test_bad_arguments_are_rejected():
    x = np.zeros((3, 2))
    with pytest.raises(ValueError):
        oracle.forward(x, np.zeros(3), np.zeros((1, 2)), 0.0)
    with pytest.raises(ValueError):
        oracle.forward(np.zeros((3, 4)), np.zeros(3), np.zeros((1, 4)), 2.0)
