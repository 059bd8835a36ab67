"""The pins catch plausible mistakes: each case plants one in a copy of the oracle's C source
(a dropped coordinate, a wrong exponent, a wrong hit count, a missing factor, a flipped
difference), builds it with gcc in a temporary directory, and checks that the pin battery
below rejects it, while the unmodified oracle passes the same battery.

The battery restates pins from the other oracle tests (closed forms, exact hits, decimal
brute force of the forward, 80-digit finite differences of every gradient, the dz sum rule,
and the condition scales pinned from above: equal to what they bound where every term has
one sign, closed forms on a constant field) so that one failure anywhere fails it."""
import os

import numpy as np
import pytest

import oracle
from oracle import exact

SRC = os.path.join(os.path.dirname(oracle.__file__), "idw_oracle.c")

# (name, text to replace, replacement): each must occur exactly once in the source.
MUTANTS = [
    ("dropped coordinate", "for (int k = 0; k < dim; ++k) {\n    double d = a[k] - b[k];",
     "for (int k = 1; k < dim; ++k) {\n    double d = a[k] - b[k];"),
    ("weight r2^-p", "return pow(r2, -0.5 * p);", "return pow(r2, -p);"),
    ("hit count off by one", "Zi = nval(&hz) / (double)h;", "Zi = nval(&hz) / (double)(h + 1);"),
    ("dq without 1/r2", "double u = (w / r2) * c;", "double u = w * c;"),
    ("dp without the 1/2", "double lp = w * 0.5 * log(r2) * c;", "double lp = w * log(r2) * c;"),
    ("dq difference flipped", "double dk = qi[k] - xj[k];", "double dk = xj[k] - qi[k];"),
    ("dx difference flipped", "const double e = qi[k] - xj[k];", "const double e = xj[k] - qi[k];"),
    ("dz without 1/D", "nadd(&dzs[j], gi * w / Di);", "nadd(&dzs[j], gi * w);"),
    # the condition scales, denominators of every parity tolerance: a stray factor in any of
    # them would loosen the GPU tests while every other pin still passed
    ("forward scale doubled", "nadd(&sab, w * fabs(z[j]));", "nadd(&sab, 2.0 * w * fabs(z[j]));"),
    ("dz scale doubled", "nadd(&dza[j], fabs(gi) * w / Di);", "nadd(&dza[j], 2.0 * fabs(gi) * w / Di);"),
    ("dp scale doubled", "nadd(&Pa, fabs(lp));", "nadd(&Pa, 2.0 * fabs(lp));"),
    ("dp condition doubled", "nadd(&Pc, fabs(w * 0.5 * log(r2)) * cabs);",
     "nadd(&Pc, 2.0 * fabs(w * 0.5 * log(r2)) * cabs);"),
    ("dq scale doubled", "nadd(&Ga, fabs(u) * ua);", "nadd(&Ga, 2.0 * fabs(u) * ua);"),
    ("dq condition doubled", "nadd(&Gc, (w / r2) * cabs * ua);", "nadd(&Gc, 2.0 * (w / r2) * cabs * ua);"),
    ("dx condition doubled", "nadd(&cnd[j], fabs(a) * f * (fabs(z[j]) + fabs(Zi)) * ea);",
     "nadd(&cnd[j], 2.0 * fabs(a) * f * (fabs(z[j]) + fabs(Zi)) * ea);"),
]


def _battery(lib):
    r = np.random.default_rng(31)
    # constant field
    x = r.random((40, 2))
    q = r.random((9, 2))
    out = oracle.forward(x, np.full(40, 0.7), q, 2.5, lib=lib)
    np.testing.assert_allclose(out["Z"], 0.7, rtol=1e-14)
    # a linear field on a symmetric 8-point stencil is reproduced exactly
    h = 0.125
    st = np.array([[h, 0], [-h, 0], [0, h], [0, -h], [h, h], [-h, -h], [h, -h], [-h, h]])
    c = np.array([0.5, 0.25])
    out = oracle.forward(c + st, 1.5 + 2.0 * (c + st)[:, 0] - 3.0 * (c + st)[:, 1], c[None, :], 2.0, lib=lib)
    np.testing.assert_allclose(out["Z"], [1.5 + 2.0 * c[0] - 3.0 * c[1]], rtol=1e-14)
    # two points, both coordinates differing: Z = (z0 d1^p + z1 d0^p) / (d0^p + d1^p)
    x2 = np.array([[0.3, 0.1], [-0.2, 0.6]])
    z2 = np.array([1.0, -2.0])
    q2 = np.array([[0.05, 0.2]])
    d0, d1 = np.linalg.norm(x2 - q2, axis=1)
    p = 2.5
    out = oracle.forward(x2, z2, q2, p, lib=lib)
    np.testing.assert_allclose(out["Z"], [(z2[0] * d1 ** p + z2[1] * d0 ** p) / (d0 ** p + d1 ** p)], rtol=1e-14)
    # an exact hit on a duplicated point returns the mean of the coincident values
    x3 = r.random((10, 2))
    x3[7] = x3[2]
    z3 = r.normal(size=10)
    out = oracle.forward(x3, z3, x3[2:3], 2.0, lib=lib)
    assert out["Z"][0] == pytest.approx((z3[2] + z3[7]) / 2, rel=1e-15)
    # decimal brute force of the forward on 8 points
    x8 = r.random((8, 3))
    z8 = r.normal(size=8)
    q8 = r.random((3, 3))
    ref = exact.forward_decimal(x8, z8, q8, "1.7")
    out = oracle.forward(x8, z8, q8, 1.7, lib=lib)
    np.testing.assert_allclose(out["Z"], [float(v) for v in ref], rtol=1e-14)
    # every gradient against 80-digit central differences of the exact forward
    x6 = r.random((6, 3)).astype(np.float32).astype(np.float64)
    z6 = r.normal(size=6)
    q6 = r.random((3, 3)).astype(np.float32).astype(np.float64)
    g6 = r.normal(size=3)
    fd = exact.gradients_fd([tuple(v) for v in x6], z6, [tuple(v) for v in q6], "2.5", g6)
    an = oracle.backward(x6, z6, q6, 2.5, g6, lib=lib)
    np.testing.assert_allclose(an["dz"], fd["dz"], rtol=1e-11, atol=1e-13)
    np.testing.assert_allclose(an["dq"], np.array(fd["dq"]), rtol=1e-10, atol=1e-12)
    assert an["dp"] == pytest.approx(fd["dp"], rel=1e-10, abs=1e-13)
    ax = oracle.backward_x(x6, z6, q6, 2.5, g6, lib=lib)
    np.testing.assert_allclose(ax["dx"], np.array(fd["dx"]), rtol=1e-10, atol=1e-12)
    # the value gradients of each query sum to its upstream gradient
    xb = r.random((50, 2))
    gb = r.normal(size=12)
    bb = oracle.backward(xb, r.normal(size=50), r.random((12, 2)), 2.0, gb, lib=lib)
    assert np.sum(bb["dz"]) == pytest.approx(np.sum(gb), rel=1e-13)
    # the condition scales from above: equal to the quantity they bound where every term
    # has one sign, and closed forms on a constant field (four points at distance h)
    zp = np.abs(r.normal(size=50))
    qp = r.random((12, 2))
    qp[0] = xb[3]
    out = oracle.forward(xb, zp, qp, 1.7, lib=lib)
    np.testing.assert_array_equal(out["S"], out["Z"])
    bp = oracle.backward(xb, zp, qp, 1.7, np.abs(gb), lib=lib)
    np.testing.assert_array_equal(bp["dz_scale"], bp["dz"])
    bs = oracle.backward(np.array([[-0.5, 0.0], [2.0, 0.0]]), np.array([1.0, 0.0]), np.zeros((1, 2)), 2.0,
                         np.array([0.8]), lib=lib)
    assert bs["dp_scale"] == bs["dp"] and bs["dq_scale"][0] == abs(bs["dq"][0, 0])
    h, cv, gv, pv = 0.375, -1.25, 0.6, 2.5
    qc = np.array([[0.3, -0.1]])
    xc = qc + np.array([[h, 0.0], [-h, 0.0], [0.0, h], [0.0, -h]])
    bc = oracle.backward(xc, np.full(4, cv), qc, pv, np.array([gv]), lib=lib)
    assert bc["dq_cond"][0] == pytest.approx(2 * pv * gv * abs(cv) / h, rel=1e-14)
    assert bc["dp_cond"] == pytest.approx(2 * gv * abs(cv) * abs(np.log(h)), rel=1e-14)
    xcnd = oracle.backward_x(xc, np.full(4, cv), qc, pv, np.array([gv]), lib=lib)["dx_cond"]
    np.testing.assert_allclose(xcnd, pv * gv * abs(cv) / (2 * h), rtol=1e-14)


def test_unmodified_oracle_passes_the_battery():
    _battery(None)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_fails_the_battery(tmp_path, name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site of '{name}' not unique"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    lib = oracle.load_library(oracle.compile_source(str(path), str(tmp_path / "libmutant.so")))
    with pytest.raises(AssertionError):
        _battery(lib)
