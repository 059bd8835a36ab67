"""Pins of the FP64 oracle against exact / 60-digit brute force on tiny inputs.

Inputs are float32-rounded, i.e. dyadic rationals, so for even p the Fraction brute force
is exact; for other p the decimal brute force is correct to ~60 digits.  A transposed
operand, a dropped coordinate, a wrong exponent or a wrong hit rule in the C loop would
all fail here.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import exact


def _case(seed, n=8, m=6, dim=2, hit=True):
    r = np.random.default_rng(2000 + seed)
    x = r.random((n, dim)).astype(np.float32).astype(np.float64)
    z = r.normal(size=n).astype(np.float32).astype(np.float64)
    q = r.random((m, dim)).astype(np.float32).astype(np.float64)
    if hit:
        q[1] = x[5]
    return x, z, q


@pytest.mark.parametrize("p", [2, 4, 6])
@pytest.mark.parametrize("dim", [2, 3])
def test_fraction_brute_force_even_p(p, dim):
    x, z, q = _case(p + dim, dim=dim)
    want = exact.forward_fraction([tuple(r) for r in x], z, [tuple(r) for r in q], p)
    got = oracle.forward(x, z, q, float(p))["Z"]
    for g, w in zip(got, want):
        assert abs(Fraction(g) - w) <= abs(w) * Fraction(1, 10 ** 15) + Fraction(1, 10 ** 300)


@pytest.mark.parametrize("p", ["1", "2.5", "3", "1.7", "0.5"])
@pytest.mark.parametrize("dim", [2, 3])
def test_decimal_brute_force_any_p(p, dim):
    x, z, q = _case(len(p) + dim, dim=dim)
    want = exact.forward_decimal([tuple(r) for r in x], z, [tuple(r) for r in q], p)
    got = oracle.forward(x, z, q, float(p))["Z"]
    for g, w in zip(got, want):
        assert abs(g - float(w)) <= 2e-15 * max(abs(float(w)), 1e-300) + 1e-300


def test_fraction_and_decimal_brute_force_agree():
    # Two independent exact routes must agree to ~60 digits (pins the decimal route).
    x, z, q = _case(9)
    a = exact.forward_fraction([tuple(r) for r in x], z, [tuple(r) for r in q], 2)
    b = exact.forward_decimal([tuple(r) for r in x], z, [tuple(r) for r in q], 2, prec=70)
    for fa, db in zip(a, b):
        assert abs(float(fa) - float(db)) <= 1e-300 + 1e-50 * abs(float(fa))
        assert abs(Fraction(db) - fa) <= abs(fa) * Fraction(1, 10 ** 55)


def test_self_index_matches_decimal_deletion():
    x, z, q = _case(11, n=8, m=8, hit=False)
    q = x.copy()
    idx = np.arange(8)
    got = oracle.forward(x, z, q, 2.5, self_index=idx)["Z"]
    for i in range(8):
        keep = [j for j in range(8) if j != i]
        want = exact.forward_decimal([tuple(x[j]) for j in keep], z[keep], [tuple(q[i])], "2.5")[0]
        assert abs(got[i] - float(want)) <= 2e-15 * abs(float(want))
