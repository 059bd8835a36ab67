"""Exact and high-precision brute force of Eq. 1 (Section 2.1) for tiny inputs.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Used to pin the C oracle:

* even integer p: every input float is a dyadic rational, so r^2, the weights d^-p and the
  ratio are computed exactly with ``fractions.Fraction``;
* any other p: ``decimal`` arithmetic at 60+ significant digits, with the weight written
  as exp(-(p/2) ln r^2) (correctly rounded ``Decimal.ln``/``Decimal.exp``);
* gradients: central finite differences of the high-precision forward with a step far
  below double precision, so they pin the analytic adjoint without sharing its formulas.

Coordinates are given as sequences of points (tuples), independent of any array layout.
"""
from __future__ import annotations

from decimal import Decimal, localcontext
from fractions import Fraction


def _frac_points(pts):
    return [tuple(Fraction(float(c)) for c in pt) for pt in pts]


def _r2(a, b):
    return sum((ai - bi) * (ai - bi) for ai, bi in zip(a, b))


def forward_fraction(x, z, q, p: int):
    """Exact Eq. 1 for an even integer p (>= 2).  Returns a list of Fractions.

    Exact hits (r^2 == 0) return the mean of the coincident values.
    """
    if p <= 0 or p % 2:
        raise ValueError("forward_fraction needs an even integer p")
    X = _frac_points(x)
    V = [Fraction(float(v)) for v in z]
    out = []
    for qi in _frac_points(q):
        hits = []
        num = Fraction(0)
        den = Fraction(0)
        for xj, vj in zip(X, V):
            r2 = _r2(qi, xj)
            if r2 == 0:
                hits.append(vj)
                continue
            w = 1 / r2 ** (p // 2)
            num += w * vj
            den += w
        out.append(sum(hits, Fraction(0)) / len(hits) if hits else num / den)
    return out


def _dec(v) -> Decimal:
    if isinstance(v, Fraction):
        return Decimal(v.numerator) / Decimal(v.denominator)
    if isinstance(v, Decimal):
        return v
    return Decimal(float(v)) if not isinstance(v, str) else Decimal(v)


def _forward_dec_one(X, V, qi, p: Decimal, skip=None):
    hits = []
    num = Decimal(0)
    den = Decimal(0)
    half_p = p / 2
    for j, (xj, vj) in enumerate(zip(X, V)):
        if skip is not None and j == skip:
            continue
        r2 = sum((a - b) * (a - b) for a, b in zip(qi, xj))
        if r2 == 0:
            hits.append(vj)
            continue
        w = (-half_p * r2.ln()).exp()
        num += w * vj
        den += w
    if hits:
        return sum(hits, Decimal(0)) / len(hits)
    return num / den


def forward_decimal(x, z, q, p, prec: int = 60, self_index=None):
    """Eq. 1 in ``decimal`` at `prec` digits for any p > 0 (given as str/float/Fraction).

    Returns a list of Decimals.
    """
    with localcontext() as ctx:
        ctx.prec = prec
        X = [tuple(_dec(c) for c in pt) for pt in x]
        V = [_dec(v) for v in z]
        P = _dec(p)
        out = []
        for i, qi in enumerate(q):
            qd = tuple(_dec(c) for c in qi)
            skip = None if self_index is None else int(self_index[i])
            out.append(+_forward_dec_one(X, V, qd, P, skip))
        return out


def gradients_fd(x, z, q, p, g, prec: int = 80, h: str = "1e-28"):
    """Central finite differences of sum_i g_i Z_i in `prec`-digit decimal.

    Returns dict(dz=[n], dp=scalar, dq=[m][dim], dx=[n][dim]) as floats.  Truncation
    error is about h^2 times the third derivative, far below double precision for
    h = 1e-28.
    """
    with localcontext() as ctx:
        ctx.prec = prec
        H = Decimal(h)
        X = [tuple(_dec(c) for c in pt) for pt in x]
        V = [_dec(v) for v in z]
        Q = [tuple(_dec(c) for c in pt) for pt in q]
        G = [_dec(v) for v in g]
        P = _dec(p)

        def loss(Xv, Vv, Qv, Pv):
            return sum(gi * _forward_dec_one(Xv, Vv, qi, Pv) for gi, qi in zip(G, Qv))

        dz = []
        for j in range(len(V)):
            vp = list(V)
            vm = list(V)
            vp[j] += H
            vm[j] -= H
            dz.append(float((loss(X, vp, Q, P) - loss(X, vm, Q, P)) / (2 * H)))
        dp = float((loss(X, V, Q, P + H) - loss(X, V, Q, P - H)) / (2 * H))
        dq = []
        for i in range(len(Q)):
            row = []
            for k in range(len(Q[i])):
                qp = list(Q)
                qm = list(Q)
                a = list(Q[i])
                b = list(Q[i])
                a[k] += H
                b[k] -= H
                qp[i] = tuple(a)
                qm[i] = tuple(b)
                row.append(float((loss(X, V, qp, P) - loss(X, V, qm, P)) / (2 * H)))
            dq.append(row)
        dx = []
        for j in range(len(X)):
            row = []
            for k in range(len(X[j])):
                xp = list(X)
                xm = list(X)
                a = list(X[j])
                b = list(X[j])
                a[k] += H
                b[k] -= H
                xp[j] = tuple(a)
                xm[j] = tuple(b)
                row.append(float((loss(xp, V, Q, P) - loss(xm, V, Q, P)) / (2 * H)))
            dx.append(row)
        return {"dz": dz, "dp": dp, "dq": dq, "dx": dx}
