"""Seeded synthetic inputs for the IDW workloads, plus host-side layout packing.

This module holds no interpolation arithmetic: it only draws points and values and packs
them into the record layouts of Sections 3.1-3.5 (SoA, AoS, aligned AoS, SoAoS, hybrid
AoS + array of values).  Both the oracle side and the GPU side of the tests read their
inputs from here, so they see bit-identical numbers.

Recipes (the paper names no dataset; it fixes only n = m in {10K .. 1000K}, 1K = 1024,
and p = 2, Section 4.1).  Every generator draws in float64 from
``numpy.random.default_rng(SeedSequence(14024986 + cfg))`` and, for float32 workloads,
rounds to float32 once; the rounded values are what every consumer sees.

* plain2d      2-D, x, q ~ U[0,1]^2, z = sin(2 pi x) cos(2 pi y) + N(0, 0.01^2).
* mixture3d    3-D data from a 16-component isotropic Gaussian mixture (equal weights,
               centres ~ U[0.1, 0.9]^3, sigma 0.02, draws outside the unit cube redrawn),
               z = exp(-|x - c|^2) + N(0, 0.01^2), c = (0.5, 0.5, 0.5); queries uniform
               in the cube with a given number of bit-exact copies of distinct data points,
               shuffled in.
* batched      independent instances: dim ~ U{2,3}, p ~ U{1,2,3}, n ~ logU[nlo, nhi],
               m ~ logU[mlo, mhi]; uniform coordinates; the plain2d / mixture3d value fields.
"""
from __future__ import annotations

import numpy as np

SEED_BASE = 14024986

LAYOUTS = ("soa", "aos", "aoas", "hybrid", "soaos")

# Named workloads: (n data points, m queries, dim, p, dtype).
WORKLOADS = {
    "plain2d_f64_10k": dict(cfg=0, n=10240, m=10240, dim=2, p=2.0, dtype="f64"),
    "plain2d_f32_1m": dict(cfg=1, n=1048576, m=1048576, dim=2, p=2.0, dtype="f32"),
    "mixture3d_p2.5_262k_1m": dict(cfg=2, n=262144, m=1048576, dim=3, p=2.5, dtype="f32", hits=1024),
    "plain2d_grad_f32_128k": dict(cfg=3, n=131072, m=131072, dim=2, p=1.5, dtype="f32"),
}


def rng_for(cfg: int, stream: int = 0) -> np.random.Generator:
    ss = np.random.SeedSequence(SEED_BASE + cfg)
    return np.random.default_rng(ss.spawn(stream + 1)[stream])


def _round(a: np.ndarray, dtype: str) -> np.ndarray:
    if dtype != "f64":  # "f32" and "f32_kahan"
        return a.astype(np.float32).astype(np.float64)
    return a.astype(np.float64)


def field2d(x: np.ndarray) -> np.ndarray:
    return np.sin(2 * np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 1])


def field3d(x: np.ndarray) -> np.ndarray:
    c = np.array([0.5, 0.5, 0.5])
    return np.exp(-np.sum((x - c) ** 2, axis=1))


def plain2d(n: int, m: int, dtype: str = "f32", cfg: int = 0):
    """Uniform 2-D data and queries with the sin*cos field plus N(0, 0.01^2) noise.

    Returns float64 arrays (already rounded to `dtype`): x [n,2], z [n], q [m,2], t [m]
    (the noise-free field at the queries, used as a held-out target).
    """
    r = rng_for(cfg)
    x = r.random((n, 2))
    z = field2d(x) + r.normal(0.0, 0.01, n)
    q = r.random((m, 2))
    x, z, q = _round(x, dtype), _round(z, dtype), _round(q, dtype)
    t = _round(field2d(q), dtype)
    return x, z, q, t


def mixture3d(n: int, m: int, hits: int, dtype: str = "f32", cfg: int = 2):
    """Gaussian-mixture 3-D data, uniform queries with `hits` exact copies of data points."""
    r = rng_for(cfg)
    centres = r.uniform(0.1, 0.9, (16, 3))
    comp = r.integers(0, 16, n)
    x = centres[comp] + r.normal(0.0, 0.02, (n, 3))
    bad = np.any((x < 0) | (x > 1), axis=1)
    while bad.any():
        k = int(bad.sum())
        x[bad] = centres[comp[bad]] + r.normal(0.0, 0.02, (k, 3))
        bad = np.any((x < 0) | (x > 1), axis=1)
    z = field3d(x) + r.normal(0.0, 0.01, n)
    x, z = _round(x, dtype), _round(z, dtype)
    hits = min(hits, n, m)
    q = _round(r.random((m - hits, 3)), dtype)
    pick = r.choice(n, size=hits, replace=False)
    q = np.concatenate([q, x[pick]], axis=0)
    perm = r.permutation(m)
    q = q[perm]
    hit_rows = np.nonzero(perm >= m - hits)[0]
    return x, z, q, hit_rows


def batched(count: int = 64, nlo: int = 1024, nhi: int = 262144, mlo: int = 1024, mhi: int = 524288,
            dtype: str = "f32", cfg: int = 4):
    """List of independent instances: dicts with dim, p, x, z, q (float64, rounded)."""
    r = rng_for(cfg)
    out = []
    for _ in range(count):
        dim = int(r.integers(2, 4))
        p = float(r.integers(1, 4))
        n = int(round(np.exp(r.uniform(np.log(nlo), np.log(nhi)))))
        m = int(round(np.exp(r.uniform(np.log(mlo), np.log(mhi)))))
        x = r.random((n, dim))
        f = field2d(x) if dim == 2 else field3d(x)
        z = f + r.normal(0.0, 0.01, n)
        q = r.random((m, dim))
        out.append(dict(dim=dim, p=p, x=_round(x, dtype), z=_round(z, dtype), q=_round(q, dtype)))
    return out


# ----------------------------------------------------------------------------------------
# Host-side packing into the record layouts.  Each function returns a list of numpy
# arrays, one per pointer slot of the library's point descriptor, in the storage dtype.
# ----------------------------------------------------------------------------------------

def _np_dtype(dtype: str):
    return np.float64 if dtype == "f64" else np.float32  # "f32" and "f32_kahan"


def pack_data(x: np.ndarray, z: np.ndarray, layout: str, dtype: str):
    """Pack data coordinates x [n,dim] and values z [n] into `layout`.

    soa     [x0[], x1[], (x2[]), z[]]
    aos     [records {x0, x1, (x2), z}]                        packed, no padding
    aoas    [records {x0, x1, (x2), z, pad...}]                16 B (f32) / 32 B (f64)
    hybrid  [coords {x0, x1, (x2)} packed, z[]]                AoS + array of values
    soaos   [aligned coords {x0, x1} or {x0, x1, x2, pad}, aligned {z, pad}]
    """
    t = _np_dtype(dtype)
    n, dim = x.shape
    if layout == "soa":
        return [np.ascontiguousarray(x[:, k], dtype=t) for k in range(dim)] + [np.ascontiguousarray(z, dtype=t)]
    if layout == "aos":
        return [np.ascontiguousarray(np.concatenate([x, z[:, None]], axis=1), dtype=t)]
    if layout == "aoas":
        rec = np.zeros((n, 4), dtype=t)
        rec[:, :dim] = x
        rec[:, dim] = z
        return [rec]
    if layout == "hybrid":
        return [np.ascontiguousarray(x, dtype=t), np.ascontiguousarray(z, dtype=t)]
    if layout == "soaos":
        w = 2 if dim == 2 else 4
        c = np.zeros((n, w), dtype=t)
        c[:, :dim] = x
        v = np.zeros((n, 2), dtype=t)
        v[:, 0] = z
        return [c, v]
    raise ValueError(layout)


def pack_query(q: np.ndarray, layout: str, dtype: str):
    """Pack query coordinates q [m,dim]; same layouts as pack_data without the values."""
    t = _np_dtype(dtype)
    m, dim = q.shape
    if layout == "soa":
        return [np.ascontiguousarray(q[:, k], dtype=t) for k in range(dim)]
    if layout in ("aos", "hybrid"):
        return [np.ascontiguousarray(q, dtype=t)]
    if layout == "aoas":
        rec = np.zeros((m, 4), dtype=t)
        rec[:, :dim] = q
        return [rec]
    if layout == "soaos":
        w = 2 if dim == 2 else 4
        c = np.zeros((m, w), dtype=t)
        c[:, :dim] = q
        return [c]
    raise ValueError(layout)
