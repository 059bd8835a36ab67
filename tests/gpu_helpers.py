"""Shared helpers of the GPU parity tests: pack seeded host inputs into a layout, upload
them, call the library through the C ABI and fetch the FP64 oracle for the same values."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1402_4986_amd import api, workloads

TOL = {"f32": 1e-5, "f32_kahan": 1e-5, "f64": 1e-12}  # scale-aware relative error of Z
GTOL = {"f32": 1e-5, "f64": 1e-12}      # condition-aware relative error of the gradients


def points(x, z, q, layout, prec, device="cuda"):
    n, dim = x.shape
    m = q.shape[0]
    d = api.Points.from_arrays(workloads.pack_data(x, z, layout, prec), n, dim, layout, device)
    qq = api.Points.from_arrays(workloads.pack_query(q, layout, prec), m, dim, layout, device)
    return d, qq


def gpu_forward(x, z, q, p, layout="aoas", prec="f32", **kw):
    d, qq = points(x, z, q, layout, prec)
    Z, D = api.forward(d, qq, p, prec, **kw)
    torch.cuda.synchronize()
    return Z.cpu().numpy().astype(np.float64), D.cpu().numpy()


def scaled_err(got, ref):
    """|got - Z| / S with S the oracle's summation scale (sum w|z| / sum w)."""
    S = np.maximum(ref["S"], 1e-300)
    return np.abs(got - ref["Z"]) / S


def rand_case(seed, n, m, dim, prec="f32", lo=0.0, hi=1.0):
    r = np.random.default_rng(seed)
    x = r.uniform(lo, hi, (n, dim))
    z = np.sin(3 * x[:, 0]) + np.cos(2 * x[:, 1]) + r.normal(0, 0.1, n)
    q = r.uniform(lo, hi, (m, dim))
    t = np.float64 if prec == "f64" else np.float32
    return x.astype(t).astype(np.float64), z.astype(t).astype(np.float64), q.astype(t).astype(np.float64)
