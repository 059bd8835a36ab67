"""Shared helpers of the GPU parity tests: pack seeded host inputs into a layout, upload
them, call the library through the C ABI and fetch the FP64 oracle for the same values."""
from __future__ import annotations

import concurrent.futures as cf
import os

import numpy as np
import torch

import oracle
from paper_1402_4986_amd import api, workloads

TOL = {"f32": 1e-5, "f32_kahan": 1e-5, "f64": 1e-12}  # scale-aware relative error of Z
GTOL = {"f32": 1e-5, "f64": 1e-12}      # condition-aware relative error of the gradients
# The plain relative error |Z - Z_oracle| / |Z_oracle|, on the queries where |Z_oracle| is at
# least a tenth of max |z| (there it is well defined): the same bounds.
PLAIN_TOL = TOL
PLAIN_FRACTION = 0.1


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


def plain_rel_err(got, ref, z):
    """|got - Z| / |Z| on the queries with |Z| >= 0.1 max|z| (an empty array if none)."""
    keep = np.abs(ref["Z"]) >= PLAIN_FRACTION * np.max(np.abs(z))
    return np.abs(got[keep] - ref["Z"][keep]) / np.abs(ref["Z"][keep])


def _threads():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _slices(m, parts):
    return [s for s in np.array_split(np.arange(m), parts) if len(s)]


def oracle_forward_par(x, z, q, p):
    """oracle.forward over slices of the queries in a thread pool (the oracle's C loop
    releases the interpreter lock); each query's result is the oracle's own."""
    sl = _slices(len(q), 4 * _threads())
    with cf.ThreadPoolExecutor(_threads()) as ex:
        parts = list(ex.map(lambda s: oracle.forward(x, z, q[s], p), sl))
    return {k: np.concatenate([r[k] for r in parts]) for k in ("Z", "D", "S", "H")}


def oracle_backward_par(x, z, q, p, g):
    """oracle.backward over slices of the queries in a thread pool.  Per-query outputs are
    concatenated; the sums over queries (dz, dp and their scales) add the slices' sums in
    slice order, in FP64 (a relative change of about 1e-16, far below every tolerance)."""
    sl = _slices(len(q), 4 * _threads())
    with cf.ThreadPoolExecutor(_threads()) as ex:
        parts = list(ex.map(lambda s: oracle.backward(x, z, q[s], p, g[s]), sl))
    out = {k: np.concatenate([r[k] for r in parts]) for k in ("dq", "dq_scale", "dq_cond")}
    for k in ("dz", "dz_scale"):
        acc = np.zeros_like(parts[0][k])
        for r in parts:
            acc += r[k]
        out[k] = acc
    for k in ("dp", "dp_scale", "dp_cond"):
        out[k] = float(sum(r[k] for r in parts))
    return out


# Where a centred gradient sum is well conditioned (its uncentred condition sum at most
# this many times its own absolute-term sum), it is also held to the tolerance relative to
# that absolute-term sum.
CENTRED_COND = 10.0


def dq_errors(dq, ref, rows=None):
    """(error of each dq row relative to dq_cond, the same relative to dq_scale on the rows
    where dq_cond <= CENTRED_COND dq_scale)."""
    rq = ref["dq"] if rows is None else ref["dq"][rows]
    cond = ref["dq_cond"] if rows is None else ref["dq_cond"][rows]
    scale = ref["dq_scale"] if rows is None else ref["dq_scale"][rows]
    err = np.max(np.abs(dq - rq), axis=1)
    well = (scale > 0) & (cond <= CENTRED_COND * scale)
    return err / np.maximum(cond, 1e-300), err[well] / scale[well]


def dp_errors(dp, ref):
    """(|dp error| / dp_cond, |dp error| / dp_scale or 0 when dp_cond > CENTRED_COND dp_scale)."""
    err = abs(dp - ref["dp"])
    well = ref["dp_scale"] > 0 and ref["dp_cond"] <= CENTRED_COND * ref["dp_scale"]
    return err / max(ref["dp_cond"], 1e-300), (err / ref["dp_scale"] if well else 0.0)
