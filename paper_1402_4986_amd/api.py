"""Python face of libidw: point descriptors, forward/backward calls, the autograd Function
and the leave-one-out fit of p.

PyTorch provides device memory and streams only; every step of the IDW path (extent,
sweeps, merges, FP64 fix-ups, reductions) runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import IdwConfig, IdwPoints, check

_TORCH_DTYPE = {"f32": torch.float32, "f64": torch.float64, "f32_kahan": torch.float32}


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    return None if t is None else t.data_ptr()


@dataclass
class Points:
    """A point set in one of the record layouts (device tensors, caller-owned).

    tensors: one contiguous tensor per pointer slot of the layout (see include/idw.h);
    n: number of points; dim: 2 or 3; layout: 'soa' | 'aos' | 'aoas' | 'hybrid' | 'soaos'.
    """
    tensors: Sequence[torch.Tensor]
    n: int
    dim: int
    layout: str

    def c(self) -> IdwPoints:
        s = IdwPoints()
        for k, t in enumerate(self.tensors):
            if not t.is_contiguous():
                raise ValueError("point tensors must be contiguous")
            s.ptr[k] = t.data_ptr()
        s.n = int(self.n)
        s.dim = int(self.dim)
        s.layout = _lib.LAYOUT_CODES[self.layout]
        return s

    @property
    def device(self) -> torch.device:
        return self.tensors[0].device

    @property
    def dtype(self) -> torch.dtype:
        return self.tensors[0].dtype

    @staticmethod
    def from_arrays(arrays, n: int, dim: int, layout: str, device="cuda") -> "Points":
        """Upload host arrays (already packed in `layout`) to the device."""
        ts = [torch.as_tensor(a).to(device).contiguous() for a in arrays]
        return Points(ts, n, dim, layout)

    @staticmethod
    def hybrid(coords: torch.Tensor, values: Optional[torch.Tensor] = None) -> "Points":
        """Coordinates [n, dim] (packed rows) plus an optional value array [n]."""
        ts = [coords.contiguous()] + ([values.contiguous()] if values is not None else [])
        return Points(ts, coords.shape[0], coords.shape[1], "hybrid")


def _cfg(queries_per_lane: int = 0, split: int = 0, near_search: int = 0,
         separate: bool = False) -> Optional[IdwConfig]:
    if not queries_per_lane and not split and not near_search and not separate:
        return None
    c = IdwConfig()
    c.queries_per_lane = queries_per_lane
    c.split = split
    c.near_search = near_search
    c.separate_adjoint = 1 if separate else 0
    return c


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


_ws_cache: dict = {}


def workspace(data: Points, query: Points, precision: str, cfg: Optional[IdwConfig] = None,
              backward: bool = True, need_dx: bool = False) -> torch.Tensor:
    """A device workspace for the forward (backward=False) or for forward and backward on
    these point sets, with room for the data-coordinate gradient when need_dx.  Cached per
    (device, current stream) and grown on demand: calls enqueued on one stream run in order,
    so they may share it, while work on another stream gets its own."""
    lib = _lib.load()
    need = ctypes.c_size_t()
    dc, qc = data.c(), query.c()
    flags = (_lib.NEED_DZ | _lib.NEED_DP | _lib.NEED_DQ) if backward else 0
    if backward and need_dx:
        flags |= _lib.NEED_DX
    check(lib.idw_workspace_size(ctypes.byref(dc), ctypes.byref(qc), _lib.PRECISION_CODES[precision], flags,
                                 ctypes.byref(cfg) if cfg is not None else None, ctypes.byref(need)))
    key = (str(data.device), _stream_handle(data.device))
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < need.value:
        ws = torch.empty(max(need.value, 256), dtype=torch.uint8, device=data.device)
        _ws_cache[key] = ws
    return ws


def forward(data: Points, query: Points, p: float, precision: str = "f32", exclude_self: bool = False,
            queries_per_lane: int = 0, split: int = 0, out_z: Optional[torch.Tensor] = None,
            out_den: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None, near_search: int = 0):
    """Z[m] (precision dtype) and D[m] (float64) for the query set (Eq. 1).  near_search=1
    makes the nearest-distance searches brute force (idw_config.near_search)."""
    lib = _lib.load()
    dt = _TORCH_DTYPE[precision]
    m = int(query.n)
    dev = data.device
    if out_z is None:
        out_z = torch.empty(m, dtype=dt, device=dev)
    if out_den is None:
        out_den = torch.empty(m, dtype=torch.float64, device=dev)
    cfg = _cfg(queries_per_lane, split, near_search)
    if ws is None:
        ws = workspace(data, query, precision, cfg, backward=False)
    dc, qc = data.c(), query.c()
    check(lib.idw_forward(ctypes.byref(dc), ctypes.byref(qc), float(p), _lib.PRECISION_CODES[precision],
                          _lib.EXCLUDE_SELF if exclude_self else 0, _ptr(out_z), _ptr(out_den), _ptr(ws),
                          ws.numel(), _stream_handle(dev), ctypes.byref(cfg) if cfg is not None else None))
    return out_z, out_den


def backward(data: Points, query: Points, p: float, grad_out: torch.Tensor, saved_z: torch.Tensor,
             saved_den: torch.Tensor, precision: str = "f32", need_dz: bool = True, need_dp: bool = True,
             need_dq: bool = True, exclude_self: bool = False, ws: Optional[torch.Tensor] = None,
             separate: bool = False, need_dx: bool = False, near_search: int = 0):
    """(dz[n] or None, dp (0-d float64 tensor) or None, dq[m, dim] or None), followed by
    dx[n, dim] when need_dx (the gradient with respect to the data coordinates).

    separate=True runs the query-direction and data-direction sweeps as two kernels
    instead of the fused FP32 sweep (for comparison); near_search=1 makes the
    nearest-distance searches brute force."""
    lib = _lib.load()
    dt = _TORCH_DTYPE[precision]
    dev = data.device
    n, m, dim = int(data.n), int(query.n), int(data.dim)
    dz = torch.empty(n, dtype=dt, device=dev) if need_dz else None
    dp = torch.empty((), dtype=torch.float64, device=dev) if need_dp else None
    dq = torch.empty((m, dim), dtype=dt, device=dev) if need_dq else None
    dx = torch.empty((n, dim), dtype=dt, device=dev) if need_dx else None
    flags = (_lib.EXCLUDE_SELF if exclude_self else 0) | (_lib.NEED_DZ if need_dz else 0) \
        | (_lib.NEED_DP if need_dp else 0) | (_lib.NEED_DQ if need_dq else 0) | (_lib.NEED_DX if need_dx else 0)
    cfg = _cfg(near_search=near_search, separate=separate)
    if ws is None:
        ws = workspace(data, query, precision, cfg, need_dx=need_dx)
    dc, qc = data.c(), query.c()
    check(lib.idw_backward(ctypes.byref(dc), ctypes.byref(qc), float(p), _lib.PRECISION_CODES[precision], flags,
                           _ptr(grad_out.contiguous()), _ptr(saved_z), _ptr(saved_den), _ptr(dz), _ptr(dp),
                           _ptr(dq), _ptr(dx), _ptr(ws), ws.numel(), _stream_handle(dev),
                           ctypes.byref(cfg) if cfg is not None else None))
    if need_dx:
        return dz, dp, dq, dx
    return dz, dp, dq


def _precision_of(t: torch.Tensor) -> str:
    if t.dtype == torch.float32:
        return "f32"
    if t.dtype == torch.float64:
        return "f64"
    raise TypeError("IDW tensors must be float32 or float64")


class IDWFunction(torch.autograd.Function):
    """Z = IDW(X, z, Q, p) with X [n, dim] data coordinates, z [n] values, Q [m, dim]
    queries and p a 0-d tensor.  Gradients flow to X, z, Q and p."""

    @staticmethod
    def forward(ctx, X, z, Q, p, exclude_self=False):
        prec = _precision_of(X)
        pv = float(p)
        data = Points.hybrid(X, z)
        query = Points.hybrid(Q)
        Z, D = forward(data, query, pv, prec, exclude_self=exclude_self)
        ctx.save_for_backward(X, z, Q, Z, D)
        ctx.pv = pv
        ctx.prec = prec
        ctx.excl = exclude_self
        ctx.p_dtype = p.dtype if torch.is_tensor(p) else torch.float64
        return Z

    @staticmethod
    def backward(ctx, gZ):
        X, z, Q, Z, D = ctx.saved_tensors
        need_x, need_z, need_q, need_p = ctx.needs_input_grad[:4]
        if not (need_x or need_z or need_q or need_p):
            return None, None, None, None, None
        data = Points.hybrid(X, z)
        query = Points.hybrid(Q)
        r = backward(data, query, ctx.pv, gZ.to(Z.dtype).contiguous(), Z, D, ctx.prec, need_dz=need_z,
                     need_dp=need_p, need_dq=need_q, exclude_self=ctx.excl, need_dx=need_x)
        dz, dp, dq = r[:3]
        dx = r[3] if need_x else None
        return dx, dz, dq, (dp.to(ctx.p_dtype) if dp is not None else None), None


def interpolate(X: torch.Tensor, z: torch.Tensor, Q: torch.Tensor, p=2.0) -> torch.Tensor:
    """Differentiable Shepard IDW of values z at X, evaluated at Q."""
    if not torch.is_tensor(p):
        p = torch.tensor(float(p), dtype=torch.float64, device=X.device)
    return IDWFunction.apply(X, z, Q, p)


def loo_loss(X: torch.Tensor, z: torch.Tensor, p: torch.Tensor) -> torch.Tensor:
    """Leave-one-out mean squared error of IDW at the data points."""
    Z = IDWFunction.apply(X, z, X, p, True)
    return torch.mean((Z.to(torch.float64) - z.to(torch.float64)) ** 2)


def fit_p_loo(X: torch.Tensor, z: torch.Tensor, p0: float = 1.5, steps: int = 50, lr: float = 0.05,
              clamp=(0.05, 6.0), method: str = "lbfgs"):
    """Fits p to the leave-one-out loss; returns (p, history of (p, loss) per evaluation).

    method "lbfgs" (default): L-BFGS with a strong-Wolfe line search over u, where
      p = lo + (hi - lo) sigmoid(u) keeps every trial p inside `clamp`; `steps` bounds the
      evaluations of the loss and its gradient.  On a smooth one-dimensional loss it reaches
      the minimiser in a few evaluations.
    method "adam": `steps` Adam steps of rate `lr` on p, clamped after each step.
    """
    lo, hi = float(clamp[0]), float(clamp[1])
    hist = []
    if method == "adam":
        p = torch.tensor(float(p0), dtype=torch.float64, device=X.device, requires_grad=True)
        opt = torch.optim.Adam([p], lr=lr)
        for _ in range(steps):
            opt.zero_grad()
            loss = loo_loss(X, z, p)
            loss.backward()
            hist.append((float(p.detach()), float(loss.detach())))
            opt.step()
            with torch.no_grad():
                p.clamp_(lo, hi)
        return float(p.detach()), hist
    if method != "lbfgs":
        raise ValueError(f"unknown method {method!r}")
    if not lo < float(p0) < hi:
        raise ValueError("p0 must lie strictly inside clamp")
    t = (float(p0) - lo) / (hi - lo)
    u = torch.tensor(float(np.log(t / (1.0 - t))), dtype=torch.float64, device=X.device, requires_grad=True)
    opt = torch.optim.LBFGS([u], lr=1.0, max_iter=steps, max_eval=steps, history_size=10,
                            tolerance_grad=1e-12, tolerance_change=1e-12, line_search_fn="strong_wolfe")
    p_of = lambda v: lo + (hi - lo) * torch.sigmoid(v)

    def closure():
        opt.zero_grad()
        p = p_of(u)
        loss = loo_loss(X, z, p)
        loss.backward()
        hist.append((float(p.detach()), float(loss.detach())))
        return loss

    opt.step(closure)
    return float(p_of(u.detach())), hist
