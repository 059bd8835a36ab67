"""Batched IDW: many independent instances swept by one persistent kernel, replayed as a
HIP graph (idw_batched_plan_create / idw_batched).  Argument marshalling only.

Every instance uses aligned-AoS float4 records for data ({x, y, v, pad} or {x, y, z, v})
and queries ({x, y, (z), pad}); each has its own dim, p and sizes.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional

import torch

from . import _lib
from ._lib import IdwConfig, IdwInstance, check

TUNING_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning", "gfx950.json")


class BatchedPlan:
    """Owns an idw_plan and its workspace; call run() to enqueue all instances.

    instances: list of dicts with keys data (float4 tensor [n, 4]), query (float4 tensor
    [m, 4]), dim, p, out_z (float32 [m]) and optionally out_den (float64 [m]).
    """

    def __init__(self, instances: List[dict], chunk: int = 0, workgroups: int = 0, tuning: Optional[dict] = None):
        lib = _lib.load()
        # chunk / workgroups left at 0 take the library's defaults: the autotuned values its
        # build compiled in (idw_batched_defaults); `tuning` overrides them from a table.
        tuning = tuning or {}
        chunk = chunk or int(tuning.get("batch_chunk", 0))
        workgroups = workgroups or int(tuning.get("batch_workgroups", 0))
        self._keep = instances
        arr = (IdwInstance * len(instances))()
        for k, inst in enumerate(instances):
            d, q = inst["data"], inst["query"]
            for t in (d, q):
                if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 4 or not t.is_contiguous():
                    raise ValueError("batched instances take contiguous float32 [*, 4] records")
            a = arr[k]
            a.data.ptr[0] = d.data_ptr()
            a.data.n, a.data.dim, a.data.layout = d.shape[0], int(inst["dim"]), _lib.AOAS
            a.query.ptr[0] = q.data_ptr() if q.shape[0] else None
            a.query.n, a.query.dim, a.query.layout = q.shape[0], int(inst["dim"]), _lib.AOAS
            a.p = float(inst["p"])
            a.out_z = inst["out_z"].data_ptr() if inst["out_z"].numel() else None
            den = inst.get("out_den")
            a.out_den = den.data_ptr() if den is not None and den.numel() else None
        cfg = IdwConfig()
        cfg.batch_chunk = int(chunk)
        cfg.batch_workgroups = int(workgroups)
        self._plan = ctypes.c_void_p()
        check(lib.idw_batched_plan_create(arr, len(instances), _lib.FP32, ctypes.byref(cfg), ctypes.byref(self._plan)))
        need = ctypes.c_size_t()
        check(lib.idw_batched_plan_workspace(self._plan, ctypes.byref(need)))
        dev = instances[0]["data"].device
        self.workspace = torch.empty(max(need.value, 256), dtype=torch.uint8, device=dev)
        self.device = dev

    def params(self) -> tuple:
        """(data points per work item, persistent workgroups) of this plan."""
        c, w = ctypes.c_int64(), ctypes.c_int32()
        check(_lib.load().idw_batched_plan_params(self._plan, ctypes.byref(c), ctypes.byref(w)))
        return c.value, w.value

    def run(self, stream: Optional[torch.cuda.Stream] = None) -> None:
        lib = _lib.load()
        s = (stream or torch.cuda.current_stream(self.device)).cuda_stream
        check(lib.idw_batched(self._plan, self.workspace.data_ptr(), self.workspace.numel(), s))

    def close(self) -> None:
        if getattr(self, "_plan", None) is not None and self._plan.value:
            _lib.load().idw_batched_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
