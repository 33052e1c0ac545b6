"""Batched iteration over uneven clips and the tile autotuner (C ABI wrappers)."""
from __future__ import annotations

import ctypes

import torch

from . import _native as N
from .api import Kernel, _dtype_code, _stream_ptr, problem_for


class BatchPlan:
    """Plan for iterating many clips (shapes [(T, H, W), ...]) with one filter.

    Clips are packed into one flat buffer at 256-byte aligned offsets.
    """

    def __init__(self, shapes, kern: Kernel, dtype: torch.dtype = torch.float32):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.kern = kern
        self.dtype = dtype
        esz = torch.tensor([], dtype=dtype).element_size()
        align = max(1, 256 // esz)
        offs, off = [], 0
        for T, H, W in self.shapes:
            offs.append(off)
            off += T * H * W
            off = (off + align - 1) // align * align
        self.offsets = offs
        self.extent = off
        arr = (N.Clip * len(self.shapes))()
        for i, ((T, H, W), o) in enumerate(zip(self.shapes, offs)):
            arr[i] = N.Clip(o, T, H, W, 0)
        h = ctypes.c_void_p()
        N.check(N.lib.stpi_batch_plan(arr, len(self.shapes), float(kern.sigma_s), float(kern.sigma_t),
                                      int(kern.r_s), int(kern.r_t), _dtype_code(dtype), ctypes.byref(h)))
        self._h = h
        self.ws_bytes = int(N.lib.stpi_batch_workspace_bytes(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            N.lib.stpi_plan_destroy(h)
            self._h = None

    def info(self) -> dict:
        a = (ctypes.c_int32 * 11)()
        N.check(N.lib.stpi_batch_info(self._h, a))
        keys = ("nclips", "ntiles", "grid", "RS", "RT", "TH", "TW", "NTHR", "RY", "QX", "PIPE")
        return dict(zip(keys, list(a)))

    def empty(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.extent, dtype=self.dtype, device=device)

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def pack(self, vols, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.empty(vols[0].device) if out is None else out
        for v, o, s in zip(vols, self.offsets, self.shapes):
            out[o:o + v.numel()].view(s).copy_(v)
        return out

    def views(self, flat: torch.Tensor):
        return [flat[o:o + T * H * W].view(T, H, W) for o, (T, H, W) in zip(self.offsets, self.shapes)]

    def iterate(self, f_flat: torch.Tensor, x_flat: torch.Tensor | None = None, init: int = 1,
                max_iters: int = 50, tol: float = 1e-4, ws: torch.Tensor | None = None, stream=None,
                check: bool = True):
        """stpi_batch_iterate; returns (x_flat, [result dict per clip])."""
        if x_flat is None:
            x_flat = torch.empty_like(f_flat)
        for name, t in (("f_flat", f_flat), ("x_flat", x_flat)):
            if t.numel() < self.extent or t.dtype != self.dtype or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"{name} must be a contiguous {self.dtype} device tensor of >= {self.extent} elements")
        ws = self.workspace(f_flat.device) if ws is None else ws
        res = (N.Result * len(self.shapes))()
        rc = N.lib.stpi_batch_iterate(self._h, f_flat.data_ptr(), x_flat.data_ptr(), int(init), int(max_iters),
                                      float(tol), ws.data_ptr(), ws.numel(), res, _stream_ptr(stream))
        if check:
            N.check(rc)
        return x_flat, [r.as_dict() for r in res]


def autotune(shape, kern: Kernel, dtype: torch.dtype = torch.float32, cache_path: str | None = None,
             reps: int = 10):
    """Times every eligible step variant for this problem; returns (variant index, ms)."""
    p = problem_for(shape, kern, dtype)
    v = ctypes.c_int32()
    ms = ctypes.c_double()
    N.check(N.lib.stpi_autotune(ctypes.byref(p), cache_path.encode() if cache_path else None, int(reps),
                                ctypes.byref(v), ctypes.byref(ms)))
    return v.value, ms.value


def autotune_load(path: str) -> None:
    N.check(N.lib.stpi_autotune_load(path.encode()))


def autotune_clear() -> None:
    N.lib.stpi_autotune_clear()
