"""Full SFSeg operator (alpha > 0, unary map distinct from the pairwise
feature): same names and arguments as the C calls stpi_sfseg_*."""
from __future__ import annotations

import ctypes

import torch

from . import _native as N
from .api import Kernel, _check_volume, _stream_ptr, problem_for


def sfseg_unary(S: torch.Tensor, p: float, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """s = S^p elementwise (stpi_sfseg_unary)."""
    _check_volume("S", S)
    out = torch.empty_like(S) if out is None else out
    _check_volume("out", out, S.shape, S.dtype)
    code = {torch.float32: N.STPI_F32, torch.float64: N.STPI_F64}.get(S.dtype)
    if code is None:
        raise TypeError("sfseg works on float32 or float64 volumes")
    N.check(N.lib.stpi_sfseg_unary(S.numel(), code, S.data_ptr(), float(p), out.data_ptr(), _stream_ptr(stream)))
    return out


def sfseg_workspace_bytes(shape, k: Kernel, dtype: torch.dtype = torch.float32) -> int:
    p = problem_for(shape, k, dtype)
    n = N.lib.stpi_sfseg_workspace_bytes(ctypes.byref(p))
    if n == 0:
        N.check(N.lib.stpi_sfseg_step(ctypes.byref(p), None, None, 1.0, None, 1.0, None, None, None, 0, None))
    return int(n)


def _ws(shape, k, dtype, device, ws):
    need = sfseg_workspace_bytes(shape, k, dtype)
    if ws is None:
        return torch.empty(need, dtype=torch.uint8, device=device)
    if ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace too small: {ws.numel()} < {need} bytes")
    return ws


def sfseg_step(s: torch.Tensor, f: torch.Tensor, x: torch.Tensor, k: Kernel, alpha: float, x_scale: float = 1.0,
               z: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """One unnormalised application (stpi_sfseg_step); returns (z, sums)."""
    _check_volume("s", s)
    _check_volume("f", f, s.shape, s.dtype)
    _check_volume("x", x, s.shape, s.dtype)
    z = torch.empty_like(s) if z is None else z
    _check_volume("z", z, s.shape, s.dtype)
    sums = torch.empty(2, dtype=torch.float64, device=s.device)
    ws = _ws(s.shape, k, s.dtype, s.device, ws)
    p = problem_for(s.shape, k, s.dtype)
    N.check(N.lib.stpi_sfseg_step(ctypes.byref(p), s.data_ptr(), f.data_ptr(), float(alpha), x.data_ptr(),
                                  float(x_scale), z.data_ptr(), sums.data_ptr(), ws.data_ptr(), ws.numel(),
                                  _stream_ptr(stream)))
    return z, sums


def sfseg_iterate(s: torch.Tensor, f: torch.Tensor, k: Kernel, alpha: float, iters: int | None = None,
                  tol: float | None = None, max_iters: int = 1000, x0: torch.Tensor | None = None,
                  x: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None, check: bool = True):
    """Power iteration with the full operator (stpi_sfseg_iterate); returns (x, result dict)."""
    _check_volume("s", s)
    _check_volume("f", f, s.shape, s.dtype)
    if iters is not None:
        n_iter, t = int(iters), 0.0
    else:
        if tol is None or not tol > 0:
            raise ValueError("give iters, or tol > 0")
        n_iter, t = int(max_iters), float(tol)
    x = torch.empty_like(s) if x is None else x
    _check_volume("x", x, s.shape, s.dtype)
    init = 1
    if x0 is not None:
        _check_volume("x0", x0, s.shape, s.dtype)
        if x0.data_ptr() != x.data_ptr():
            x.copy_(x0)
        init = 0
    ws = _ws(s.shape, k, s.dtype, s.device, ws)
    p = problem_for(s.shape, k, s.dtype)
    res = N.Result()
    rc = N.lib.stpi_sfseg_iterate(ctypes.byref(p), s.data_ptr(), f.data_ptr(), float(alpha), x.data_ptr(), init,
                                  n_iter, t, ws.data_ptr(), ws.numel(), ctypes.byref(res), _stream_ptr(stream))
    out = res.as_dict()
    out["rc"] = rc
    if check:
        N.check(rc)
    return x, out


def _exp_ws(shape, k, dtype, device, ws):
    p = problem_for(shape, k, dtype)
    need = int(N.lib.stpi_exp_workspace_bytes(ctypes.byref(p)))
    if need == 0:
        N.check(N.lib.stpi_exp_step(ctypes.byref(p), None, None, 1.0, None, 1.0, None, None, None, 0, None))
    if ws is None:
        return torch.empty(need, dtype=torch.uint8, device=device)
    if ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace too small: {ws.numel()} < {need} bytes")
    return ws


def exp_step(s: torch.Tensor, f: torch.Tensor, x: torch.Tensor, k: Kernel, alpha: float, x_scale: float = 1.0,
             z: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None):
    """One application with the exact exponential affinity (stpi_exp_step); returns (z, sums)."""
    _check_volume("s", s)
    _check_volume("f", f, s.shape, s.dtype)
    _check_volume("x", x, s.shape, s.dtype)
    z = torch.empty_like(s) if z is None else z
    sums = torch.empty(2, dtype=torch.float64, device=s.device)
    ws = _exp_ws(s.shape, k, s.dtype, s.device, ws)
    p = problem_for(s.shape, k, s.dtype)
    N.check(N.lib.stpi_exp_step(ctypes.byref(p), s.data_ptr(), f.data_ptr(), float(alpha), x.data_ptr(),
                                float(x_scale), z.data_ptr(), sums.data_ptr(), ws.data_ptr(), ws.numel(),
                                _stream_ptr(stream)))
    return z, sums


def exp_iterate(s: torch.Tensor, f: torch.Tensor, k: Kernel, alpha: float, iters: int | None = None,
                tol: float | None = None, max_iters: int = 1000, x0: torch.Tensor | None = None,
                x: torch.Tensor | None = None, ws: torch.Tensor | None = None, stream=None, check: bool = True):
    """Power iteration with the exact affinity (stpi_exp_iterate); returns (x, result dict)."""
    _check_volume("s", s)
    _check_volume("f", f, s.shape, s.dtype)
    if iters is not None:
        n_iter, t = int(iters), 0.0
    else:
        if tol is None or not tol > 0:
            raise ValueError("give iters, or tol > 0")
        n_iter, t = int(max_iters), float(tol)
    x = torch.empty_like(s) if x is None else x
    init = 1
    if x0 is not None:
        if x0.data_ptr() != x.data_ptr():
            x.copy_(x0)
        init = 0
    ws = _exp_ws(s.shape, k, s.dtype, s.device, ws)
    p = problem_for(s.shape, k, s.dtype)
    res = N.Result()
    rc = N.lib.stpi_exp_iterate(ctypes.byref(p), s.data_ptr(), f.data_ptr(), float(alpha), x.data_ptr(), init,
                                n_iter, t, ws.data_ptr(), ws.numel(), ctypes.byref(res), _stream_ptr(stream))
    out = res.as_dict()
    out["rc"] = rc
    if check:
        N.check(rc)
    return x, out
