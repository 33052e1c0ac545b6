"""Python entry points over the C ABI: same names and arguments as the C calls."""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import torch

from . import _native as N


@dataclass(frozen=True)
class Kernel:
    """Truncated space-time Gaussian filter: sigmas (pixels, frames) and box radii."""
    sigma_s: float
    sigma_t: float
    r_s: int
    r_t: int


_DTYPES = {torch.float32: N.STPI_F32, torch.bfloat16: N.STPI_BF16, torch.float64: N.STPI_F64}


def _dtype_code(dt: torch.dtype) -> int:
    if dt not in _DTYPES:
        raise TypeError(f"unsupported dtype {dt}; use float32, bfloat16 or float64")
    return _DTYPES[dt]


def problem_for(shape, k: Kernel, dtype: torch.dtype) -> N.Problem:
    T, H, W = (int(s) for s in shape)
    return N.Problem(T, H, W, float(k.sigma_s), float(k.sigma_t), int(k.r_s), int(k.r_t), _dtype_code(dtype))


def _check_volume(name: str, t: torch.Tensor, shape=None, dtype=None) -> None:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous [T][H][W]")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} has dtype {t.dtype}, expected {dtype}")


def _stream_ptr(stream) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def workspace_bytes(shape, k: Kernel, dtype: torch.dtype = torch.float32) -> int:
    p = problem_for(shape, k, dtype)
    n = N.lib.stpi_workspace_bytes(ctypes.byref(p))
    if n == 0:
        N.check(N.STPI_EINVAL)
    return int(n)


def _workspace(shape, k, dtype, device, ws):
    need = workspace_bytes(shape, k, dtype)
    if ws is None:
        ws = torch.empty(need, dtype=torch.uint8, device=device)
    elif ws.numel() * ws.element_size() < need:
        raise ValueError(f"workspace too small: {ws.numel()} < {need} bytes")
    return ws


def step(f: torch.Tensor, x: torch.Tensor, k: Kernel, x_scale: float = 1.0, z: torch.Tensor | None = None,
         ws: torch.Tensor | None = None, stream=None):
    """One unnormalised application z = f * G * (f * x * x_scale) (stpi_step).

    Returns (z, sums) with sums a device float64 tensor (sum z^2, sum z x x_scale).
    """
    _check_volume("f", f)
    _check_volume("x", x, f.shape, f.dtype)
    if z is None:
        z = torch.empty_like(f)
    _check_volume("z", z, f.shape, f.dtype)
    sums = torch.empty(2, dtype=torch.float64, device=f.device)
    ws = _workspace(f.shape, k, f.dtype, f.device, ws)
    p = problem_for(f.shape, k, f.dtype)
    N.check(N.lib.stpi_step(ctypes.byref(p), f.data_ptr(), x.data_ptr(), float(x_scale), z.data_ptr(),
                            sums.data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(stream)))
    return z, sums


def step_noalloc(f: torch.Tensor, x: torch.Tensor, k: Kernel, x_scale: float, z: torch.Tensor,
                 sums: torch.Tensor, stream=None):
    """stpi_step_noalloc: stpi_step with the library's per-device scratch
    instead of a workspace; z and sums (2 device doubles) are the caller's."""
    _check_volume("f", f)
    _check_volume("x", x, f.shape, f.dtype)
    _check_volume("z", z, f.shape, f.dtype)
    if sums.dtype != torch.float64 or sums.numel() < 2 or not sums.is_cuda:
        raise ValueError("sums must be a device float64 tensor of 2 elements")
    p = problem_for(f.shape, k, f.dtype)
    N.check(N.lib.stpi_step_noalloc(ctypes.byref(p), f.data_ptr(), x.data_ptr(), float(x_scale), z.data_ptr(),
                                    sums.data_ptr(), _stream_ptr(stream)))
    return z, sums


def power_iterate(f: torch.Tensor, k: Kernel, iters: int | None = None, tol: float | None = None,
                  max_iters: int = 1000, x0: torch.Tensor | None = None, x: torch.Tensor | None = None,
                  ws: torch.Tensor | None = None, stream=None, check: bool = True, wait: bool = True,
                  rise_check: bool = False):
    """Power iteration x <- A x / ||A x|| (stpi_iterate).

    iters: exact number of applications; otherwise stop when
    ||x_k - x_{k-1}|| < tol or after max_iters. x0 (optional) is the start
    vector (uniform 1/sqrt(N) otherwise). Returns (x, result dict); with
    wait=False the chain is only enqueued on `stream` and the result is None.
    rise_check (with x0): stop after the second application if its residual
    is above the first (result flags bit 2), the warm-start fallback test.
    """
    _check_volume("f", f)
    if iters is not None:
        n_iter, t = int(iters), 0.0
    else:
        if tol is None or not tol > 0:
            raise ValueError("give iters, or tol > 0")
        n_iter, t = int(max_iters), float(tol)
    if x is None:
        x = torch.empty_like(f)
    _check_volume("x", x, f.shape, f.dtype)
    init = 1
    if x0 is not None:
        _check_volume("x0", x0, f.shape, f.dtype)
        if x0.data_ptr() != x.data_ptr():
            x.copy_(x0)
        init = 2 if rise_check else 0
    ws = _workspace(f.shape, k, f.dtype, f.device, ws)
    p = problem_for(f.shape, k, f.dtype)
    res = N.Result()
    rc = N.lib.stpi_iterate(ctypes.byref(p), f.data_ptr(), x.data_ptr(), init, n_iter, t, ws.data_ptr(),
                            ws.numel(), ctypes.byref(res) if wait else None, _stream_ptr(stream))
    if check or not wait:
        N.check(rc)
    if not wait:
        return x, None
    out = res.as_dict()
    out["rc"] = rc
    return x, out


def coarse_problem(shape, k: Kernel, sy: int, st: int, dtype: torch.dtype = torch.float32):
    """stpi_coarse_problem: the coarse grid's shape and kernel for factors (sy, st)."""
    c = N.Problem()
    N.check(N.lib.stpi_coarse_problem(ctypes.byref(problem_for(shape, k, dtype)), int(sy), int(st), ctypes.byref(c)))
    return (c.T, c.H, c.W), Kernel(float(c.sigma_s), float(c.sigma_t), int(c.r_s), int(c.r_t))


def coarse_shape(shape, sy: int, st: int):
    return coarse_problem(shape, Kernel(1.0, 1.0, 0, 0), sy, st)[0]


def scale(x: torch.Tensor, s: float, s_dev: torch.Tensor | None = None, out: torch.Tensor | None = None,
          stream=None) -> torch.Tensor:
    """stpi_scale: out = x * s (* s_dev, a float64 device scalar, when given)."""
    if not isinstance(x, torch.Tensor) or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous device tensor")
    if s_dev is not None and (s_dev.dtype != torch.float64 or not s_dev.is_cuda or s_dev.numel() != 1):
        raise ValueError("s_dev must be one float64 device value")
    out = torch.empty_like(x) if out is None else out
    if out.shape != x.shape or out.dtype != x.dtype or not out.is_contiguous() or out.device != x.device:
        raise ValueError("out must match x")
    N.check(N.lib.stpi_scale(x.numel(), _dtype_code(x.dtype), x.data_ptr(), float(s),
                             s_dev.data_ptr() if s_dev is not None else None, out.data_ptr(), _stream_ptr(stream)))
    return out


def downsample(x: torch.Tensor, sy: int, st: int, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Box average to the coarse grid (stpi_downsample)."""
    _check_volume("x", x)
    cs = coarse_shape(x.shape, sy, st)
    out = torch.empty(cs, dtype=x.dtype, device=x.device) if out is None else out
    _check_volume("out", out, cs, x.dtype)
    T, H, W = x.shape
    N.check(N.lib.stpi_downsample(T, H, W, int(sy), int(st), _dtype_code(x.dtype), x.data_ptr(), out.data_ptr(),
                                  _stream_ptr(stream)))
    return out


def upsample(xc: torch.Tensor, shape, sy: int, st: int, mode: int = 1, mul: torch.Tensor | None = None,
             out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Coarse volume back to `shape` (stpi_upsample), times mul if given."""
    shape = tuple(int(v) for v in shape)
    _check_volume("xc", xc, coarse_shape(shape, sy, st))
    if mul is not None:
        _check_volume("mul", mul, shape, xc.dtype)
    out = torch.empty(shape, dtype=xc.dtype, device=xc.device) if out is None else out
    _check_volume("out", out, shape, xc.dtype)
    N.check(N.lib.stpi_upsample(*shape, int(sy), int(st), int(mode), _dtype_code(xc.dtype), xc.data_ptr(),
                                mul.data_ptr() if mul is not None else None, out.data_ptr(), _stream_ptr(stream)))
    return out


def launch_shape(shape, k: Kernel, dtype: torch.dtype = torch.float32, variant: int = -1) -> dict:
    """stpi_launch_shape: the variant, tiles, frame segments and workgroups a step uses."""
    p = problem_for(shape, k, dtype)
    a = (ctypes.c_int32 * 5)()
    N.check(N.lib.stpi_launch_shape(ctypes.byref(p), int(variant), a))
    return dict(zip(("variant", "tiles", "segments", "blocks_per_cu", "workgroups"), list(a)))


def time_step(f: torch.Tensor, x: torch.Tensor, k: Kernel, z: torch.Tensor | None = None, reps: int = 20,
              variant: int = -1, ws: torch.Tensor | None = None, stream=None) -> float:
    """Average step-kernel duration in ms over `reps` launches (stpi_time_step, HIP events)."""
    _check_volume("f", f)
    _check_volume("x", x, f.shape, f.dtype)
    if z is None:
        z = torch.empty_like(f)
    ws = _workspace(f.shape, k, f.dtype, f.device, ws)
    p = problem_for(f.shape, k, f.dtype)
    ms = ctypes.c_double()
    N.check(N.lib.stpi_time_step(ctypes.byref(p), f.data_ptr(), x.data_ptr(), z.data_ptr(), ws.data_ptr(),
                                 ws.numel(), int(variant), int(reps), _stream_ptr(stream), ctypes.byref(ms)))
    return ms.value


def time_chain_step(f: torch.Tensor, k: Kernel, x: torch.Tensor | None = None, reps: int = 20, variant: int = -1,
                    ws: torch.Tensor | None = None, stream=None) -> tuple[float, bool]:
    """Average duration in ms of one step of an iteration chain as power_iterate
    runs it (stpi_time_chain_step, HIP events), and whether it ran in product
    form. x is scratch (overwritten)."""
    _check_volume("f", f)
    if x is None:
        x = torch.empty_like(f)
    _check_volume("x", x, f.shape, f.dtype)
    ws = _workspace(f.shape, k, f.dtype, f.device, ws)
    p = problem_for(f.shape, k, f.dtype)
    ms = ctypes.c_double()
    pf = ctypes.c_int()
    N.check(N.lib.stpi_time_chain_step(ctypes.byref(p), f.data_ptr(), x.data_ptr(), ws.data_ptr(), ws.numel(),
                                       int(variant), int(reps), _stream_ptr(stream), ctypes.byref(ms),
                                       ctypes.byref(pf)))
    return ms.value, bool(pf.value)
