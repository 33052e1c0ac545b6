"""Online / partial iteration over video sub-windows (Sec. 4, "Online vs
Offline processing"): the video is processed in q-frame windows that move by
`shift` frames; each window runs a few power iterations from the previous
window's final solution on the frames they share (stpi_window_start) and
the uniform value on the new frames. Every frame keeps the value of the last
window that contains it. All arithmetic runs in libstpi; this module holds
the window schedule and the buffers (device copies of frame ranges)."""
from __future__ import annotations

import ctypes

import torch

from . import _native as N
from .api import Kernel, _check_volume, _stream_ptr, power_iterate, problem_for, workspace_bytes


def window_start(x_prev: torch.Tensor | None, shift: int, k: Kernel, x0: torch.Tensor, stream=None):
    """stpi_window_start: x0 of a window `shift` frames after x_prev's."""
    _check_volume("x0", x0)
    if x_prev is not None:
        _check_volume("x_prev", x_prev, x0.shape, x0.dtype)
    p = problem_for(x0.shape, k, x0.dtype)
    N.check(N.lib.stpi_window_start(ctypes.byref(p), None if x_prev is None else x_prev.data_ptr(), int(shift),
                                    x0.data_ptr(), _stream_ptr(stream)))
    return x0


def window_starts(T: int, q: int, shift: int):
    """First frames of the windows: 0, shift, 2 shift, ...; the last window ends at frame T."""
    if not (1 <= q <= T) or shift < 1:
        raise ValueError("need 1 <= q <= T and shift >= 1")
    starts = list(range(0, T - q + 1, shift))
    if starts[-1] != T - q:
        starts.append(T - q)
    return starts


def online_iterate(f: torch.Tensor, k: Kernel, q: int, shift: int, iters: int | None = None, tol: float | None = None,
                   max_iters: int = 1000, out: torch.Tensor | None = None, stream=None, wait: bool = True):
    """Whole video in sub-windows; returns (x, [per-window result dict]).

    x[t] is the final unit solution of the last window containing frame t
    (each window's solution is a unit vector over its own q frames). With a
    fixed count (iters) and wait=False every window is only enqueued (no
    host round trip) and the result list is empty."""
    _check_volume("f", f)
    T = f.shape[0]
    starts = window_starts(T, q, shift)
    wshape = (q,) + tuple(f.shape[1:])
    fbuf = torch.empty(wshape, dtype=f.dtype, device=f.device)
    xa = torch.empty_like(fbuf)
    xb = torch.empty_like(fbuf)
    ws = torch.empty(workspace_bytes(wshape, k, f.dtype), dtype=torch.uint8, device=f.device)
    out = torch.empty_like(f) if out is None else out
    _check_volume("out", out, f.shape, f.dtype)
    results = []
    prev, cur = None, xa
    s = stream if stream is not None else torch.cuda.current_stream()
    with torch.cuda.stream(s):
        for w, a in enumerate(starts):
            fbuf.copy_(f[a:a + q])
            moved = q if prev is None else a - starts[w - 1]
            window_start(prev, moved, k, cur, stream=s)
            enqueue_only = not wait and iters is not None
            _, r = power_iterate(fbuf, k, iters=iters, tol=tol, max_iters=max_iters, x0=cur, x=cur, ws=ws,
                                 stream=s, check=True, wait=not enqueue_only)
            out[a:a + q].copy_(cur)
            if r is not None:
                r["start"] = a
                results.append(r)
            prev, cur = cur, (xb if cur is xa else xa)
    return out, results
