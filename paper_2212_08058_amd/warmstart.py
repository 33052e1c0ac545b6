"""Warm starts: a two-level (coarse-grid) start and a learned 3x3x3 conv net.

Two-level start: f is box-averaged to a coarse grid (sy x sy pixels, st
frames per cell), the power iteration runs there with the filter in coarse
units, and its eigenvector, prolongated back and multiplied by f, starts the
full-resolution iteration. On clips with several objects the slowest modes of
the iteration are the competition between objects far apart; the coarse
iteration settles them at a fraction of the cost.

Learned start: a 4-layer 3x3x3 conv net maps its input volume to the start
vector, trained on eigenvectors of the plain method (uniform start, tight
tolerance) with the library's forward/backward kernels and AdamW; its output
gives x0 = max(y, 0) + eps. Its input is either f, or the two-level start
(scaled to O(1)), which the net then refines locally.

The plain uniform-start iteration stays the fallback of every warm start: if,
from the warm start, the residual of the second step exceeds that of the
first (r2 > r1), the run restarts from the uniform vector (the wasted steps
count in its time).
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np
import torch

from . import _native as N
from .api import (Kernel, _stream_ptr, coarse_problem, downsample, power_iterate, problem_for, scale, upsample,
                  workspace_bytes)
from .learn import AdamW

CHANNELS = (1, 16, 16, 16, 1)


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-style random initialisation of the FP32 master parameters (flat)."""
    rng = np.random.default_rng(seed)
    chunks = []
    for li in range(4):
        cin, cout = CHANNELS[li], CHANNELS[li + 1]
        fan_in = cin * 27
        w = rng.standard_normal((cout, cin, 3, 3, 3)) * math.sqrt(2.0 / fan_in)
        b = np.zeros(cout)
        if li == 3:
            b[:] = 1.0  # start from a roughly uniform output
        chunks += [w.reshape(-1), b]
    flat = np.concatenate(chunks).astype(np.float32)
    assert flat.size == N.lib.stpi_net_param_count()
    return torch.from_numpy(flat).to(device)


def unflatten(flat) -> list:
    """[(w, b)] per layer (numpy, PyTorch conv3d layout) from the flat master vector."""
    a = flat.detach().double().cpu().numpy() if isinstance(flat, torch.Tensor) else np.asarray(flat, np.float64)
    out, off = [], 0
    for li in range(4):
        cin, cout = CHANNELS[li], CHANNELS[li + 1]
        n = cout * cin * 27
        w = a[off:off + n].reshape(cout, cin, 3, 3, 3)
        off += n
        b = a[off:off + cout]
        off += cout
        out.append((w, b))
    return out


class WarmStartNet:
    def __init__(self, params: torch.Tensor | None = None, device="cuda", lr=2e-3, weight_decay=0.0):
        self.device = torch.device(device)
        self.params = init_params(device=device) if params is None else params.to(device).contiguous()
        self.prep = torch.empty(N.lib.stpi_net_prep_bytes(), dtype=torch.uint8, device=self.device)
        self.grad = torch.zeros_like(self.params)
        self.opt = AdamW([self.params], lr=lr, weight_decay=weight_decay)
        self._ws = {}
        self.prepare()

    def prepare(self):
        N.check(N.lib.stpi_net_prepare(self.params.data_ptr(), self.prep.data_ptr(), _stream_ptr(None)))

    def _workspace(self, shape):
        key = tuple(shape)
        if key not in self._ws:
            p = problem_for(shape, Kernel(1.0, 1.0, 0, 0), torch.float32)
            n = N.lib.stpi_net_workspace_bytes(ctypes.byref(p))
            self._ws = {key: torch.empty(n, dtype=torch.uint8, device=self.device)}
        return self._ws[key]

    def forward(self, f: torch.Tensor) -> torch.Tensor:
        p = problem_for(f.shape, Kernel(1.0, 1.0, 0, 0), torch.float32)
        ws = self._workspace(f.shape)
        y = torch.empty_like(f)
        N.check(N.lib.stpi_net_forward(ctypes.byref(p), f.data_ptr(), self.prep.data_ptr(), y.data_ptr(),
                                       ws.data_ptr(), ws.numel(), _stream_ptr(None)))
        return y

    def backward(self, f: torch.Tensor, y: torch.Tensor, x_star: torch.Tensor) -> torch.Tensor:
        """Gradient into self.grad after forward(f) = y; returns the device loss."""
        p = problem_for(f.shape, Kernel(1.0, 1.0, 0, 0), torch.float32)
        ws = self._workspace(f.shape)
        loss = torch.empty((), dtype=torch.float64, device=self.device)
        N.check(N.lib.stpi_net_backward(ctypes.byref(p), f.data_ptr(), self.prep.data_ptr(), y.data_ptr(),
                                        x_star.data_ptr(), loss.data_ptr(), self.grad.data_ptr(), ws.data_ptr(),
                                        ws.numel(), _stream_ptr(None)))
        return loss

    def train_step(self, f: torch.Tensor, x_star: torch.Tensor) -> torch.Tensor:
        y = self.forward(f)
        loss = self.backward(f, y, x_star)
        self.opt.step([self.grad])
        self.prepare()
        return loss

    def x0(self, f: torch.Tensor, eps: float = 1e-6) -> torch.Tensor:
        y = self.forward(f)
        x0 = torch.empty_like(y)
        N.check(N.lib.stpi_net_warm_start(y.numel(), y.data_ptr(), float(eps), x0.data_ptr(), _stream_ptr(None)))
        return x0


class TwoLevel:
    """Coarse-grid start for clips of one shape (buffers kept for graph reuse)."""

    def __init__(self, shape, kern: Kernel, sy: int = 4, st: int = 2, mode: int = 1, tol: float = 1e-4,
                 cap: int = 2000, device="cuda"):
        self.shape = tuple(int(v) for v in shape)
        self.sy, self.st, self.mode, self.tol, self.cap = int(sy), int(st), int(mode), float(tol), int(cap)
        self.cshape, self.kc = coarse_problem(self.shape, kern, sy, st)
        self.fc = torch.empty(self.cshape, dtype=torch.float32, device=device)
        self.xc = torch.empty_like(self.fc)
        self.wsc = torch.empty(workspace_bytes(self.cshape, self.kc), dtype=torch.uint8, device=device)
        self.u0 = torch.empty(self.shape, dtype=torch.float32, device=device)
        self.last = None

    def start(self, f: torch.Tensor, stream=None) -> torch.Tensor:
        """u0 = f * up(x_coarse) (not normalised; iterate normalises it)."""
        downsample(f, self.sy, self.st, out=self.fc, stream=stream)
        _, r = power_iterate(self.fc, self.kc, tol=self.tol, max_iters=self.cap, x=self.xc, ws=self.wsc,
                             stream=stream, check=False)
        self.last = r
        return upsample(self.xc, self.shape, self.sy, self.st, self.mode, mul=f, out=self.u0, stream=stream)

    def net_input(self, u0: torch.Tensor) -> torch.Tensor:
        """The start scaled to O(1) for the net: u0 * sqrt(coarse voxels)."""
        return scale(u0, math.sqrt(self.fc.numel()))


def solve_from(x0: torch.Tensor, f, kern, tol=1e-4, cap=2000, x=None, ws=None, stream=None):
    """Iterate from x0 with the fallback rule; x0 is copied into x (or used as x).

    One device chain: it stops after its second step if that residual is
    above the first (the rule is checked on the device), and only then is the
    iteration restarted from the uniform start. A warm start the iteration
    cannot use at all (a zero or non-finite norm on its first steps: e.g. an
    x0 that vanishes wherever f > 0, or a non-finite net output) falls back
    the same way. Returns (x, info dict); info has iters (all applications,
    including the fallback's wasted ones), fallback flag, r1, r2, converged,
    residual.
    """
    if x is None:
        x = x0
    elif x.data_ptr() != x0.data_ptr():
        x.copy_(x0)
    x, r = power_iterate(f, kern, tol=tol, max_iters=cap, x0=x, x=x, ws=ws, stream=stream, check=False,
                         rise_check=True)
    failed = bool(r["flags"] & 3)  # zero or non-finite norm
    info = dict(r1=r["r1"], r2=r["r2"] if r["iters"] >= 2 else None, fallback=bool(r["flags"] & 4) or failed,
                iters=r["iters"], converged=r["converged"], residual=r["residual"])
    if info["fallback"]:
        x, r2 = power_iterate(f, kern, tol=tol, max_iters=cap, x=x, ws=ws, stream=stream, check=False)
        info.update(iters=r["iters"] + r2["iters"], converged=r2["converged"], residual=r2["residual"])
    return x, info


def solve_plain(f, kern, tol=1e-4, cap=2000, x=None, ws=None, stream=None):
    """Uniform start to tolerance; returns (x, result, seconds)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, r = power_iterate(f, kern, tol=tol, max_iters=cap, x=x, ws=ws, stream=stream, check=False)
    torch.cuda.synchronize()
    return x, r, time.perf_counter() - t0


def solve_warm(net: WarmStartNet, f, kern, tol=1e-4, cap=2000, x=None, ws=None, stream=None):
    """Net start from f, with the fallback; returns (x, info, seconds)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, info = solve_from(net.x0(f), f, kern, tol, cap, x, ws, stream)
    torch.cuda.synchronize()
    return x, info, time.perf_counter() - t0


def solve_two_level(tl: TwoLevel, f, kern, net: WarmStartNet | None = None, tol=1e-4, cap=2000, x=None, ws=None,
                    stream=None):
    """Two-level start (refined by the net if given), with the fallback.

    Returns (x, info, seconds); info adds the coarse iteration count."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    u0 = tl.start(f, stream)
    x0 = net.x0(tl.net_input(u0)) if net is not None else u0
    x, info = solve_from(x0, f, kern, tol, cap, x, ws, stream)
    torch.cuda.synchronize()
    info["coarse_iters"] = tl.last["iters"]
    return x, info, time.perf_counter() - t0
