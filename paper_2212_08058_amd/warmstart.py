"""Learned warm start: a 4-layer 3x3x3 conv net predicts the start vector.

Training targets are eigenvectors computed by the plain method (uniform start,
tight tolerance). The net is trained with the library's own forward/backward
kernels and AdamW; at inference its output gives x0 = max(y, 0) + eps. The
plain uniform-start iteration stays the fallback: if, from the warm start, the
residual of the second step exceeds that of the first (r2 > r1), the run
restarts from the uniform vector (the two wasted steps count in its time).
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np
import torch

from . import _native as N
from .api import Kernel, _stream_ptr, power_iterate, problem_for, workspace_bytes
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


def solve_plain(f, kern, tol=1e-4, cap=2000, ws=None, stream=None):
    """Uniform start to tolerance; returns (x, result, seconds)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x, r = power_iterate(f, kern, tol=tol, max_iters=cap, ws=ws, stream=stream, check=False)
    torch.cuda.synchronize()
    return x, r, time.perf_counter() - t0


def solve_warm(net: WarmStartNet, f, kern, tol=1e-4, cap=2000, ws=None, stream=None):
    """Net start, fallback to uniform when the second residual exceeds the first.

    Returns (x, info dict, seconds); info has iters (all applications,
    including the fallback's wasted ones), fallback flag, r1, r2.
    """
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    x = net.x0(f)
    _, r1 = power_iterate(f, kern, iters=1, x0=x, x=x, ws=ws, stream=stream, check=False)
    if r1["residual"] < tol:
        torch.cuda.synchronize()
        return x, dict(iters=1, fallback=False, r1=r1["residual"], r2=None, converged=True,
                       residual=r1["residual"]), time.perf_counter() - t0
    _, r2 = power_iterate(f, kern, iters=1, x0=x, x=x, ws=ws, stream=stream, check=False)
    info = dict(r1=r1["residual"], r2=r2["residual"], fallback=False)
    if not (r2["residual"] <= r1["residual"]):
        info["fallback"] = True
        x, r = power_iterate(f, kern, tol=tol, max_iters=cap, x=x, ws=ws, stream=stream, check=False)
        info.update(iters=2 + r["iters"], converged=r["converged"], residual=r["residual"])
    elif r2["residual"] < tol:
        info.update(iters=2, converged=True, residual=r2["residual"])
    else:
        x, r = power_iterate(f, kern, tol=tol, max_iters=cap - 2, x0=x, x=x, ws=ws, stream=stream, check=False)
        info.update(iters=2 + r["iters"], converged=r["converged"], residual=r["residual"])
    torch.cuda.synchronize()
    return x, info, time.perf_counter() - t0
