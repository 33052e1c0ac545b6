"""Learning the channel combination end to end through the power iteration.

The paper learns per-channel weights by back-propagating a segmentation loss
through every spectral iteration (Sec. 3.4). Here:

* ``SpectralIterate`` is a ``torch.autograd.Function`` whose forward combines
  the channels (f = sum_c softmax(w)_c fc_c) and runs `iters` normalised
  power-iteration steps on the device, keeping only every `ckpt`-th iterate;
  its backward recomputes each segment from its checkpoint (saving
  v_k = G (f x_k)), then runs the hand-written adjoint kernels in reverse and
  finishes with the combination's backward. Nothing is differentiated by
  torch: every arithmetic step runs in libstpi's kernels.
* ``BCELoss`` is the binary cross-entropy on x / max(x) with its gradient
  from the library.
* ``AdamW`` wraps the library's AdamW kernel (Eq. 13, with AMSGrad).
"""
from __future__ import annotations

import ctypes

import torch

from . import _native as N
from .api import Kernel, _stream_ptr, problem_for, workspace_bytes


def _dt(t: torch.Tensor) -> int:
    return {torch.float32: N.STPI_F32, torch.bfloat16: N.STPI_BF16, torch.float64: N.STPI_F64}[t.dtype]


def _aux_ws(device) -> torch.Tensor:
    return torch.empty(N.AUX_WS_BYTES, dtype=torch.uint8, device=device)


def combine(fc: torch.Tensor, w: torch.Tensor, stream=None) -> torch.Tensor:
    """f = sum_c softmax(w)_c fc[c] (stpi_combine_fwd). fc [C][T][H][W], w [C] logits."""
    C = fc.shape[0]
    f = torch.empty(fc.shape[1:], dtype=fc.dtype, device=fc.device)
    wf = w.detach().to(torch.float64).contiguous()
    N.check(N.lib.stpi_combine_fwd(C, f.numel(), _dt(fc), fc.data_ptr(), wf.data_ptr(), f.data_ptr(),
                                   _stream_ptr(stream)))
    return f


class _Tape:
    """Device buffers of one forward pass: f, norms, checkpoints and workspaces."""

    def __init__(self, fc, w, kern, iters, ckpt):
        self.C, T, H, W = fc.shape
        self.shape = (T, H, W)
        self.n = T * H * W
        self.kern = kern
        self.iters = iters
        self.ckpt = ckpt
        self.dtype = fc.dtype
        self.dev = fc.device
        self.p = problem_for(self.shape, kern, fc.dtype)
        self.ws = torch.empty(workspace_bytes(self.shape, kern, fc.dtype), dtype=torch.uint8, device=self.dev)
        self.aux = _aux_ws(self.dev)
        self.norms = torch.empty(iters + 1, dtype=torch.float64, device=self.dev)

    def vol(self):
        return torch.empty(self.shape, dtype=self.dtype, device=self.dev)

    def step(self, f, z_in, k, z_out, v_out, norm_out):
        N.check(N.lib.stpi_train_step(ctypes.byref(self.p), f.data_ptr(), z_in.data_ptr(),
                                      self.norms[k:].data_ptr(), z_out.data_ptr(),
                                      v_out.data_ptr() if v_out is not None else None,
                                      norm_out.data_ptr(), self.ws.data_ptr(), self.ws.numel(), _stream_ptr(None)))


class SpectralIterate(torch.autograd.Function):
    """x_K of `iters` normalised power-iteration steps on f = combine(fc, w)."""

    @staticmethod
    def forward(ctx, fc: torch.Tensor, w: torch.Tensor, kern: Kernel, iters: int, ckpt: int):
        if fc.dim() != 4 or not fc.is_cuda or not fc.is_contiguous():
            raise ValueError("fc must be a contiguous device tensor [C][T][H][W]")
        if iters < 1 or ckpt < 1:
            raise ValueError("iters and ckpt must be >= 1")
        tp = _Tape(fc, w, kern, iters, ckpt)
        f = combine(fc, w)
        saved = {}
        z = tp.vol()
        N.check(N.lib.stpi_train_init(ctypes.byref(tp.p), z.data_ptr(), tp.norms.data_ptr(), _stream_ptr(None)))
        saved[0] = z
        spare = [tp.vol(), tp.vol()]
        for k in range(iters):
            keep = (k + 1) % ckpt == 0 or k + 1 == iters
            z_out = tp.vol() if keep else spare[k % 2]
            tp.step(f, z, k, z_out, None, tp.norms[k + 1:])
            if keep:
                saved[k + 1] = z_out
            z = z_out
        x = tp.vol()
        N.check(N.lib.stpi_normalize(tp.n, _dt(fc), z.data_ptr(), tp.norms[iters:].data_ptr(), x.data_ptr(),
                                     _stream_ptr(None)))
        ctx.tape = tp
        ctx.saved = saved
        ctx.fc = fc
        ctx.w = w.detach().to(torch.float64).contiguous()
        ctx.f = f
        ctx.w_dtype = w.dtype
        return x

    @staticmethod
    def backward(ctx, g_x):
        tp, saved, f = ctx.tape, ctx.saved, ctx.f
        K, ck = tp.iters, tp.ckpt
        g = g_x.to(tp.dtype).contiguous().clone()
        d = torch.empty(K + 1, dtype=torch.float64, device=tp.dev)
        rec_norms = torch.empty(K + 1, dtype=torch.float64, device=tp.dev)
        N.check(N.lib.stpi_dot(tp.n, _dt(f), saved[K].data_ptr(), tp.norms[K:].data_ptr(), g.data_ptr(),
                               d[K:].data_ptr(), tp.aux.data_ptr(), tp.aux.numel(), _stream_ptr(None)))
        g_f = torch.zeros_like(f)
        g_new = tp.vol()
        seg_starts = list(range(0, K, ck))
        for s0 in reversed(seg_starts):
            s1 = min(s0 + ck, K)
            zs = [saved[s0]]
            vs = []
            for k in range(s0, s1):
                z_out = saved[k + 1] if k + 1 == s1 else tp.vol()
                v = tp.vol()
                if k + 1 == s1:
                    # the checkpoint of the next segment already holds z_{s1}; recompute into a temporary to get v
                    tmp = tp.vol()
                    tp.step(f, zs[-1], k, tmp, v, rec_norms[k + 1:])
                    del tmp
                else:
                    tp.step(f, zs[-1], k, z_out, v, rec_norms[k + 1:])
                zs.append(z_out)
                vs.append(v)
            for k in range(s1 - 1, s0 - 1, -1):
                j = k - s0
                N.check(N.lib.stpi_adjoint_step(ctypes.byref(tp.p), f.data_ptr(), zs[j].data_ptr(),
                                                tp.norms[k:].data_ptr(), zs[j + 1].data_ptr(),
                                                tp.norms[k + 1:].data_ptr(), vs[j].data_ptr(), g.data_ptr(),
                                                d[k + 1:].data_ptr(), g_new.data_ptr(), g_f.data_ptr(),
                                                d[k:].data_ptr(), tp.ws.data_ptr(), tp.ws.numel(),
                                                _stream_ptr(None)))
                g, g_new = g_new, g
        g_w = torch.empty(tp.C, dtype=torch.float64, device=tp.dev)
        N.check(N.lib.stpi_combine_bwd(tp.C, tp.n, _dt(f), ctx.fc.data_ptr(), ctx.w.data_ptr(), g_f.data_ptr(),
                                       g_w.data_ptr(), tp.aux.data_ptr(), tp.aux.numel(), _stream_ptr(None)))
        ctx.g_f = g_f
        return None, g_w.to(ctx.w_dtype), None, None, None


def spectral_iterate(fc, w, kern: Kernel, iters: int = 15, ckpt: int = 5) -> torch.Tensor:
    return SpectralIterate.apply(fc, w, kern, iters, ckpt)


class BCELoss(torch.autograd.Function):
    """BCE(clip(x / max x), gt) with the library's forward and gradient (stpi_bce)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, gt: torch.Tensor):
        xc = x.detach().contiguous()
        gtb = gt.to(torch.uint8).contiguous()
        loss = torch.empty((), dtype=torch.float64, device=x.device)
        g = torch.empty_like(xc)
        aux = _aux_ws(x.device)
        N.check(N.lib.stpi_bce(xc.numel(), _dt(xc), xc.data_ptr(), gtb.data_ptr(), loss.data_ptr(), g.data_ptr(),
                               aux.data_ptr(), aux.numel(), _stream_ptr(None)))
        ctx.save_for_backward(g)
        return loss.to(x.dtype if x.dtype != torch.bfloat16 else torch.float32)

    @staticmethod
    def backward(ctx, g_out):
        (g,) = ctx.saved_tensors
        return g * g_out.to(g.dtype), None


def bce(x, gt):
    return BCELoss.apply(x, gt)


class AdamW:
    """AdamW with AMSGrad on float32 or float64 device parameters (stpi_adamw)."""

    def __init__(self, params, lr=1e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01, amsgrad=True):
        self.params = [p for p in params]
        for p in self.params:
            if p.dtype not in (torch.float32, torch.float64) or not p.is_cuda or not p.is_contiguous():
                raise ValueError("AdamW parameters must be contiguous float32/float64 device tensors")
        self.lr, self.betas, self.eps, self.wd, self.amsgrad = lr, betas, eps, weight_decay, amsgrad
        self.state = [(torch.zeros_like(p), torch.zeros_like(p), torch.zeros_like(p)) for p in self.params]
        self.t = 0

    def step(self, grads=None):
        self.t += 1
        for i, p in enumerate(self.params):
            g = grads[i] if grads is not None else p.grad
            if g is None:
                continue
            g = g.detach().to(p.dtype).contiguous()
            m, v, vm = self.state[i]
            N.check(N.lib.stpi_adamw(p.numel(), _dt(p), p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(),
                                     vm.data_ptr(), self.t, self.lr, self.betas[0], self.betas[1], self.eps,
                                     self.wd, 1 if self.amsgrad else 0, _stream_ptr(None)))
