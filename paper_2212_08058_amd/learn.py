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
from .api import Kernel, _stream_ptr, problem_for, scale, workspace_bytes


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
        return scale(g, 1.0, s_dev=g_out.detach().to(torch.float64).reshape(1).contiguous()), None


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


# ---------------------------------------------------------------------------
# The paper's objective (SFSeg++) on the single-field operator: Eq. 9's
# sigmoid-affine combination with bias, Alg. 1's loop with soft-binarised
# iterations after the first n_cont, and the Focal-Dice loss of Eq. 12.
# ---------------------------------------------------------------------------

class SFSegPP(torch.autograd.Function):
    """Output of Alg. 1's loop on f = sigmoid(sum_c w_c fc_c + b).

    Every iteration applies A and normalises; iterations after the first
    n_cont are then soft-binarised, b = sigmoid(kappa (sqrt(N) y - theta)),
    and the next iteration takes b (normalised inside the step). The output is
    the last soft mask (or the unit iterate if n_cont = n_iter). The whole
    tape is kept (n_iter volumes); the backward runs the library's adjoint
    step, soft-binarisation backward and combination backward."""

    @staticmethod
    def forward(ctx, fc, w, b, kern: Kernel, n_iter: int, n_cont: int, kappa: float, theta: float):
        if fc.dim() != 4 or not fc.is_cuda or not fc.is_contiguous() or fc.dtype not in (torch.float32,
                                                                                         torch.float64):
            raise ValueError("fc must be a contiguous float32/float64 device tensor [C][T][H][W]")
        if n_iter < 1 or not 0 <= n_cont <= n_iter:
            raise ValueError("need n_iter >= 1 and 0 <= n_cont <= n_iter")
        C, T, H, W = fc.shape
        n = T * H * W
        dev, dt = fc.device, fc.dtype
        p = problem_for((T, H, W), kern, dt)
        ws = torch.empty(workspace_bytes((T, H, W), kern, dt), dtype=torch.uint8, device=dev)
        aux = _aux_ws(dev)
        wd = w.detach().to(torch.float64).contiguous()
        bd = b.detach().to(torch.float64).reshape(1).contiguous()
        f = torch.empty((T, H, W), dtype=dt, device=dev)
        N.check(N.lib.stpi_combine_sigmoid_fwd(C, n, _dt(fc), fc.data_ptr(), wd.data_ptr(), bd.data_ptr(),
                                               f.data_ptr(), _stream_ptr(None)))
        # tape: the input of every step (and its norm), its output, v, and the output's norm
        norms_in = torch.empty(n_iter + 1, dtype=torch.float64, device=dev)
        norms_out = torch.empty(n_iter, dtype=torch.float64, device=dev)
        z = torch.empty((T, H, W), dtype=dt, device=dev)
        N.check(N.lib.stpi_train_init(ctypes.byref(p), z.data_ptr(), norms_in.data_ptr(), _stream_ptr(None)))
        ins, outs, vs = [z], [], []
        for it in range(n_iter):
            zo = torch.empty_like(z)
            v = torch.empty_like(z)
            N.check(N.lib.stpi_train_step(ctypes.byref(p), f.data_ptr(), ins[-1].data_ptr(),
                                          norms_in[it:].data_ptr(), zo.data_ptr(), v.data_ptr(),
                                          norms_out[it:].data_ptr(), ws.data_ptr(), ws.numel(), _stream_ptr(None)))
            outs.append(zo)
            vs.append(v)
            if it >= n_cont:
                bb = torch.empty_like(z)
                N.check(N.lib.stpi_softbin_fwd(n, _dt(fc), zo.data_ptr(), norms_out[it:].data_ptr(), float(kappa),
                                               float(theta), bb.data_ptr(), norms_in[it + 1:].data_ptr(),
                                               aux.data_ptr(), aux.numel(), _stream_ptr(None)))
                ins.append(bb)
            else:
                ins.append(zo)
                norms_in[it + 1:it + 2].copy_(norms_out[it:it + 1])
        if n_cont < n_iter:
            x = ins[-1]
        else:
            x = torch.empty_like(z)
            N.check(N.lib.stpi_normalize(n, _dt(fc), outs[-1].data_ptr(), norms_out[n_iter - 1:].data_ptr(),
                                         x.data_ptr(), _stream_ptr(None)))
        ctx.save = dict(fc=fc, f=f, p=p, ws=ws, aux=aux, ins=ins, outs=outs, vs=vs, norms_in=norms_in,
                        norms_out=norms_out, n_iter=n_iter, n_cont=n_cont, kappa=kappa, n=n, C=C,
                        w_dtype=w.dtype, b_dtype=b.dtype)
        return x.clone() if n_cont < n_iter else x

    @staticmethod
    def backward(ctx, g_x):
        S = ctx.save
        fc, f, p, ws, aux, n = S["fc"], S["f"], S["p"], S["ws"], S["aux"], S["n"]
        ins, outs, vs, nin, nout = S["ins"], S["outs"], S["vs"], S["norms_in"], S["norms_out"]
        K, n_cont, kappa = S["n_iter"], S["n_cont"], S["kappa"]
        dt = _dt(f)
        s = _stream_ptr(None)
        g = g_x.to(f.dtype).contiguous().clone()
        d = torch.empty(K + 1, dtype=torch.float64, device=f.device)
        g_new = torch.empty_like(g)
        # gradient w.r.t. the unit output y_K of the last step, and <y_K, g>
        if K > n_cont:
            N.check(N.lib.stpi_softbin_bwd(n, dt, 0, g.data_ptr(), None, ins[K].data_ptr(), None,
                                           outs[K - 1].data_ptr(), nout[K - 1:].data_ptr(), float(kappa),
                                           g_new.data_ptr(), d[K:].data_ptr(), aux.data_ptr(), aux.numel(), s))
            g, g_new = g_new, g
        else:
            N.check(N.lib.stpi_dot(n, dt, outs[K - 1].data_ptr(), nout[K - 1:].data_ptr(), g.data_ptr(),
                                   d[K:].data_ptr(), aux.data_ptr(), aux.numel(), s))
        g_f = torch.zeros_like(f)
        for k in range(K - 1, -1, -1):
            # step k: input ins[k] (norm nin[k]), output outs[k] (norm nout[k]); g is w.r.t. outs[k] / nout[k]
            N.check(N.lib.stpi_adjoint_step(ctypes.byref(p), f.data_ptr(), ins[k].data_ptr(), nin[k:].data_ptr(),
                                            outs[k].data_ptr(), nout[k:].data_ptr(), vs[k].data_ptr(), g.data_ptr(),
                                            d[k + 1:].data_ptr(), g_new.data_ptr(), g_f.data_ptr(),
                                            d[k:].data_ptr(), ws.data_ptr(), ws.numel(), s))
            g, g_new = g_new, g  # now w.r.t. ins[k] / nin[k]
            if k >= 1 and k - 1 >= n_cont:
                # ins[k] is the soft mask made from outs[k - 1]
                N.check(N.lib.stpi_softbin_bwd(n, dt, 1, g.data_ptr(), d[k:].data_ptr(), ins[k].data_ptr(),
                                               nin[k:].data_ptr(), outs[k - 1].data_ptr(), nout[k - 1:].data_ptr(),
                                               float(kappa), g_new.data_ptr(), d[k:].data_ptr(), aux.data_ptr(),
                                               aux.numel(), s))
                g, g_new = g_new, g
        g_wb = torch.empty(S["C"] + 1, dtype=torch.float64, device=f.device)
        N.check(N.lib.stpi_combine_sigmoid_bwd(S["C"], n, dt, fc.data_ptr(), f.data_ptr(), g_f.data_ptr(),
                                               g_wb.data_ptr(), aux.data_ptr(), aux.numel(), s))
        return (None, g_wb[:S["C"]].to(S["w_dtype"]), g_wb[S["C"]].reshape(()).to(S["b_dtype"]), None, None, None,
                None, None)


def sfseg_pp(fc, w, b, kern: Kernel, n_iter: int = 10, n_cont: int = 5, kappa: float = 2.0,
             theta: float = 1.0) -> torch.Tensor:
    return SFSegPP.apply(fc, w, b, kern, n_iter, n_cont, kappa, theta)


class FocalDiceLoss(torch.autograd.Function):
    """Eq. 12 per frame, soft Dice, with the library's forward and gradient (stpi_focal_dice)."""

    @staticmethod
    def forward(ctx, x: torch.Tensor, gt: torch.Tensor, gamma: float, eps: float):
        xc = x.detach().contiguous()
        gtb = gt.to(torch.uint8).contiguous()
        T = xc.shape[0]
        plane = xc.numel() // T
        loss = torch.empty((), dtype=torch.float64, device=x.device)
        g = torch.empty_like(xc)
        wsz = int(N.lib.stpi_focal_dice_workspace_bytes(T))
        ws = torch.empty(wsz, dtype=torch.uint8, device=x.device)
        N.check(N.lib.stpi_focal_dice(T, plane, _dt(xc), xc.data_ptr(), gtb.data_ptr(), float(gamma), float(eps),
                                      loss.data_ptr(), g.data_ptr(), ws.data_ptr(), wsz, _stream_ptr(None)))
        ctx.save_for_backward(g)
        return loss.to(x.dtype)

    @staticmethod
    def backward(ctx, g_out):
        (g,) = ctx.saved_tensors
        return scale(g, 1.0, s_dev=g_out.detach().to(torch.float64).reshape(1).contiguous()), None, None, None


def focal_dice(x, gt, gamma: float = 0.75, eps: float = 1.0):
    return FocalDiceLoss.apply(x, gt, gamma, eps)
