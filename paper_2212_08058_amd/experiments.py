"""Measurement drivers for the batched, channel-learning and warm-start workloads.

Each returns a plain dict (JSON-ready). All arithmetic runs in libstpi; this
module only generates the synthetic inputs, orders the calls and times them.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

import synth

from . import batch as B
from . import learn
from .api import Kernel, power_iterate
from .warmstart import WarmStartNet, solve_plain, solve_warm


def _sync():
    torch.cuda.synchronize()


def batched_workload(n=48, seed=3000, tol=1e-4, cap=50, reps=3, scale=1, device="cuda", log=print):
    """48 uneven clips (T ~ U{8..96}, frames 240x432 / 360x640 / 480x854), one graph launch per chain.

    scale > 1 divides T, H, W (smaller smoke-sized runs). Returns timing and per-clip outcomes.
    """
    c = synth.CONFIGS["batch"]
    kern = Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    specs = synth.batch_specs(n=n, seed=seed)
    shapes = [(max(1, s.T // scale), max(8, s.H // scale), max(8, s.W // scale)) for s in specs]
    plan = B.BatchPlan(shapes, kern)
    log(f"batched: {len(shapes)} clips, {sum(a * b * c for a, b, c in shapes) / 1e6:.1f} M voxels; plan {plan.info()}")
    f_flat = plan.empty(device)
    for spec, shp, view in zip(specs, shapes, plan.views(f_flat)):
        f, _ = synth.blob_clip(*shp, spec.nblobs, spec.seed)
        view.copy_(torch.from_numpy(f))
    x_flat = plan.empty(device)
    ws = plan.workspace(device)
    stream = torch.cuda.Stream()
    _sync()
    plan.iterate(f_flat, x_flat, max_iters=cap, tol=tol, ws=ws, stream=stream)  # capture + warm-up
    times = []
    for _ in range(reps):
        _sync()
        t0 = time.perf_counter()
        _, res = plan.iterate(f_flat, x_flat, max_iters=cap, tol=tol, ws=ws, stream=stream)
        _sync()
        times.append(time.perf_counter() - t0)
    t = float(np.median(times))
    active = sum(r["iters"] * a * b * cc for r, (a, b, cc) in zip(res, shapes))
    return dict(clips=len(shapes), voxels=int(sum(a * b * cc for a, b, cc in shapes)), seconds=t,
                active_voxel_iters_per_s=active / t, iters=[r["iters"] for r in res],
                converged=sum(bool(r["converged"]) for r in res), capped=sum(not r["converged"] for r in res),
                tol=tol, cap=cap, plan=plan.info())


def channel_training_step(reps=5, device="cuda", log=print):
    """C = 8, 32x240x432, 15 iterations checkpointed every 5, BCE: one forward + backward + AdamW."""
    c = synth.CONFIGS["channels"]
    kern = Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    fc, gt = synth.channel_stack(c["C"], c["T"], c["H"], c["W"], seed=c["seed"])
    fcd = torch.from_numpy(fc).to(device)
    gtd = torch.from_numpy(gt).to(device)
    w = torch.zeros(c["C"], dtype=torch.float64, device=device, requires_grad=True)
    opt = learn.AdamW([w], lr=0.1, weight_decay=0.0)

    def step():
        w.grad = None
        x = learn.spectral_iterate(fcd, w, kern, c["iters"], c["ckpt"])
        L = learn.bce(x, gtd)
        L.backward()
        opt.step()
        return L

    step()
    _sync()
    ts, losses = [], []
    for _ in range(reps):
        _sync()
        t0 = time.perf_counter()
        L = step()
        _sync()
        ts.append(time.perf_counter() - t0)
        losses.append(float(L))
    t = float(np.median(ts))
    N = c["T"] * c["H"] * c["W"]
    # forward 15 steps + recompute 15 + 15 adjoint steps
    return dict(seconds_per_step=t, losses=losses, voxels=N, iters=c["iters"], ckpt=c["ckpt"],
                weights=torch.softmax(w.detach(), 0).cpu().tolist(),
                step_voxel_iters_per_s=N * 3 * c["iters"] / t)


def warm_start_experiment(n_train=2000, n_eval=200, epochs=2, train_shape=(16, 240, 432), eval_shape=(32, 480, 854),
                          tol=1e-4, target_tol=1e-6, cap=2000, lr=2e-3, device="cuda", log=print):
    """Train the warm-start net on plain-method eigenvectors, then compare wall time to tol."""
    c = synth.CONFIGS["warm"]
    kern = Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    net = WarmStartNet(lr=lr, device=device)
    t_gen = time.perf_counter()
    train = []
    for i in range(n_train):
        f, _ = synth.blob_clip(*train_shape, 3, c["train_seed"] + i)
        fd = torch.from_numpy(f).to(device)
        x, r = power_iterate(fd, kern, tol=target_tol, max_iters=20000, check=False)
        train.append((fd, x.clone()))
    _sync()
    log(f"warm start: {n_train} training targets in {time.perf_counter() - t_gen:.1f} s")
    rng = np.random.default_rng(0)
    hist = []
    t_train = time.perf_counter()
    for ep in range(epochs):
        tot = torch.zeros((), dtype=torch.float64, device=device)
        for i in rng.permutation(n_train):
            tot += net.train_step(*train[i])
        hist.append(float(tot) / n_train)
        log(f"  epoch {ep}: mean loss {hist[-1]:.4f}")
    _sync()
    train_s = time.perf_counter() - t_train
    del train
    ws = None
    plain_t, warm_t, rows = [], [], []
    for i in range(n_eval):
        f, _ = synth.blob_clip(*eval_shape, 3, c["eval_seed"] + i)
        fd = torch.from_numpy(f).to(device)
        if i == 0:  # warm-up (graph capture, allocations)
            solve_plain(fd, kern, tol=tol, cap=cap)
            solve_warm(net, fd, kern, tol=tol, cap=cap)
        xp, rp, tp = solve_plain(fd, kern, tol=tol, cap=cap)
        xw, iw, tw = solve_warm(net, fd, kern, tol=tol, cap=cap)
        x0 = net.x0(fd)
        cosd = 1.0 - float(torch.sum(x0.double() * xp.double()) / torch.linalg.vector_norm(x0.double()))
        plain_t.append(tp)
        warm_t.append(tw)
        rows.append(dict(plain_iters=rp["iters"], warm_iters=iw["iters"], fallback=iw["fallback"],
                         plain_s=tp, warm_s=tw, x0_cos_dist=cosd,
                         agree_cos_dist=1.0 - float(torch.sum(xp.double() * xw.double()))))
    ratios = [p / w for p, w in zip(plain_t, warm_t)]
    return dict(n_train=n_train, n_eval=n_eval, epochs=epochs, train_shape=train_shape, eval_shape=eval_shape,
                loss_history=hist, train_seconds=train_s, sum_ratio=sum(plain_t) / sum(warm_t),
                median_ratio=float(np.median(ratios)), fallbacks=sum(r["fallback"] for r in rows),
                plain_iters=[r["plain_iters"] for r in rows], warm_iters=[r["warm_iters"] for r in rows],
                rows=rows)
