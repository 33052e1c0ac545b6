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
from .api import workspace_bytes
from .warmstart import TwoLevel, WarmStartNet, solve_plain, solve_two_level, solve_warm


def _sync():
    torch.cuda.synchronize()


def batched_workload(n=48, seed=3000, tol=1e-4, cap=50, reps=3, scale=1, autotune=True, device="cuda", log=print):
    """48 uneven clips (T ~ U{8..96}, frames 240x432 / 360x640 / 480x854), one graph launch per chain.

    scale > 1 divides T, H, W (smaller smoke-sized runs). Returns timing and per-clip outcomes.
    """
    c = synth.CONFIGS["batch"]
    kern = Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    specs = synth.batch_specs(n=n, seed=seed)
    shapes = [(max(1, s.T // scale), max(8, s.H // scale), max(8, s.W // scale)) for s in specs]
    # the project autotuner times the step variants on the frame size carrying
    # the most voxels; the plan takes its choice
    by_frame = {}
    for T, H, W in shapes:
        by_frame[(H, W)] = by_frame.get((H, W), 0) + T * H * W
    H0, W0 = max(by_frame, key=by_frame.get)
    tuned, tuned_ms = (B.autotune((64, H0, W0), kern, reps=5) if autotune else (None, None))
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
    elem = 4 if plan.dtype == torch.float32 else 2
    rate = active / t
    return dict(clips=len(shapes), voxels=int(sum(a * b * cc for a, b, cc in shapes)), seconds=t,
                active_voxel_iters_per_s=rate, hbm_frac=3 * elem * rate / 8.0e12,
                iters=[r["iters"] for r in res],
                converged=sum(bool(r["converged"]) for r in res), capped=sum(not r["converged"] for r in res),
                tol=tol, cap=cap, plan=plan.info(),
                autotuned=None if tuned is None else dict(frame=[H0, W0], variant=tuned, chain_step_ms=tuned_ms))


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


def _targets_batched(fs, kern, tol, cap, device, log):
    """Plain eigenvectors of many clips of one shape in one batched plan."""
    plan = B.BatchPlan([tuple(fs[0].shape)] * len(fs), kern)
    f_flat = plan.pack(fs)
    x_flat, res = plan.iterate(f_flat, max_iters=cap, tol=tol, check=False)
    xs = [v.clone() for v in plan.views(x_flat)]
    iters = [r["iters"] for r in res]
    log(f"  targets: {len(fs)} clips, iterations median {int(np.median(iters))}, max {max(iters)}, "
        f"unconverged {sum(not r['converged'] for r in res)}")
    del f_flat, x_flat, plan
    return xs, iters


def warm_start_experiment(n_train=2000, n_eval=200, epochs=2, train_shape=(16, 240, 432), eval_shape=(32, 480, 854),
                          tol=1e-4, target_tol=1e-6, cap=2000, lr=2e-3, sy=4, st=2, coarse_tol=1e-3, chunk=250,
                          batched=True, device="cuda", log=print):
    """Warm starts against the plain method, wall time to tol per clip.

    Trains two nets with the library's kernels: one on f (net_f) and one on
    the two-level start (net_tl). Evaluates, clip by clip with preallocated
    buffers: plain (uniform start), net_f, two-level, two-level + net_tl; and
    batched: plain vs two-level + net_tl over all evaluation clips.
    """
    c = synth.CONFIGS["warm"]
    kern = Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    t_gen = time.perf_counter()
    fs, xs, tl_in = [], [], []
    tl_train = TwoLevel(train_shape, kern, sy, st, tol=coarse_tol, device=device)
    for c0 in range(0, n_train, chunk):
        fc = [torch.from_numpy(synth.blob_clip(*train_shape, 3, c["train_seed"] + i)[0]).to(device)
              for i in range(c0, min(n_train, c0 + chunk))]
        xc, _ = _targets_batched(fc, kern, target_tol, 20000, device, log)
        for f in fc:
            tl_in.append(tl_train.net_input(tl_train.start(f)).clone())
        fs += fc
        xs += xc
    _sync()
    gen_s = time.perf_counter() - t_gen
    log(f"warm start: {n_train} training clips (targets + two-level inputs) in {gen_s:.1f} s")
    nets = {"net_f": WarmStartNet(lr=lr, device=device), "net_tl": WarmStartNet(lr=lr, device=device)}
    hist = {k: [] for k in nets}
    rng = np.random.default_rng(0)
    t_train = time.perf_counter()
    for ep in range(epochs):
        tot = {k: torch.zeros((), dtype=torch.float64, device=device) for k in nets}
        for i in rng.permutation(n_train):
            tot["net_f"] += nets["net_f"].train_step(fs[i], xs[i])
            tot["net_tl"] += nets["net_tl"].train_step(tl_in[i], xs[i])
        for k in nets:
            hist[k].append(float(tot[k]) / n_train)
        log(f"  epoch {ep}: mean loss net_f {hist['net_f'][-1]:.4f} net_tl {hist['net_tl'][-1]:.4f}")
    _sync()
    train_s = time.perf_counter() - t_train
    del fs, xs, tl_in

    # clip-by-clip evaluation, one set of buffers (captured graphs are reused)
    fbuf = torch.empty(eval_shape, dtype=torch.float32, device=device)
    xbuf = torch.empty_like(fbuf)
    ws = torch.empty(workspace_bytes(eval_shape, kern), dtype=torch.uint8, device=device)
    tl = TwoLevel(eval_shape, kern, sy, st, tol=coarse_tol, device=device)
    modes = ("plain", "net_f", "two_level", "two_level_net")
    times = {m: [] for m in modes}
    iters = {m: [] for m in modes}
    falls = {m: 0 for m in modes}
    coarse_it, cosd = [], {m: [] for m in modes}
    eval_fs = []
    for i in range(-1, n_eval):
        f, _ = synth.blob_clip(*eval_shape, 3, c["eval_seed"] + max(i, 0))
        fbuf.copy_(torch.from_numpy(f))
        if i >= 0:
            eval_fs.append(fbuf.clone())
        xp, rp, tp = solve_plain(fbuf, kern, tol=tol, cap=cap, x=xbuf, ws=ws)
        xref = xp.double().clone()
        runs = {"plain": (rp["iters"], tp, False)}
        _, info, t = solve_warm(nets["net_f"], fbuf, kern, tol=tol, cap=cap, x=xbuf, ws=ws)
        runs["net_f"] = (info["iters"], t, info["fallback"])
        cosd["net_f"].append(1.0 - float(torch.sum(xbuf.double() * xref)))
        _, info, t = solve_two_level(tl, fbuf, kern, tol=tol, cap=cap, x=xbuf, ws=ws)
        runs["two_level"] = (info["iters"], t, info["fallback"])
        cosd["two_level"].append(1.0 - float(torch.sum(xbuf.double() * xref)))
        ci = info["coarse_iters"]
        _, info, t = solve_two_level(tl, fbuf, kern, net=nets["net_tl"], tol=tol, cap=cap, x=xbuf, ws=ws)
        runs["two_level_net"] = (info["iters"], t, info["fallback"])
        cosd["two_level_net"].append(1.0 - float(torch.sum(xbuf.double() * xref)))
        if i < 0:
            continue  # first pass: graph capture and allocations
        if (i + 1) % 25 == 0:
            log(f"  evaluated {i + 1} of {n_eval} clips")
        coarse_it.append(ci)
        for m, (it, t, fb) in runs.items():
            iters[m].append(it)
            times[m].append(t)
            falls[m] += int(fb)
    out = dict(n_train=n_train, n_eval=n_eval, epochs=epochs, train_shape=train_shape, eval_shape=eval_shape,
               coarse=dict(sy=sy, st=st, shape=tl.cshape, kernel=vars(tl.kc), iters_median=float(np.median(coarse_it))),
               gen_seconds=gen_s, train_seconds=train_s, loss_history=hist, tol=tol, cap=cap)
    for m in modes:
        out[m] = dict(seconds=sum(times[m]), iters_median=float(np.median(iters[m])), iters_max=int(max(iters[m])),
                      fallbacks=falls[m])
        if m != "plain":
            out[m]["sum_ratio"] = sum(times["plain"]) / sum(times[m])
            out[m]["median_ratio"] = float(np.median([p / w for p, w in zip(times["plain"], times[m])]))
            out[m]["cos_dist_max"] = float(max(cosd[m]))
    out["iters"] = {m: iters[m] for m in modes}
    out["ms"] = {m: [round(t * 1e3, 3) for t in times[m]] for m in modes}
    out["coarse"]["tol"] = coarse_tol

    if batched:
        # batched: plain (uniform) vs two-level and two-level + net_tl starts, all evaluation clips in one plan
        plan = B.BatchPlan([eval_shape] * n_eval, kern)
        f_flat = plan.pack(eval_fs)
        x_flat = plan.empty(device)
        bws = plan.workspace(device)
        s = torch.cuda.Stream()
        plan.iterate(f_flat, x_flat, max_iters=cap, tol=tol, ws=bws, stream=s, check=False)  # capture
        _sync()
        t0 = time.perf_counter()
        _, res_p = plan.iterate(f_flat, x_flat, max_iters=cap, tol=tol, ws=bws, stream=s, check=False)
        _sync()
        t_bp = time.perf_counter() - t0
        out["batched"] = dict(plain_seconds=t_bp, plain_iters_median=float(np.median([r["iters"] for r in res_p])),
                              unconverged_plain=sum(not r["converged"] for r in res_p))
        for mode in ("two_level", "two_level_net"):
            for rep in range(2):  # first repetition captures the graphs
                _sync()
                t0 = time.perf_counter()
                with torch.cuda.stream(s):
                    for f, xv in zip(eval_fs, plan.views(x_flat)):
                        u0 = tl.start(f, s)
                        xv.copy_(nets["net_tl"].x0(tl.net_input(u0)) if mode == "two_level_net" else u0)
                # the fallback rule runs per clip on the device (init = 2)
                _, res_w = plan.iterate(f_flat, x_flat, init=2, max_iters=cap, tol=tol, ws=bws, stream=s,
                                        check=False)
                _sync()
                t_bw = time.perf_counter() - t0
                nfb = sum(bool(r["flags"] & 4) for r in res_w)
            out["batched"][mode] = dict(seconds=t_bw, ratio_vs_batched_plain=t_bp / t_bw,
                                        ratio_vs_single_plain=sum(times["plain"]) / t_bw, fallbacks=nfb,
                                        iters_median=float(np.median([r["iters"] for r in res_w])),
                                        unconverged=sum(not r["converged"] for r in res_w))
    return out


def online_vs_full(f_np, kern, settings=((16, 8, 5), (16, 8, 10), (32, 16, 10)), full_iters=20, tol=1e-4, cap=2000,
                   reps=3, device="cuda", log=print):
    """Partial iterations over sub-windows (Sec. 4, "Online vs Offline
    processing") against iterating the whole video: wall time, and per-frame
    agreement with the full video's solution converged to `tol` (cosine of the
    frame's vectors, IoU of the masks x >= max(x) / 2 per frame), for the
    windowed run and for a fixed full_iters-iteration full run."""
    from . import online

    f = torch.from_numpy(f_np).to(device)
    x_conv, r_conv = power_iterate(f, kern, tol=tol, max_iters=cap)
    x_full = torch.empty_like(f)
    ws = torch.empty(workspace_bytes(f.shape, kern), dtype=torch.uint8, device=device)
    out = torch.empty_like(f)

    def timed(fn):
        fn()
        _sync()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            _sync()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts))

    t_full = timed(lambda: power_iterate(f, kern, iters=full_iters, x=x_full, ws=ws))

    def agree(x):
        a = x.double()
        b = x_conv.double()
        cos = (a * b).sum(dim=(1, 2)) / (a.norm(dim=(1, 2)) * b.norm(dim=(1, 2)))
        ma = a >= 0.5 * a.amax(dim=(1, 2), keepdim=True)
        mb = b >= 0.5 * b.amax(dim=(1, 2), keepdim=True)
        iou = (ma & mb).sum(dim=(1, 2)).double() / (ma | mb).sum(dim=(1, 2)).clamp(min=1).double()
        return dict(cos_median=float(cos.median()), cos_min=float(cos.min()), iou_median=float(iou.median()),
                    iou_min=float(iou.min()))

    T = f.shape[0]
    res = dict(full_iters=full_iters, converged_iters=r_conv["iters"], seconds_full=t_full,
               frame_iterations_full=T * full_iters, full_vs_converged=agree(x_full), windows=[])
    for q, shift, it in settings:
        t_online = timed(lambda: online.online_iterate(f, kern, q, shift, iters=it, out=out, wait=False))
        nwin = len(online.window_starts(T, q, shift))
        res["windows"].append(dict(q=q, shift=shift, window_iters=it, windows=nwin, seconds=t_online,
                                   speedup_vs_full=t_full / t_online, frame_iterations=nwin * q * it,
                                   vs_converged=agree(out)))
        log(f"  online q={q} shift={shift} iters={it}: {t_online * 1e3:.2f} ms, {res['windows'][-1]['vs_converged']}")
    return res


def noisy_study_fields(shape, seed, noise=0.5, p=0.2):
    """The exact-vs-Taylor study's synthetic input: a soft blob mask with
    heavy additive U[0, noise] noise, clipped to [0, 1], raised to p as the
    unary map s, and the same mask with an independent noise draw as the
    pairwise feature f."""
    T, H, W = shape
    mask, rng = synth.blob_mask(T, H, W, 3, seed)
    S = np.clip(mask + rng.uniform(0.0, noise, mask.shape), 0.0, 1.0)
    F = np.clip(mask + rng.uniform(0.0, noise, mask.shape), 0.0, 1.0)
    return (S ** p).astype(np.float32), F.astype(np.float32), mask


def taylor_study(shape=(10, 20, 20), seed=90, alpha=1.0, iters=30, start_deg=70.0, sigma_s=2.0, sigma_t=1.0,
                 r_s=4, r_t=2, device="cuda", log=print):
    """Sec. 4, "Quantitative analysis": the SFSeg iterates (Taylor affinity,
    Eq. 2 / Eq. 7) against the exact eigenvector of the exponential affinity
    (Eq. 1), from a start start_deg degrees away from it: angle (degrees) and
    IoU of the masks x >= max(x) / 2 after every iteration, the angle between
    the two converged eigenvectors, and the time per iteration of each
    operator on the GPU."""
    from . import sfseg as SF

    kern = Kernel(sigma_s, sigma_t, r_s, r_t)
    s_np, f_np, _ = noisy_study_fields(shape, seed)
    s = torch.from_numpy(s_np).to(device)
    f = torch.from_numpy(f_np).to(device)
    v, rv = SF.exp_iterate(s, f, kern, alpha, tol=1e-8, max_iters=5000)
    xt, rt = SF.sfseg_iterate(s, f, kern, alpha, tol=1e-8, max_iters=5000)
    vd = v.double().reshape(-1)
    vd = vd / vd.norm()
    rng = np.random.default_rng(seed + 1)
    w = torch.from_numpy(rng.uniform(0.0, 1.0, vd.numel())).to(device)
    w = w - (w @ vd) * vd
    w = w / w.norm()
    th = math.radians(start_deg)
    x = (math.cos(th) * vd + math.sin(th) * w).to(torch.float32).reshape(s.shape).contiguous()

    def metrics(xv):
        a = xv.double().reshape(-1)
        a = a / a.norm()
        ang = math.degrees(math.acos(min(1.0, abs(float(a @ vd)))))
        ma, mb = a >= 0.5 * a.max(), vd >= 0.5 * vd.max()
        iou = float((ma & mb).sum()) / max(1, int((ma | mb).sum()))
        return ang, iou

    curve = [metrics(x)]
    for _ in range(iters):
        x, _ = SF.sfseg_iterate(s, f, kern, alpha, iters=1, x0=x, x=x)
        curve.append(metrics(x))
    ang_conv, iou_conv = metrics(xt)
    # time per iteration of the three operators (HIP events on the current stream)
    import paper_2212_08058_amd as P
    z = torch.empty_like(s)

    def per_iter(fn, reps=20):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        return e0.elapsed_time(e1) / reps
    ms_exp = per_iter(lambda: SF.exp_step(s, f, x, kern, alpha, z=z))
    ms_tay = per_iter(lambda: SF.sfseg_step(s, f, x, kern, alpha, z=z))
    ms_plain = per_iter(lambda: P.step(s, x, kern, z=z))
    log(f"  taylor study {shape}: start {curve[0][0]:.1f} deg -> {curve[-1][0]:.2f} deg after {iters} "
        f"iterations (IoU {curve[-1][1]:.3f}); converged Taylor vs exact {ang_conv:.3f} deg, IoU {iou_conv:.3f}")
    return dict(shape=list(shape), alpha=alpha, seed=seed, kernel=dict(sigma_s=sigma_s, sigma_t=sigma_t, r_s=r_s,
                                                                        r_t=r_t),
                exact_iters=rv["iters"], taylor_iters=rt["iters"],
                angle_deg=[round(a, 4) for a, _ in curve], iou=[round(b, 4) for _, b in curve],
                converged_angle_deg=ang_conv, converged_iou=iou_conv,
                ms_per_iter=dict(exact_gather=ms_exp, taylor_three_fields=ms_tay, single_field=ms_plain))


def pp_training_step(n_iter=15, n_cont=10, kappa=2.0, theta=1.0, reps=5, device="cuda", log=print):
    """The paper's objective on the channel workload (C = 8, 32x240x432, K as
    the channel workload): sigmoid-affine combination (Eq. 9), n_iter
    iterations of which the last n_iter - n_cont are soft-binarised (Alg. 1),
    Focal-Dice (Eq. 12, gamma 0.75), backward and one AdamW step."""
    c = synth.CONFIGS["channels"]
    kern = Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    fc, gt = synth.channel_stack(c["C"], c["T"], c["H"], c["W"], seed=c["seed"])
    fcd = torch.from_numpy(fc).to(device)
    gtd = torch.from_numpy(gt).to(device)
    w = torch.zeros(c["C"], dtype=torch.float64, device=device, requires_grad=True)
    b = torch.zeros((), dtype=torch.float64, device=device, requires_grad=True)
    opt = learn.AdamW([w, b.reshape(1)], lr=0.05, weight_decay=0.0)

    def step():
        w.grad = None
        b.grad = None
        J = learn.focal_dice(learn.sfseg_pp(fcd, w, b, kern, n_iter, n_cont, kappa, theta), gtd)
        J.backward()
        opt.step([w.grad, b.grad.reshape(1)])
        return J

    step()
    _sync()
    ts, losses = [], []
    for _ in range(reps):
        _sync()
        t0 = time.perf_counter()
        J = step()
        _sync()
        ts.append(time.perf_counter() - t0)
        losses.append(float(J))
    N = c["T"] * c["H"] * c["W"]
    t = float(np.median(ts))
    return dict(seconds_per_step=t, losses=losses, n_iter=n_iter, n_cont=n_cont, kappa=kappa, theta=theta,
                weights=w.detach().cpu().tolist(), bias=float(b), voxels=N, step_voxel_iters_per_s=2 * N * n_iter / t)
