#!/usr/bin/env python3
"""Benchmark: voxel-iterations/s of the space-time power iteration on one MI355X.

Workload: one synthetic full-resolution clip, 64 x 480 x 854 (the paper's
DAVIS frame size), 5 moving Gaussian blobs plus U[0, 0.1] noise, filter
sigma_s = 5, sigma_t = 2, r_s = 15, r_t = 5. One benchmark step is one
complete stpi_iterate call: uniform start, 20 (step, finalise) pairs on the
device, final normalisation, one host synchronisation.

value = 64*480*854 * 20 / (seconds per step), inputs resident in HBM.
roofline: the fused step kernel alone, timed with HIP events on the stream it
runs on. With the matrix-core tile loop (both spatial passes on MFMA) the step
is bound by memory traffic: achieved = algorithmic bytes (read f and x, write
z) over the kernel time, against 8 TB/s. With a vector-ALU tile loop its bound
is the non-packed FP32 FMA rate (78.6 TFLOP/s on 256 CUs at 2.4 GHz). The other
figure is reported beside the bound in either case.
cpu_baseline: the FP64 oracle on a bounded sample of the same voxels.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12   # 78.6: FMA lanes x 2 flop x clock


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# Sources that define the f32 step kernel; the committed counter summary is
# used only while their hash matches the one recorded with the counters.
STEP_SOURCES = ["paper_2212_08058_amd/csrc/common.hpp", "paper_2212_08058_amd/csrc/stencil.hpp",
                "paper_2212_08058_amd/csrc/stencil_mfma.hpp", "paper_2212_08058_amd/csrc/forward.hpp",
                "paper_2212_08058_amd/csrc/kernels_f32.hip", "paper_2212_08058_amd/csrc/host.cpp"]
LOOP_KIND = {0: "plain", 1: "pipelined", 2: "straight-line", 3: "matrix-core"}


def profiled_traffic(tag: str):
    """HBM bytes per launch from profiles/<tag>_hbm_counters.md (rocprofv3
    FETCH_SIZE and WRITE_SIZE, calibrated on a streaming kernel of known
    size), or None if the kernel sources changed since they were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"{tag}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    text = open(path).read()
    rec = json.loads(text.split("```json")[1].split("```")[0])
    h = hashlib.sha256()
    for p in STEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != rec["source_sha"]:
        return None
    return rec


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(f_np, kern, seconds: float):
    import numpy as np

    import oracle

    oracle.build(force=False)
    k = oracle.Kernel(kern.sigma_s, kern.sigma_t, kern.r_s, kern.r_t)
    x = np.full(f_np.shape, 1.0 / math.sqrt(f_np.size))
    f64 = f_np.astype(np.float64)
    rng = np.random.default_rng(0)

    def timed(n_threads, secs):
        oracle.set_threads(n_threads)
        # a short probe sizes the timed sample to about `secs` of CPU work
        idx = rng.integers(0, f_np.size, 200 * n_threads)
        t0 = time.perf_counter()
        oracle.apply_at(f64, x, k, idx)
        rate = idx.size / max(time.perf_counter() - t0, 1e-6)
        n = int(min(max(rate * secs, 200), 50_000_000))
        idx = rng.integers(0, f_np.size, n)
        t0 = time.perf_counter()
        oracle.apply_at(f64, x, k, idx)
        return n, time.perf_counter() - t0

    threads = oracle.num_threads()
    n1, dt1 = timed(1, min(5.0, seconds / 3))
    n, dt = timed(threads, seconds)
    return dict(value=n / dt, unit="voxel-iters/s", cores=threads, kind="oracle",
                cpu_model=_cpu_model(), nproc=os.cpu_count(), value_1_thread=n1 / dt1,
                sample=f"{n} voxels drawn uniformly from the 64x480x854 clip, one application each "
                       f"(direct FP64 neighbourhood loop, {(2 * k.r_t + 1) * (2 * k.r_s + 1) ** 2} taps/voxel), "
                       f"{dt:.1f} s on {threads} threads; {n1} voxels in {dt1:.1f} s on 1 thread")


def sfseg_leg(f_np, kern, iters, steps, warmup, reps, stream, dev):
    """The full operator of Eq. 7 (three filtered fields) on the same clip: s =
    the soft mask to the power p = 0.2, f = a second soft mask in [0, 1]
    (standing in for the optical-flow magnitude), alpha = 1. Whole 20-iteration
    jobs from the uniform start, and the step kernel timed with HIP events on
    its stream (each timed call also launches the two-sum reduction kernel)."""
    import numpy as np
    import torch

    import synth
    from paper_2212_08058_amd import sfseg as SF

    T, H, W = f_np.shape
    g, _ = synth.blob_clip(T, H, W, 3, 1001)
    with torch.cuda.stream(stream):
        s = SF.sfseg_unary(torch.from_numpy(f_np).to(dev), 0.2, stream=stream)
        fd = torch.from_numpy(g).to(dev)
        x = torch.empty_like(s)
        ws = torch.empty(SF.sfseg_workspace_bytes(s.shape, kern), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    for _ in range(warmup):
        SF.sfseg_iterate(s, fd, kern, 1.0, iters=iters, x=x, ws=ws, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        _, r = SF.sfseg_iterate(s, fd, kern, 1.0, iters=iters, x=x, ws=ws, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    N = s.numel()
    z = torch.empty_like(s)
    SF.sfseg_step(s, fd, x, kern, 1.0, z=z, ws=ws, stream=stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        SF.sfseg_step(s, fd, x, kern, 1.0, z=z, ws=ws, stream=stream)
    e1.record(stream)
    e1.synchronize()
    kms = e0.elapsed_time(e1) / reps
    # per voxel: 3 fields x (y, x and t taps) multiply-adds + staging and recombination
    flop = 2 * 3 * (2 * (2 * kern.r_s + 1) + (2 * kern.r_t + 1)) + 12
    return {"value": N * iters / dt, "unit": "voxel-iters/s", "ms_per_step": dt * 1e3, "iters": iters,
            "alpha": 1.0, "p": 0.2, "lambda": r["lambda_"], "residual": r["residual"],
            "roofline": {"bound": "alu", "achieved": flop * N / (kms * 1e-3) / 1e12, "peak": VALU_FP32_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": flop * N / (kms * 1e-3) / 1e12 / VALU_FP32_PEAK_TFLOPS,
                         "flop_per_voxel": flop, "kernel": "sfseg_step_kernel", "kernel_ms": kms,
                         "hbm_gbs": 16 * N / (kms * 1e-3) / 1e9, "bytes_per_voxel": 16}}


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dtype", choices=["f32", "bf16"], default="f32")
    ap.add_argument("--kernel-reps", type=int, default=40, help="launches timed for the roofline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="let the autotuner pick the FP32 tile (default: the cost model's choice, which the "
                         "committed counter profile covers); the BF16 leg is always tuned")
    ap.add_argument("--extras", default="bf16,copy,sfseg,taylor,online,objective,channels,batch,warm",
                    help="comma list of extra measurements to attach: bf16, copy, sfseg, taylor, online, objective, "
                         "batch, channels, warm (or none)")
    ap.add_argument("--warm-train", type=int, default=200, help="training clips for the warm-start extra")
    ap.add_argument("--warm-eval", type=int, default=24, help="evaluation clips for the warm-start extra")
    ap.add_argument("--warm-epochs", type=int, default=2, help="training epochs for the warm-start extra")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(clips would shard across GPUs without per-iteration communication). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_2212_08058_amd as P

    c = synth.CONFIGS["full"]
    T, H, W, iters = c["T"], c["H"], c["W"], c["iters"]
    Nvox = T * H * W
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    dtype = torch.float32 if args.dtype == "f32" else torch.bfloat16
    elem = 4 if args.dtype == "f32" else 2
    log(f"generating {T}x{H}x{W} clip")
    f_np, _ = synth.blob_clip(T, H, W, c["nblobs"], c["seed"])
    dev = torch.device("cuda:0")
    stream = torch.cuda.Stream(device=dev)
    with torch.cuda.stream(stream):
        f = torch.from_numpy(f_np).to(dev).to(dtype)
        x = torch.empty_like(f)
        ws = torch.empty(P.workspace_bytes(f.shape, kern, dtype), dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()

    # the project's autotuner picks the tile variant for this problem (timed
    # with HIP events on the step kernel; outside the timed region)
    from paper_2212_08058_amd import batch as PB
    from paper_2212_08058_amd import _native as PN
    import ctypes as _ct
    if args.autotune or args.dtype == "bf16":
        tuned_idx, tuned_ms = PB.autotune(f.shape, kern, dtype, reps=10)
        log(f"autotuned variant {tuned_idx}: {tuned_ms * 1e3:.1f} us")
    vinfo = (_ct.c_int * 9)()
    PN.lib.stpi_variant_info(0 if args.dtype == "f32" else 1, P.launch_shape(f.shape, kern, dtype)["variant"], vinfo)

    def one_step():
        return P.power_iterate(f, kern, iters=iters, x=x, ws=ws, stream=stream)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        _, res = one_step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, res = one_step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / args.steps
    value = Nvox * iters / (dt / args.steps)

    # dominant kernel alone, HIP events on its own stream
    log("timing the step kernel")
    xs = torch.empty_like(f)
    kern_ms, product = P.time_chain_step(f, kern, x=xs, reps=args.kernel_reps, ws=ws, stream=stream)
    bytes_per_voxel = 3 * elem
    flops_per_voxel = 2 * (2 * (2 * kern.r_s + 1) + (2 * kern.r_t + 1)) + 6
    hbm_gbs = bytes_per_voxel * Nvox / (kern_ms * 1e-3) / 1e9
    tflops = flops_per_voxel * Nvox / (kern_ms * 1e-3) / 1e12

    out = {
        "metric": "voxel-iters/s @64x480x854 (%HBM roofline); wall-time to 1e-4, warm vs plain",
        "value": value,
        "unit": "voxel-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {
            "workload": f"single clip {T}x{H}x{W}, {c['nblobs']} moving Gaussian blobs + U[0,0.1] noise (seed "
                        f"{c['seed']}), sigma_s={c['sigma_s']} sigma_t={c['sigma_t']} r_s={c['r_s']} r_t={c['r_t']}, "
                        f"{iters} iterations from the uniform start, {args.dtype} storage",
            "voxels": Nvox,
            "iters": iters,
            "parallelism": "single GPU",
            "tile": dict(zip(("r_s", "r_t", "TH", "TW", "threads", "RY", "QX", "min_waves"), list(vinfo)[:8]),
                         loop=LOOP_KIND.get(vinfo[8], str(vinfo[8])),
                         chain_form="product" if product else "plain",
                         segments=P.launch_shape(f.shape, kern, dtype)["segments"]),
        },
        "roofline": {},
        "result": {"residual": res["residual"], "lambda": res["lambda_"], "iters": res["iters"]},
    }
    alu = {"achieved": tflops, "peak": VALU_FP32_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tflops / VALU_FP32_PEAK_TFLOPS,
           "flop_per_voxel": flops_per_voxel}
    hbm = {"achieved": hbm_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": hbm_gbs / HBM_PEAK_GBS,
           "bytes_per_voxel": bytes_per_voxel}
    if vinfo[8] == 3:
        # the roofline that bounds a stencil is HBM bandwidth; what limits this
        # kernel below it is recorded beside it (rocprofv3 SQ counters)
        out["roofline"] = {"bound": "hbm", **hbm, "traffic": None, "kernel": "fwd_step_kernel", "kernel_ms": kern_ms,
                           "alu": alu,
                           "limiter": "instruction issue and latency, not HBM: per SIMD the vector ALU is busy ~50% "
                                      "of the kernel time; a wavefront spends ~37% of its life in memory or barrier "
                                      "waits and ~24% waiting to issue (two wavefronts per SIMD, one LDS-bound "
                                      "workgroup per CU, a barrier per frame phase, 39 phases per workgroup; "
                                      "vector-memory latency ~1050 cycles, L2 hit rate ~59%)"}
    else:
        out["roofline"] = {"bound": "alu", **alu, "traffic": None, "kernel": "fwd_step_kernel", "kernel_ms": kern_ms,
                           "hbm": hbm}
    prof = profiled_traffic(f"fwd_step_{T}x{H}x{W}_{args.dtype}")
    ctype = "float" if args.dtype == "f32" else "stpi::bf16"
    sig = f"fwd_step_kernel<{ctype}, " + ", ".join(str(v) for v in vinfo) + (", true>" if product else ", false>")
    if prof is not None and sig not in prof["kernel"]:
        prof = None  # the counters were taken on another tile variant
    if prof is not None:
        out["roofline"]["traffic"] = prof["traffic_bytes"]
        out["roofline"]["traffic_note"] = (f"HBM bytes per launch from rocprofv3 FETCH_SIZE x {prof['fetch_scale']:.3f} + "
                                           f"WRITE_SIZE x {prof['write_scale']:.3f} (calibrated on a streaming kernel); "
                                           f"{prof['traffic_bytes'] / (bytes_per_voxel * Nvox):.2f}x the algorithmic "
                                           f"{bytes_per_voxel * Nvox} B")
    extras = [e for e in args.extras.split(",") if e and e != "none"]
    if "bf16" in extras and args.dtype == "f32":
        log("bf16 storage leg")
        with torch.cuda.stream(stream):
            fb = f.to(torch.bfloat16)
            xb = torch.empty_like(fb)
            wsb = torch.empty(P.workspace_bytes(fb.shape, kern, torch.bfloat16), dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        PB.autotune(fb.shape, kern, torch.bfloat16, reps=10)
        for _ in range(args.warmup):
            P.power_iterate(fb, kern, iters=iters, x=xb, ws=wsb, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            P.power_iterate(fb, kern, iters=iters, x=xb, ws=wsb, stream=stream)
        torch.cuda.synchronize()
        dtb = (time.perf_counter() - t0) / args.steps
        kb, pfb = P.time_chain_step(fb, kern, x=torch.empty_like(fb), reps=args.kernel_reps, ws=wsb, stream=stream)
        out["bf16"] = {"value": Nvox * iters / dtb, "ms_per_step": dtb * 1e3, "kernel_ms": kb,
                       "chain_form": "product" if pfb else "plain",
                       "hbm_gbs": 6 * Nvox / (kb * 1e-3) / 1e9,
                       "alu_tflops": flops_per_voxel * Nvox / (kb * 1e-3) / 1e12}
    if "copy" in extras:
        # A plain streaming kernel of known traffic (x = z / 1: reads and writes
        # one array of the clip's size), timed like the step kernel. Its HBM
        # counters calibrate the step kernel's measured traffic.
        from paper_2212_08058_amd import _native as N
        one = torch.ones(1, dtype=torch.float64, device=dev)
        dst = torch.empty_like(f)
        code = 0 if args.dtype == "f32" else 1
        sp = stream.cuda_stream

        def launch():
            N.check(N.lib.stpi_normalize(Nvox, code, f.data_ptr(), one.data_ptr(), dst.data_ptr(), sp))

        for _ in range(3):
            launch()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.kernel_reps):
            launch()
        e1.record(stream)
        e1.synchronize()
        cms = e0.elapsed_time(e1) / args.kernel_reps
        out["copy"] = {"kernel": "scale_by_norm_kernel (reads one array, writes one array)",
                       "bytes_read": Nvox * elem, "bytes_written": Nvox * elem, "kernel_ms": cms,
                       "gbs": 2 * Nvox * elem / (cms * 1e-3) / 1e9}
    if "sfseg" in extras and args.dtype == "f32":
        log("full SFSeg operator (alpha = 1, p = 0.2)")
        out["sfseg"] = sfseg_leg(f_np, kern, iters, args.steps, args.warmup, args.kernel_reps, stream, dev)
    from paper_2212_08058_amd import experiments as X
    if "taylor" in extras and args.dtype == "f32":
        log("exact (Eq. 1) vs Taylor (Eq. 2) affinity study")
        out["taylor"] = [X.taylor_study(shape=(10, 20, 20), log=log), X.taylor_study(shape=(16, 64, 112), log=log)]
    if "online" in extras and args.dtype == "f32":
        log("online sub-windows vs the full video")
        out["online"] = X.online_vs_full(f_np, kern, log=log)
    if "batch" in extras:
        log("batched uneven clips")
        out["batch"] = X.batched_workload(log=log)
    if "channels" in extras:
        log("channel-combination training step")
        out["channels"] = X.channel_training_step(log=log)
    if "objective" in extras:
        log("the paper's objective: sigmoid-affine combination, soft-binarisation, Focal-Dice")
        out["objective"] = X.pp_training_step(log=log)
    if "warm" in extras:
        log("warm start vs plain")
        r = X.warm_start_experiment(n_train=args.warm_train, n_eval=args.warm_eval, epochs=args.warm_epochs, log=log)
        r.pop("iters", None)
        r.pop("ms", None)
        out["warm"] = r
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on a sample")
        out["cpu_baseline"] = cpu_baseline(f_np, kern, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
