"""GPU parity of the fused step and the power iteration against the FP64 oracle.

Bars: FP32 per step relative L2 <= 1e-5; FP64 <= 1e-12; BF16 storage
<= 2^-8 against the oracle on the bf16-rounded inputs; converged vectors
within 1e-3 cosine distance. Every comparison also prints the FP64 error.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import Kernel as OK

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def P():
    import paper_2212_08058_amd as P
    return P


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)


def bf16_np(a):
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


TOL = {torch.float32: 1e-5, torch.float64: 1e-12, torch.bfloat16: 2.0 ** -8}


def OKf(ss, st, rs, rt):
    """Oracle kernel with the sigmas rounded to float, as the C ABI carries them."""
    return OK(float(np.float32(ss)), float(np.float32(st)), rs, rt)


def _step_case(P, shape, kern, dtype, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    if dtype == torch.bfloat16:
        f64, x64 = bf16_np(f), bf16_np(x)
    else:
        f64, x64 = f.astype(np.float64), x.astype(np.float64)
    scale = 0.7
    ref = oracle.apply(f64, x64 * scale, OKf(kern.sigma_s, kern.sigma_t, kern.r_s, kern.r_t))
    fd, xd = to_dev(f64, dtype), to_dev(x64, dtype)
    z, sums = P.step(fd, xd, kern, x_scale=scale)
    torch.cuda.synchronize()
    zz = z.double().cpu().numpy()
    err = rel_l2(zz, ref)
    s = sums.cpu().numpy()
    zs = zz  # sums are over the stored values
    print(f"step {shape} r=({kern.r_s},{kern.r_t}) {dtype}: rel L2 {err:.3e}")
    assert err <= TOL[dtype], err
    # block sums of exact double products: only the summation order differs
    assert abs(s[0] - np.sum(zs * zs)) <= 1e-12 * np.sum(zs * zs) + 1e-300
    assert abs(s[1] - scale * np.sum(zs * x64)) <= 1e-12 * abs(scale * np.sum(zs * x64)) + 1e-300
    return err


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64, torch.bfloat16])
def test_step_small_workload(P, dtype):
    c = synth.CONFIGS["small"]
    _step_case(P, (c["T"], c["H"], c["W"]), P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"]), dtype, 0)


@pytest.mark.parametrize("shape,kern", [
    ((5, 37, 70), (2.0, 1.0, 4, 2)),      # ragged in H and W, several tiles
    ((13, 40, 131), (4.0, 1.5, 8, 3)),
    ((12, 35, 150), (5.0, 2.0, 15, 5)),
    ((3, 17, 19), (1.3, 0.7, 1, 1)),
    ((4, 20, 23), (3.0, 2.0, 6, 4)),      # radii that use a larger compiled bucket
    ((2, 9, 11), (2.0, 1.0, 16, 8)),      # radius beyond the volume
    ((1, 1, 1), (1.0, 1.0, 2, 1)),        # single voxel
    ((1, 30, 1), (2.0, 1.0, 4, 2)),       # single column
    ((9, 1, 40), (2.0, 1.0, 4, 2)),       # single row
    ((3, 18, 20), (2.0, 1.0, 0, 0)),      # no neighbours: A = diag(f^2)
])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_step_shapes_and_radii(P, shape, kern, dtype):
    _step_case(P, shape, P.Kernel(*kern), dtype, 1)


def test_every_compiled_variant(P):
    """Each compiled (radii, tile) variant matches the oracle on a ragged multi-tile volume."""
    from paper_2212_08058_amd import _native as N
    import ctypes
    n = N.lib.stpi_variant_count(N.STPI_F32)
    assert n >= 1
    rng = np.random.default_rng(3)
    shape = (11, 45, 150)
    f = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    fd, xd = to_dev(f, torch.float32), to_dev(x, torch.float32)
    try:
        for i in range(n):
            info = (ctypes.c_int * 9)()
            assert N.lib.stpi_variant_info(N.STPI_F32, i, info) == 0
            RS, RT = info[0], info[1]
            kern = P.Kernel(0.6 * RS + 0.5, 0.6 * RT + 0.5, RS, RT)
            ref = oracle.apply(f, x, OKf(kern.sigma_s, kern.sigma_t, RS, RT))
            assert N.lib.stpi_set_variant(i) == 0
            z, _ = P.step(fd, xd, kern)
            torch.cuda.synchronize()
            err = rel_l2(z.double().cpu().numpy(), ref)
            print("variant", i, list(info), err)
            assert err <= 1e-5
    finally:
        N.lib.stpi_set_variant(-1)


def test_iterate_small_workload_matches_oracle(P):
    c = synth.CONFIGS["small"]
    f, _ = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], c["seed"])
    k = OKf(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    xs_ref = oracle.iterate(f, k, iters=c["iters"], keep=True)
    x_ref, info = xs_ref[0], xs_ref[1]
    traj = xs_ref[2]
    fd = to_dev(f, torch.float32)
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    # per-step parity along the oracle's own trajectory
    for j in range(c["iters"]):
        z, _ = P.step(fd, to_dev(traj[j].astype(np.float32), torch.float32), kern)
        ref = oracle.apply(f, traj[j].astype(np.float32), k)
        err = rel_l2(z.double().cpu().numpy(), ref)
        assert err <= 1e-5, (j, err)
    x, res = P.power_iterate(fd, kern, iters=c["iters"])
    xg = x.double().cpu().numpy()
    err = rel_l2(xg, x_ref)
    cosd = 1.0 - float(np.sum(xg * x_ref)) / float(np.linalg.norm(xg))
    print(f"iterate small: rel L2 {err:.3e}, cos dist {cosd:.3e}, residual {res['residual']:.6e} vs "
          f"{info.residuals[-1]:.6e}, lambda {res['lambda_']:.9f} vs {info.lambdas[-1]:.9f}")
    assert res["iters"] == c["iters"] and not res["converged"]
    assert err <= 1e-5 and cosd <= 1e-9
    assert abs(res["lambda_"] - info.lambdas[-1]) <= 1e-5 * info.lambdas[-1]
    assert abs(res["rayleigh"] - info.rayleigh[-1]) <= 1e-5 * info.rayleigh[-1]
    assert abs(res["residual"] - info.residuals[-1]) <= 1e-3 * info.residuals[-1] + 1e-7
    assert abs(float(np.linalg.norm(xg)) - 1.0) < 1e-5


def test_iterate_tolerance_mode(P):
    c = synth.CONFIGS["small"]
    f, _ = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], seed=1)
    k = OKf(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    x_ref, info = oracle.iterate(f, k, tol=1e-4, cap=500)
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    for dtype in (torch.float32, torch.float64):
        x, res = P.power_iterate(to_dev(f, dtype), kern, tol=1e-4, max_iters=500)
        xg = x.double().cpu().numpy()
        cosd = 1.0 - float(np.sum(xg * x_ref))
        print(dtype, "tol mode iters", res["iters"], "oracle", info.iters, "cos dist", cosd)
        assert res["converged"] and info.converged
        assert abs(res["iters"] - info.iters) <= (0 if dtype == torch.float64 else 2)
        assert res["residual"] < 1e-4
        assert cosd <= 1e-3
    # the cap binds
    x, res = P.power_iterate(to_dev(f, torch.float32), kern, tol=1e-12, max_iters=7)
    assert res["iters"] == 7 and not res["converged"]


def test_iterate_bf16_storage(P):
    c = synth.CONFIGS["small"]
    f, _ = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], c["seed"])
    fb = bf16_np(f)
    k = OKf(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    x_ref, info = oracle.iterate(fb, k, tol=1e-4, cap=500)
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    x, res = P.power_iterate(to_dev(fb, torch.bfloat16), kern, iters=info.iters + 20)
    xg = x.double().cpu().numpy()
    cosd = 1.0 - float(np.sum(xg * x_ref)) / float(np.linalg.norm(xg))
    print("bf16 cos dist", cosd)
    assert cosd <= 1e-3


def test_start_vector_and_edge_cases(P):
    kern = P.Kernel(2.0, 1.0, 4, 2)
    k = OKf(2.0, 1.0, 4, 2)
    rng = np.random.default_rng(5)
    f = rng.uniform(0.1, 1, (4, 20, 30)).astype(np.float32)
    x0 = rng.uniform(0.1, 1, f.shape).astype(np.float32) * 37.0  # unnormalised start
    x_ref, info = oracle.iterate(f, k, x0=x0, iters=5)
    x, res = P.power_iterate(to_dev(f, torch.float32), kern, iters=5, x0=to_dev(x0, torch.float32))
    assert rel_l2(x.double().cpu().numpy(), x_ref) < 1e-5
    # zero iterations returns the normalised start
    x, res = P.power_iterate(to_dev(f, torch.float32), kern, iters=0, x0=to_dev(x0, torch.float32))
    assert res["iters"] == 0
    np.testing.assert_allclose(x.double().cpu().numpy(), x0 / np.linalg.norm(x0.astype(np.float64)), rtol=1e-6)
    # f = 0: A x = 0 is reported, x keeps the start
    from paper_2212_08058_amd import StpiError
    with pytest.raises(StpiError) as ei:
        P.power_iterate(torch.zeros((2, 8, 9), device=DEV), kern, iters=3)
    assert ei.value.status == 3
    # zero start vector
    with pytest.raises(StpiError):
        P.power_iterate(to_dev(f, torch.float32), kern, iters=3, x0=torch.zeros_like(to_dev(f, torch.float32)))
    # NaN in f
    fn = f.copy()
    fn[1, 2, 3] = np.nan
    with pytest.raises(StpiError) as ei:
        P.power_iterate(to_dev(fn, torch.float32), kern, iters=3)
    assert ei.value.status == 4
    # radius 0: A = diag(f^2), the limit is the one-hot at the largest f
    g = np.full((3, 5, 6), 0.5, dtype=np.float32)
    g[1, 2, 3] = 0.9
    x, res = P.power_iterate(to_dev(g, torch.float32), P.Kernel(1.0, 1.0, 0, 0), tol=1e-6, max_iters=200)
    xg = x.cpu().numpy()
    assert xg[1, 2, 3] > 0.999 and res["converged"]
    assert abs(res["lambda_"] - 0.81) < 1e-4


def test_deterministic(P):
    c = synth.CONFIGS["small"]
    f, _ = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], 2)
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    fd = to_dev(f, torch.float32)
    x1, r1 = P.power_iterate(fd, kern, iters=12)
    x1 = x1.clone()
    x2, r2 = P.power_iterate(fd, kern, iters=12)
    assert torch.equal(x1, x2) and r1 == r2


def _kron_reference(a, b, c, kern, iters):
    """Full-size exact reference for separable f = a (x) b (x) c: the iterate stays
    separable, so three 1D oracle iterations (one per axis) give it."""
    xt, it = oracle.iterate(a.reshape(-1, 1, 1), OKf(kern.sigma_s, kern.sigma_t, kern.r_s, kern.r_t), iters=iters)
    xy, iy = oracle.iterate(b.reshape(1, -1, 1), OKf(kern.sigma_s, kern.sigma_t, kern.r_s, kern.r_t), iters=iters)
    xx, ix = oracle.iterate(c.reshape(1, 1, -1), OKf(kern.sigma_s, kern.sigma_t, kern.r_s, kern.r_t), iters=iters)
    lam = it.lambdas[-1] * iy.lambdas[-1] * ix.lambdas[-1]
    return xt.reshape(-1), xy.reshape(-1), xx.reshape(-1), lam


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_full_size_kronecker(P, dtype):
    """64 x 480 x 854, r_s = 15, r_t = 5, 20 iterations: exact separable reference."""
    c = synth.CONFIGS["full"]
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    rng = np.random.default_rng(11)
    a = rng.uniform(0.3, 1.0, c["T"])
    b = rng.uniform(0.3, 1.0, c["H"])
    cc = rng.uniform(0.3, 1.0, c["W"])
    f = np.einsum("i,j,l->ijl", a, b, cc)
    # storing f rounds it (f32: ~6e-8, bf16: ~2e-3 relative), which breaks exact
    # separability by that much; the bars below allow for it
    x, res = P.power_iterate(to_dev(f, dtype), kern, iters=c["iters"])
    torch.cuda.synchronize()
    xt, xy, xx, lam = _kron_reference(a, b, cc, kern, c["iters"])
    xr = torch.from_numpy(np.einsum("i,j,l->ijl", xt, xy, xx)).to(DEV)
    xg = x.double()
    err = float(torch.linalg.vector_norm(xg - xr) / torch.linalg.vector_norm(xr))
    cosd = 1.0 - float(torch.sum(xg * xr) / torch.linalg.vector_norm(xg))
    print(f"full-size kronecker {dtype}: rel L2 {err:.3e} cos dist {cosd:.3e} lambda {res['lambda_']} vs {lam}")
    if dtype == torch.float32:
        assert err < 1e-4
        assert abs(res["lambda_"] - lam) / lam < 1e-5
    else:
        assert cosd < 1e-3
        assert abs(res["lambda_"] - lam) / lam < 1e-2


def test_full_size_sampled_step(P):
    """Full workload shape, one step in the benchmark's launch configuration, checked on
    sampled voxels (corners, faces, interior) against the oracle voxel by voxel."""
    c = synth.CONFIGS["full"]
    f, _ = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], c["seed"])
    rng = np.random.default_rng(12)
    x = rng.uniform(0.0, 1.0, f.shape).astype(np.float32)
    kern = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    k = OKf(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    T, H, W = f.shape
    pts = [(t, y, xx) for t in (0, 1, 5, T // 2, T - 6, T - 1) for y in (0, 3, 15, H // 2, H - 16, H - 1)
           for xx in (0, 14, 15, 127, 128, W // 2, W - 16, W - 1)]
    idx = np.array([(t * H + y) * W + xx for t, y, xx in pts] + list(rng.integers(0, f.size, 1500)), dtype=np.int64)
    ref = oracle.apply_at(f, x, k, idx)
    for dtype in (torch.float32, torch.bfloat16):
        if dtype == torch.bfloat16:
            fr, xr = bf16_np(f), bf16_np(x)
            ref = oracle.apply_at(fr, xr, k, idx)
        else:
            fr, xr = f, x
        z, sums = P.step(to_dev(fr, dtype), to_dev(xr, dtype), kern)
        torch.cuda.synchronize()
        zs = z.double().reshape(-1)[torch.from_numpy(idx).to(DEV)].cpu().numpy()
        err = rel_l2(zs, ref)
        print("full-size sampled step", dtype, err)
        assert err <= TOL[dtype]


def test_frame_segments_match_oracle(P):
    """Every variant at the full 64 x 480 x 854 shape (r = (15, 5) and (8, 3)),
    in whatever frame-segment split it launches with; sampled voxels include
    every frame within r_t + 1 of each segment boundary."""
    from paper_2212_08058_amd import _native as N
    import ctypes
    c = synth.CONFIGS["full"]
    f, _ = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], c["seed"])
    rng = np.random.default_rng(21)
    x = rng.uniform(0.0, 1.0, f.shape).astype(np.float32)
    T, H, W = f.shape
    fd, xd = to_dev(f, torch.float32), to_dev(x, torch.float32)
    seen_split = False
    try:
        for kern in (P.Kernel(5.0, 2.0, 15, 5), P.Kernel(4.0, 1.5, 8, 3)):
            k = OKf(kern.sigma_s, kern.sigma_t, kern.r_s, kern.r_t)
            for i in range(N.lib.stpi_variant_count(N.STPI_F32)):
                info = (ctypes.c_int * 9)()
                N.lib.stpi_variant_info(N.STPI_F32, i, info)
                if info[0] < kern.r_s or info[1] < kern.r_t or info[0] > kern.r_s + 1:
                    continue
                shape = P.launch_shape(f.shape, kern, variant=i)
                nseg = shape["segments"]
                seen_split |= nseg > 1
                bounds = sorted({s * T // nseg for s in range(1, nseg)})
                frames = sorted({t for b in bounds for t in range(b - kern.r_t - 1, b + kern.r_t + 1)} | {0, T - 1})
                pts = [(t, y, xx) for t in frames for y in (0, 7, H // 2, H - 1) for xx in (0, 100, W // 2, W - 1)]
                idx = np.array([(t * H + y) * W + xx for t, y, xx in pts] + list(rng.integers(0, f.size, 300)),
                               dtype=np.int64)
                ref = oracle.apply_at(f, x, k, idx)
                assert N.lib.stpi_set_variant(i) == 0
                z, _ = P.step(fd, xd, kern)
                torch.cuda.synchronize()
                zs = z.double().reshape(-1)[torch.from_numpy(idx).to(DEV)].cpu().numpy()
                err = rel_l2(zs, ref)
                print("variant", i, list(info), shape, err)
                assert err <= 1e-5
    finally:
        N.lib.stpi_set_variant(-1)
    assert seen_split, "no compiled variant split the frames at this shape"


def test_long_tolerance_runs_stop_in_chunks(P):
    """A tolerance run with a large cap replays short chain segments and stops
    once converged: it must end exactly where a fixed-count run of the same
    number of steps ends (bitwise), on the captured-graph and the direct path,
    and the same holds for the batched chain."""
    from paper_2212_08058_amd import batch as B
    f, _ = synth.blob_clip(12, 60, 100, 3, 7)
    kern = P.Kernel(4.0, 1.5, 8, 3)
    fd = to_dev(f, torch.float32)
    s = torch.cuda.Stream()
    for stream in (s, None):
        x_tol, r_tol = P.power_iterate(fd, kern, tol=1e-6, max_iters=5000, stream=stream)
        torch.cuda.synchronize()
        assert r_tol["converged"] and 48 < r_tol["iters"] < 5000, r_tol  # several 16-step segments
        x_fix, r_fix = P.power_iterate(fd, kern, iters=r_tol["iters"], stream=stream)
        torch.cuda.synchronize()
        assert torch.equal(x_tol, x_fix) and r_tol["residual"] == r_fix["residual"]
    shapes = [(12, 60, 100), (9, 40, 70)]
    fs = [f, synth.blob_clip(9, 40, 70, 2, 8)[0]]
    plan = B.BatchPlan(shapes, kern)
    f_flat = plan.pack([to_dev(v, torch.float32) for v in fs])
    x_flat, res = plan.iterate(f_flat, max_iters=5000, tol=1e-4, stream=s)
    torch.cuda.synchronize()
    for v, xv, r in zip(fs, plan.views(x_flat), res):
        assert r["converged"] and r["iters"] < 5000
        xs, rs = P.power_iterate(to_dev(v, torch.float32), kern, tol=1e-4, max_iters=5000)
        cosd = 1.0 - float(torch.sum(xs.double() * xv.double()))
        assert abs(r["iters"] - rs["iters"]) <= 1 and cosd < 1e-6


def test_fused_finalisation_is_bitwise_equal(P, monkeypatch):
    """The last workgroup's in-kernel step finalisation sums the partials in
    the separate finalisation kernel's order: every variant gives bitwise the
    same iterate and results either way (direct launches, so nothing cached)."""
    from paper_2212_08058_amd import _native as N
    import ctypes
    f, _ = synth.blob_clip(20, 64, 240, 3, 9)
    fd = to_dev(f, torch.float32)
    try:
        for i in range(N.lib.stpi_variant_count(N.STPI_F32)):
            info = (ctypes.c_int * 9)()
            N.lib.stpi_variant_info(N.STPI_F32, i, info)
            kern = P.Kernel(0.5 * info[0] + 0.5, 0.5 * info[1] + 0.5, info[0], info[1])
            assert N.lib.stpi_set_variant(i) == 0
            out = []
            for flag in ("0", "1"):
                monkeypatch.setenv("STPI_NO_FUSE", flag)
                x, r = P.power_iterate(fd, kern, iters=7)
                torch.cuda.synchronize()
                out.append((x, r))
            (xa, ra), (xb, rb) = out
            assert torch.equal(xa, xb), list(info)
            assert ra == rb, (list(info), ra, rb)
    finally:
        N.lib.stpi_set_variant(-1)


def test_enqueued_chains_survive_graph_eviction(P):
    """Chains enqueued without waiting stay queued behind a busy stream while
    later calls capture more graphs than the cache holds; evicting a queued
    graph must wait for it. Each result equals the direct (graph-free) run."""
    f, _ = synth.blob_clip(6, 40, 72, 2, 8)
    fd = torch.from_numpy(f).to(DEV)
    kern = P.Kernel(2.0, 1.0, 4, 2)
    s = torch.cuda.Stream()
    ws = torch.empty(P.workspace_bytes(fd.shape, kern), dtype=torch.uint8, device=DEV)
    xs = [torch.empty_like(fd) for _ in range(20)]
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        torch.cuda._sleep(100_000_000)  # keeps the chains below queued while they are captured
    for i, xv in enumerate(xs):
        P.power_iterate(fd, kern, iters=3 + i, x=xv, ws=ws, stream=s, wait=False)
    torch.cuda.synchronize()
    for i, xv in enumerate(xs):
        ref, r = P.power_iterate(fd, kern, iters=3 + i)
        torch.cuda.synchronize()
        assert r["iters"] == 3 + i and torch.equal(ref, xv), i


def test_first_residuals_and_rise_check(P):
    """The result carries the residuals of the first two applications (as the
    oracle's trajectory gives them); with the rise check a start near the
    second eigenvector (its residual grows as the principal component takes
    over) stops after two applications with flag bit 2, and a start near the
    principal eigenvector runs on."""
    shape = (2, 8, 10)
    rng = np.random.default_rng(4)
    f = rng.uniform(0.2, 1.0, shape)
    k = P.Kernel(2.0, 1.0, 3, 1)
    ok = OKf(k.sigma_s, k.sigma_t, k.r_s, k.r_t)
    A = oracle.dense_matrix(f.astype(np.float32).astype(np.float64), ok)
    w, V = np.linalg.eigh(A)
    v1, v2 = V[:, -1], V[:, -2]
    fd = to_dev(f, torch.float32)
    x0_rise = (v2 + 0.05 * v1).reshape(shape)  # residuals 0.0154, 0.0202, ... (eigenvalue ratio 1.31)
    _, info = oracle.iterate(f.astype(np.float32), ok, x0=x0_rise, iters=2)
    assert info.residuals[1] > info.residuals[0]
    x, r = P.power_iterate(fd, k, tol=1e-9, max_iters=50, x0=to_dev(x0_rise, torch.float32), rise_check=True)
    torch.cuda.synchronize()
    print("rise", r, info.residuals)
    assert r["iters"] == 2 and r["flags"] & 4 and not r["converged"]
    assert abs(r["r1"] - info.residuals[0]) <= 1e-4 * info.residuals[0] + 1e-6
    assert abs(r["r2"] - info.residuals[1]) <= 1e-4 * info.residuals[1] + 1e-6
    x0_good = (v1 + 1e-2 * v2).reshape(shape)
    x, r = P.power_iterate(fd, k, tol=1e-6, max_iters=200, x0=to_dev(x0_good, torch.float32), rise_check=True)
    torch.cuda.synchronize()
    assert not (r["flags"] & 4) and r["converged"] and r["iters"] > 2


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
@pytest.mark.parametrize("shape,kp", [((16, 128, 250), (5.0, 2.0, 15, 5)), ((9, 40, 70), (2.0, 1.0, 4, 2))])
def test_fixed_count_skips_no_reported_value(P, dtype, shape, kp):
    """A fixed-count chain forms the inner product with the previous iterate
    only on the steps whose residual it reports (the first two and the last);
    every reported value and the iterate must equal, bitwise, those of a run
    that forms it on every step (a tolerance run whose tolerance is never
    reached). Matrix-core product form (r = (15, 5)) and vector loop."""
    f, _ = synth.blob_clip(*shape, 3, 17)
    kern = P.Kernel(*kp)
    fd = to_dev(f, dtype)
    for iters in (3, 12):
        x_fix, r_fix = P.power_iterate(fd, kern, iters=iters)
        x_fix = x_fix.clone()
        x_all, r_all = P.power_iterate(fd, kern, tol=1e-300, max_iters=iters)
        torch.cuda.synchronize()
        print(shape, dtype, iters, r_fix["residual"], r_all["residual"], r_fix["rayleigh"])
        assert r_fix["iters"] == r_all["iters"] == iters and not r_all["converged"]
        assert torch.equal(x_fix, x_all)
        for key in ("residual", "lambda_", "rayleigh", "r1", "r2", "flags"):
            assert r_fix[key] == r_all[key], (key, r_fix[key], r_all[key])
