"""Batched uneven clips: parity with the FP64 oracle per clip, bitwise agreement
with the single-clip path, per-clip stopping, and the autotuner."""
import ctypes
import os

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
    from paper_2212_08058_amd import batch
    return P, batch


def okf(k):
    return OK(float(np.float32(k.sigma_s)), float(np.float32(k.sigma_t)), k.r_s, k.r_t)


SHAPES = [(9, 40, 70), (3, 17, 23), (1, 64, 80), (12, 31, 33), (5, 5, 5), (7, 70, 40)]


def _clips(shapes, seed=0):
    return [synth.blob_clip(T, H, W, 2, seed + i)[0] for i, (T, H, W) in enumerate(shapes)]


def test_batch_fixed_iterations_match_oracle(P):
    Pm, B = P
    kern = Pm.Kernel(2.0, 1.0, 4, 2)
    fs = _clips(SHAPES)
    plan = B.BatchPlan(SHAPES, kern)
    print(plan.info())
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    x_flat, res = plan.iterate(f_flat, max_iters=8, tol=0.0)
    for f, xv, r in zip(fs, plan.views(x_flat), res):
        xr, info = oracle.iterate(f, okf(kern), iters=8)
        err = float(np.linalg.norm(xv.double().cpu().numpy() - xr) / np.linalg.norm(xr))
        assert r["iters"] == 8 and err < 1e-5, (f.shape, err)
        assert abs(r["lambda_"] - info.lambdas[-1]) < 1e-5 * info.lambdas[-1]


def test_batch_bitwise_equals_single_clip_path(P):
    """Same kernel variant, same tiles, same reduction order: per-clip results are
    identical where the single-clip launch does not split the clip's frames,
    and agree to float rounding where it does (a split changes the order of
    the partial sums, and its backward-walked last segment the order of each
    output's temporal sum, so the iterates differ by float rounding)."""
    Pm, B = P
    from paper_2212_08058_amd import _native as N
    kern = Pm.Kernel(4.0, 1.5, 8, 3)
    # the 3-frame clip stays whole in a single-clip launch (splitting it would
    # save less than two phases), so it is compared bitwise
    shapes = [(11, 60, 216), (3, 45, 108), (20, 30, 150)]
    fs = _clips(shapes, seed=10)
    plan = B.BatchPlan(shapes, kern)
    info = plan.info()
    # force the single-clip path onto the same compiled variant
    nv = N.lib.stpi_variant_count(0)
    idx = None
    for i in range(nv):
        a = (ctypes.c_int * 9)()
        N.lib.stpi_variant_info(0, i, a)
        if a[8] == info["PIPE"] and [a[k] for k in range(7)] == [info[k] for k in
                                                              ("RS", "RT", "TH", "TW", "NTHR", "RY", "QX")]:
            idx = i
            break
    assert idx is not None
    s = torch.cuda.Stream()
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    torch.cuda.synchronize()
    x_flat, res = plan.iterate(f_flat, max_iters=60, tol=1e-4, stream=s)
    try:
        N.lib.stpi_set_variant(idx)
        split = 0
        for f, xv, r in zip(fs, plan.views(x_flat), res):
            xs, rs = Pm.power_iterate(torch.from_numpy(f).to(DEV), kern, tol=1e-4, max_iters=60)
            if Pm.launch_shape(f.shape, kern)["segments"] == 1:
                assert torch.equal(xs, xv), f.shape
                assert r["iters"] == rs["iters"] and r["converged"] == rs["converged"]
                assert r["residual"] == rs["residual"] and r["lambda_"] == rs["lambda_"]
            else:
                split += 1
                assert abs(r["iters"] - rs["iters"]) <= 1 and r["converged"] == rs["converged"]
                assert abs(r["lambda_"] - rs["lambda_"]) <= 1e-6 * rs["lambda_"]
                assert float((xs.double() - xv.double()).norm()) <= 1e-5
        assert split < len(fs), "no clip compared bitwise"
    finally:
        N.lib.stpi_set_variant(-1)


def test_batch_tolerance_per_clip_and_failures(P):
    Pm, B = P
    kern = Pm.Kernel(2.0, 1.0, 4, 2)
    shapes = [(6, 30, 40), (6, 30, 40), (4, 20, 20)]
    fs = _clips(shapes, seed=20)
    fs[2] = np.zeros_like(fs[2])  # A x = 0 for this clip only
    plan = B.BatchPlan(shapes, kern)
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    x_flat, res = plan.iterate(f_flat, max_iters=400, tol=1e-4, check=False)
    for f, xv, r in list(zip(fs, plan.views(x_flat), res))[:2]:
        xr, info = oracle.iterate(f, okf(kern), tol=1e-4, cap=400)
        assert r["converged"] and abs(r["iters"] - info.iters) <= 2
        cosd = 1 - float(np.sum(xv.double().cpu().numpy() * xr))
        assert cosd < 1e-3
    assert res[2]["status"] == 3 and not res[2]["converged"]
    # the capped case: every clip stops at the cap
    x_flat, res = plan.iterate(f_flat, max_iters=3, tol=1e-12, check=False)
    assert [r["iters"] for r in res[:2]] == [3, 3]


def test_batch_start_vectors(P):
    Pm, B = P
    kern = Pm.Kernel(2.0, 1.0, 4, 2)
    shapes = [(4, 20, 30), (3, 25, 21)]
    fs = _clips(shapes, seed=30)
    rng = np.random.default_rng(1)
    x0 = [rng.uniform(0.1, 1, s).astype(np.float32) * 5 for s in shapes]
    plan = B.BatchPlan(shapes, kern)
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    x_flat = plan.pack([torch.from_numpy(v).to(DEV) for v in x0])
    x_flat, res = plan.iterate(f_flat, x_flat, init=0, max_iters=4, tol=0.0)
    for f, v0, xv in zip(fs, x0, plan.views(x_flat)):
        xr, _ = oracle.iterate(f, okf(kern), x0=v0, iters=4)
        assert np.linalg.norm(xv.double().cpu().numpy() - xr) / np.linalg.norm(xr) < 1e-5


def test_autotune_roundtrip(P, tmp_path):
    Pm, B = P
    from paper_2212_08058_amd import _native as N
    kern = Pm.Kernel(4.0, 1.5, 8, 3)
    path = str(tmp_path / "tune.txt")
    v, ms = B.autotune((16, 120, 216), kern, cache_path=path, reps=3)
    assert v >= 0 and ms > 0
    text = open(path).read()
    assert "gfx950" in text
    B.autotune_clear()
    B.autotune_load(path)
    # the tuned variant is used: results still match the oracle
    f, _ = synth.blob_clip(16, 120, 216, 3, 5)
    x, r = Pm.power_iterate(torch.from_numpy(f).to(DEV), kern, iters=3)
    xr, _ = oracle.iterate(f, okf(kern), iters=3)
    assert np.linalg.norm(x.double().cpu().numpy() - xr) / np.linalg.norm(xr) < 1e-5
    B.autotune_clear()


def test_pipelined_batch_variant(P, tmp_path):
    """A tuned entry for the dominant frame size steers the plan to the
    pipelined 15 x 108 tile: its results match the oracle per clip and are
    bitwise those of the single-clip path on the same variant."""
    Pm, B = P
    from paper_2212_08058_amd import _native as N
    kern = Pm.Kernel(4.0, 1.5, 8, 3)
    shapes = [(14, 45, 216), (6, 45, 216), (9, 30, 108), (3, 45, 216)]
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = tmp_path / "tune.txt"
    path.write_text(f"{arch} 0 8 3 45 216 8 3 15 108 512 5 4 1 1 1.0\n")
    B.autotune_clear()
    B.autotune_load(str(path))
    try:
        plan = B.BatchPlan(shapes, kern)
        info = plan.info()
        assert (info["TH"], info["TW"], info["PIPE"]) == (15, 108, 1), info
        fs = _clips(shapes, seed=40)
        f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
        s = torch.cuda.Stream()
        x_flat, res = plan.iterate(f_flat, max_iters=6, tol=0.0, stream=s)
        torch.cuda.synchronize()
        whole = 0
        for f, xv, r in zip(fs, plan.views(x_flat), res):
            xr, _ = oracle.iterate(f, okf(kern), iters=6)
            err = float(np.linalg.norm(xv.double().cpu().numpy() - xr) / np.linalg.norm(xr))
            assert r["iters"] == 6 and err < 1e-5, (f.shape, err)
            xs, rs = Pm.power_iterate(torch.from_numpy(f).to(DEV), kern, iters=6)
            if Pm.launch_shape(f.shape, kern)["segments"] == 1:
                assert torch.equal(xs, xv), f.shape
                whole += 1
        assert whole, "no clip compared bitwise"
    finally:
        B.autotune_clear()


@pytest.mark.parametrize("kp,tile", [((4.0, 1.5, 8, 3), "8 3 32 64"), ((5.0, 2.0, 15, 5), "16 5 32 128")])
def test_batch_matrix_core_product_form(P, tmp_path, kp, tile):
    """The matrix-core batch variants run in product form (every clip's buffers
    hold f x g with its own g). A tuned entry for the dominant frame size steers
    the plan to them, so ragged small clips are covered: per-clip results from
    the uniform start and from given starts match the oracle, and a clip with
    f = 0 fails alone."""
    Pm, B = P
    kern = Pm.Kernel(*kp)
    shapes = [(9, 40, 70), (3, 17, 23), (1, 64, 80), (12, 31, 33), (1, 1, 1), (7, 70, 140)]
    fs = _clips(shapes, seed=50)
    fs[1] = fs[1] * 1e-6  # a clip on another scale (its own power of two)
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    path = tmp_path / "tune.txt"
    path.write_text(f"{arch} 0 {kern.r_s} {kern.r_t} 70 140 {tile} 512 16 4 1 3 1.0\n")
    B.autotune_clear()
    B.autotune_load(str(path))
    try:
        _batch_product_form_checks(Pm, B, kern, shapes, fs)
    finally:
        B.autotune_clear()


def _batch_product_form_checks(Pm, B, kern, shapes, fs):
    plan = B.BatchPlan(shapes, kern)
    info = plan.info()
    print(info)
    assert info["PIPE"] == 3
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    x_flat, res = plan.iterate(f_flat, max_iters=6, tol=0.0)
    for f, xv, r in zip(fs, plan.views(x_flat), res):
        xr, oi = oracle.iterate(f, okf(kern), iters=6)
        err = float(np.linalg.norm(xv.double().cpu().numpy() - xr) / np.linalg.norm(xr))
        print(f.shape, "uniform", f"{err:.3e}")
        assert r["iters"] == 6 and err < 1e-5, (f.shape, err)
        assert abs(r["lambda_"] - oi.lambdas[-1]) < 1e-5 * oi.lambdas[-1]
    rng = np.random.default_rng(3)
    x0 = [rng.uniform(0.1, 1, s).astype(np.float32) for s in shapes]
    x_flat = plan.pack([torch.from_numpy(v).to(DEV) for v in x0])
    x_flat, res = plan.iterate(f_flat, x_flat, init=0, max_iters=5, tol=0.0)
    for f, v0, xv in zip(fs, x0, plan.views(x_flat)):
        xr, _ = oracle.iterate(f, okf(kern), x0=v0, iters=5)
        err = float(np.linalg.norm(xv.double().cpu().numpy() - xr) / np.linalg.norm(xr))
        print(f.shape, "x0", f"{err:.3e}")
        assert err < 1e-5, (f.shape, err)
    fz = list(fs)
    fz[2] = np.zeros_like(fs[2])
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fz])
    x_flat, res = plan.iterate(f_flat, max_iters=50, tol=1e-4, check=False)
    assert res[2]["status"] == 3 and not res[2]["converged"]
    for k in (0, 3, 5):
        xr, oi = oracle.iterate(fz[k], okf(kern), tol=1e-4, cap=50)
        assert abs(res[k]["iters"] - oi.iters) <= 1, (k, res[k]["iters"], oi.iters)


@pytest.mark.parametrize("kp", [(2.0, 1.0, 4, 2), (4.0, 1.5, 8, 3)])
def test_batch_rise_check_restarts_on_device(P, kp):
    """init = 2: per clip, the warm-start rule (restart from the uniform start
    if the second residual exceeds the first) runs on the device. Warm starts
    made to rise (the second eigenvector of the clip's dense A plus 1e-3 of the
    first: the iterate then turns away from it faster at the second step)
    restart: their result is bitwise that of a uniform-start run two steps
    shorter, flags bit 2 set, iteration count including the discarded steps.
    The other clips (start near the Perron vector) are bitwise the init = 0
    run. Both the plain tile loop (r = (4, 2)) and the matrix-core loop in
    product form (r = (8, 3))."""
    Pm, B = P
    kern = Pm.Kernel(*kp)
    shapes = [(3, 8, 12), (2, 10, 14), (4, 6, 15), (3, 9, 9)]
    fs = _clips(shapes, seed=40)
    x0s, bad = [], []
    for i, f in enumerate(fs):
        A = oracle.dense_matrix(f, okf(kern))
        lam, V = np.linalg.eigh(A)
        v1, v2 = V[:, -1] * np.sign(V[:, -1].sum()), V[:, -2]
        if i % 2 == 0:
            x0 = v2 + 1e-3 * v1
        else:
            x0 = v1 + 1e-3 * np.random.default_rng(i).standard_normal(v1.size)
        x0s.append(torch.from_numpy((x0 / np.linalg.norm(x0)).reshape(f.shape).astype(np.float32)).to(DEV))
        bad.append(i % 2 == 0)
    plan = B.BatchPlan(shapes, kern)
    print("plan", plan.info())
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    n = 12
    x_warm = plan.pack(x0s)
    x_warm, res = plan.iterate(f_flat, x_warm, init=2, max_iters=n, tol=0.0)
    x_unif, res_u = plan.iterate(f_flat, init=1, max_iters=n - 2, tol=0.0)
    x_plain = plan.pack(x0s)
    x_plain, res_p = plan.iterate(f_flat, x_plain, init=0, max_iters=n, tol=0.0)
    torch.cuda.synchronize()
    for i, (r, ru, rp) in enumerate(zip(res, res_u, res_p)):
        xw, xu, xp = (list(plan.views(v))[i] for v in (x_warm, x_unif, x_plain))
        print(i, "bad" if bad[i] else "good", "r1", r["r1"], "r2", r["r2"], "flags", r["flags"], "iters", r["iters"])
        assert r["iters"] == n
        if bad[i]:
            assert r["r2"] > r["r1"] and r["flags"] & 4
            assert torch.equal(xw, xu) and r["lambda_"] == ru["lambda_"] and r["residual"] == ru["residual"]
        else:
            assert r["r2"] <= r["r1"] and not r["flags"] & 4
            assert torch.equal(xw, xp) and r["lambda_"] == rp["lambda_"]


def test_batch_converged_clips_leave_the_tile_list(P):
    """Clips that stop at different iterations leave the active tile list
    (rebuilt after every step): every clip's result is bitwise that of the
    same clip planned alone, iteration count and convergence included."""
    Pm, B = P
    kern = Pm.Kernel(4.0, 1.5, 8, 3)
    shapes = [(16, 120, 216)] * 6 + [(16, 120, 216)]
    fs = _clips(shapes, seed=50)
    plan = B.BatchPlan(shapes, kern)
    f_flat = plan.pack([torch.from_numpy(f).to(DEV) for f in fs])
    x_flat, res = plan.iterate(f_flat, max_iters=300, tol=1e-4)
    iters = [r["iters"] for r in res]
    print("iterations", iters)
    for i, f in enumerate(fs):
        one = B.BatchPlan([shapes[i]], kern)
        xo, ro = one.iterate(one.pack([torch.from_numpy(f).to(DEV)]), max_iters=300, tol=1e-4)
        assert ro[0]["iters"] == res[i]["iters"] and ro[0]["converged"] == res[i]["converged"]
        assert torch.equal(list(one.views(xo))[0], list(plan.views(x_flat))[i])
