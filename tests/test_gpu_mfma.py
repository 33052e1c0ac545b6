"""Matrix-core step variants (both spatial passes as banded products on
v_mfma_f32_16x16x32_f16, operands split into two half-precision parts)
against the FP64 oracle: every space radius they serve, ragged and
degenerate shapes, values far from 1 and of both signs, the single-step
scale, the iteration chain and bfloat16 storage. Same bars as the plain
variants: FP32 per step relative L2 <= 1e-5, BF16 storage <= 2^-8."""
import ctypes

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


def OKf(k):
    return OK(float(np.float32(k.sigma_s)), float(np.float32(k.sigma_t)), k.r_s, k.r_t)


def mfma_variants(dtype_code):
    from paper_2212_08058_amd import _native as N
    out = []
    for i in range(N.lib.stpi_variant_count(dtype_code)):
        info = (ctypes.c_int * 9)()
        assert N.lib.stpi_variant_info(dtype_code, i, info) == 0
        if info[8] == 3:
            out.append((i, list(info)))
    return out


class forced:
    def __init__(self, i):
        from paper_2212_08058_amd import _native as N
        self.N, self.i = N, i

    def __enter__(self):
        assert self.N.lib.stpi_set_variant(self.i) == 0

    def __exit__(self, *a):
        self.N.lib.stpi_set_variant(-1)


def test_variants_are_compiled():
    from paper_2212_08058_amd import _native as N
    v32 = mfma_variants(N.STPI_F32)
    assert v32 and all(info[0] in (8, 16) for _, info in v32)
    assert {info[0] for _, info in v32} == {8, 16}
    assert mfma_variants(N.STPI_BF16)


CASES = [
    ((5, 37, 70), (2.0, 1.0, 4, 2)),       # ragged, one tile
    ((13, 40, 131), (4.0, 1.5, 8, 3)),     # three tiles across
    ((12, 35, 150), (5.0, 2.0, 15, 5)),
    ((7, 70, 200), (10.0, 3.0, 16, 5)),    # the largest space radius, two tile rows
    ((20, 64, 64), (5.0, 2.0, 15, 5)),     # exactly one tile
    ((2, 129, 67), (3.0, 1.0, 6, 3)),      # ragged bottom tile row
    ((3, 17, 19), (1.3, 0.7, 1, 1)),
    ((1, 1, 1), (1.0, 1.0, 2, 1)),         # single voxel
    ((1, 30, 1), (2.0, 1.0, 4, 2)),        # single column
    ((9, 1, 40), (2.0, 1.0, 4, 2)),        # single row
    ((3, 18, 20), (2.0, 1.0, 0, 0)),       # no neighbours: A = diag(f^2)
    ((16, 33, 47), (3.0, 1.0, 5, 0)),      # no temporal neighbours
]


@pytest.mark.parametrize("shape,kp", CASES)
def test_step_matches_oracle(P, shape, kp):
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(*kp)
    rng = np.random.default_rng(sum(shape))
    f = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    ref = 0.7 * oracle.apply(f.astype(np.float64), x.astype(np.float64), OKf(kern))
    fd, xd = torch.from_numpy(f).to(DEV), torch.from_numpy(x).to(DEV)
    ran = 0
    for i, info in mfma_variants(N.STPI_F32):
        if info[1] < kern.r_t or info[0] < kern.r_s:
            continue
        with forced(i):
            z, sums = P.step(fd, xd, kern, x_scale=0.7)
            torch.cuda.synchronize()
        zz = z.double().cpu().numpy()
        err = rel_l2(zz, ref)
        print(shape, kp, "variant", i, info[:5], f"rel L2 {err:.3e}")
        assert err <= 1e-5, (i, err)
        s = sums.cpu().numpy()
        assert abs(s[0] - np.sum(zz * zz)) <= 1e-12 * np.sum(zz * zz)
        ran += 1
    assert ran


@pytest.mark.parametrize("kp", [(5.0, 2.0, 15, 5), (4.0, 1.5, 8, 3)])
@pytest.mark.parametrize("kind", ["tiny", "huge", "signed", "decades"])
def test_value_ranges(P, kind, kp):
    """The half-precision operands are scaled by a power of two from max |f x|:
    results keep float accuracy for inputs far from 1, of either sign, or
    spread over many decades (both slab margins)."""
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(*kp)
    shape = (10, 50, 90)
    rng = np.random.default_rng(7)
    f = rng.uniform(0.05, 1.0, shape)
    x = rng.uniform(0.0, 1.0, shape)
    if kind == "tiny":
        f, x = f * 1e-12, x * 1e-9
    elif kind == "huge":
        f, x = f * 1e8, x * 1e11
    elif kind == "signed":
        f = rng.uniform(-1.0, 1.0, shape)
        x = rng.uniform(-1.0, 1.0, shape)
    else:
        f = 10.0 ** rng.uniform(-7, 0, shape)
    f, x = f.astype(np.float32), x.astype(np.float32)
    scale = {"tiny": 1e6, "huge": 1e-9}.get(kind, 1.0)
    ref = scale * oracle.apply(f.astype(np.float64), x.astype(np.float64), OKf(kern))
    fd, xd = torch.from_numpy(f).to(DEV), torch.from_numpy(x).to(DEV)
    for i, info in mfma_variants(N.STPI_F32):
        if info[1] < kern.r_t or info[0] < kern.r_s:
            continue
        with forced(i):
            z, _ = P.step(fd, xd, kern, x_scale=scale)
            torch.cuda.synchronize()
        err = rel_l2(z.double().cpu().numpy(), ref)
        print(kind, "variant", i, info[:5], f"rel L2 {err:.3e}")
        assert err <= 1e-5, (kind, i, err)


def test_iteration_chain_matches_oracle(P):
    from paper_2212_08058_amd import _native as N
    c = synth.CONFIGS["small"]
    f, _ = synth.blob_clip(c["T"], 96, 150, 3, 0)
    kern = P.Kernel(5.0, 2.0, 15, 5)
    xr, info = oracle.iterate(f, OKf(kern), iters=10)
    fd = torch.from_numpy(f).to(DEV)
    for i, vi in mfma_variants(N.STPI_F32):
        if vi[1] < kern.r_t or vi[0] < kern.r_s:
            continue
        with forced(i):
            x, r = P.power_iterate(fd, kern, iters=10)
            torch.cuda.synchronize()
        err = rel_l2(x.double().cpu().numpy(), xr)
        print("chain variant", i, vi[:5], f"rel L2 {err:.3e}", r["lambda_"], info.lambdas[-1])
        assert r["iters"] == 10 and err <= 1e-5
        assert abs(r["lambda_"] - info.lambdas[-1]) <= 1e-5 * info.lambdas[-1]


def test_tolerance_run_converges_to_oracle(P):
    from paper_2212_08058_amd import _native as N
    f, _ = synth.blob_clip(8, 64, 112, 3, 4)
    kern = P.Kernel(2.0, 1.0, 4, 2)
    xr, info = oracle.iterate(f, OKf(kern), tol=1e-4, cap=400)
    fd = torch.from_numpy(f).to(DEV)
    i, vi = mfma_variants(N.STPI_F32)[0]
    with forced(i):
        x, r = P.power_iterate(fd, kern, tol=1e-4, max_iters=400)
        torch.cuda.synchronize()
    cosd = 1.0 - float(np.sum(x.double().cpu().numpy() * xr))
    print("tolerance run", r["iters"], info.iters, f"cos distance {cosd:.3e}")
    assert r["converged"] and abs(r["iters"] - info.iters) <= 2 and cosd <= 1e-3


def test_bf16_storage(P):
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(5.0, 2.0, 15, 5)
    shape = (9, 70, 133)
    rng = np.random.default_rng(11)
    f = torch.from_numpy(rng.uniform(0.05, 1.0, shape).astype(np.float32)).to(torch.bfloat16)
    x = torch.from_numpy(rng.uniform(0.0, 1.0, shape).astype(np.float32)).to(torch.bfloat16)
    ref = oracle.apply(f.double().numpy(), x.double().numpy(), OKf(kern))
    fd, xd = f.to(DEV), x.to(DEV)
    for i, vi in mfma_variants(N.STPI_BF16):
        if vi[1] < kern.r_t or vi[0] < kern.r_s:
            continue
        with forced(i):
            z, _ = P.step(fd, xd, kern)
            torch.cuda.synchronize()
        err = rel_l2(z.double().cpu().numpy(), ref)
        print("bf16 variant", i, vi[:5], f"rel L2 {err:.3e}")
        assert err <= 2.0 ** -8


def test_matches_plain_variant_at_full_frame(P):
    """At 16 x 480 x 854 the matrix-core and the plain variant agree to float
    accuracy everywhere (the oracle is sampled by the frame-segment test)."""
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(5.0, 2.0, 15, 5)
    f, _ = synth.blob_clip(16, 480, 854, 5, 3)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.0, 1.0, f.shape).astype(np.float32)
    fd, xd = torch.from_numpy(f).to(DEV), torch.from_numpy(x).to(DEV)
    plain = None
    for i in range(N.lib.stpi_variant_count(N.STPI_F32)):
        info = (ctypes.c_int * 9)()
        N.lib.stpi_variant_info(N.STPI_F32, i, info)
        if info[0] == 15 and info[1] == 5 and info[8] == 0:
            plain = i
            break
    assert plain is not None
    with forced(plain):
        zp, sp = P.step(fd, xd, kern)
        torch.cuda.synchronize()
    idx = np.random.default_rng(5).integers(0, f.size, 400)
    ref = oracle.apply_at(f, x, OKf(kern), idx)
    for i, vi in mfma_variants(N.STPI_F32):
        if vi[1] < kern.r_t or vi[0] < kern.r_s:
            continue
        with forced(i):
            z, s = P.step(fd, xd, kern)
            torch.cuda.synchronize()
        d = rel_l2(z.double().cpu().numpy(), zp.double().cpu().numpy())
        e = rel_l2(z.double().reshape(-1)[torch.from_numpy(idx).to(DEV)].cpu().numpy(), ref)
        print("full frame variant", i, vi[:5], f"vs plain {d:.3e}, sampled vs oracle {e:.3e}")
        assert d <= 1e-5 and e <= 1e-5
        assert abs(float(s[0]) / float(sp[0]) - 1.0) <= 2e-5


class plain_form:
    """Selects the plain chain form (both operands staged) for the duration."""

    def __enter__(self):
        import os
        self.old = os.environ.get("STPI_NO_PRODUCT")
        os.environ["STPI_NO_PRODUCT"] = "1"

    def __exit__(self, *a):
        import os
        if self.old is None:
            del os.environ["STPI_NO_PRODUCT"]
        else:
            os.environ["STPI_NO_PRODUCT"] = self.old


PRODUCT_CASES = [
    ((5, 37, 70), (2.0, 1.0, 4, 2)),
    ((13, 40, 131), (4.0, 1.5, 8, 3)),
    ((12, 35, 150), (5.0, 2.0, 15, 5)),
    ((2, 129, 67), (3.0, 1.0, 6, 3)),
    ((1, 1, 1), (1.0, 1.0, 2, 1)),
    ((3, 18, 20), (2.0, 1.0, 0, 0)),
]


@pytest.mark.parametrize("shape,kp", PRODUCT_CASES)
@pytest.mark.parametrize("start", ["uniform", "x0"])
def test_product_form_chain_matches_oracle(P, shape, kp, start):
    """Chains on the matrix-core variants run in product form (the buffers hold
    f x 2^-2e): per variant, the result, lambda and the last residual match the
    oracle's power iteration, from the uniform start and from a given x0."""
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(*kp)
    rng = np.random.default_rng(sum(shape) + 1)
    f = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    x0 = rng.uniform(0.1, 1.0, shape).astype(np.float32) if start == "x0" else None
    xr, info = oracle.iterate(f, OKf(kern), x0=x0, iters=6)
    fd = torch.from_numpy(f).to(DEV)
    ran = 0
    for i, vi in mfma_variants(N.STPI_F32):
        if vi[1] < kern.r_t or vi[0] < kern.r_s:
            continue
        x = None if x0 is None else torch.from_numpy(x0).to(DEV)
        with forced(i):
            ms, pf = P.time_chain_step(fd, kern, reps=1)
            assert pf
            xg, r = P.power_iterate(fd, kern, iters=6, x0=x)
            torch.cuda.synchronize()
        err = rel_l2(xg.double().cpu().numpy(), xr)
        print(shape, kp, start, "variant", i, vi[:5], f"rel L2 {err:.3e}", r["residual"], info.residuals[-1])
        assert r["iters"] == 6 and err <= 1e-5, (i, err)
        assert abs(r["lambda_"] - info.lambdas[-1]) <= 1e-5 * info.lambdas[-1]
        assert abs(r["residual"] - info.residuals[-1]) <= 1e-4 * info.residuals[-1] + 1e-6
        ran += 1
    assert ran


@pytest.mark.parametrize("kind", ["tiny", "huge", "holes", "signed"])
def test_product_form_value_ranges(P, kind):
    """The power-of-two factor 2^-2e keeps w = f x in range for f far from 1;
    voxels with f = 0 (where A x is 0) and f of both signs are exact cases."""
    kern = P.Kernel(5.0, 2.0, 15, 5)
    shape = (10, 50, 90)
    rng = np.random.default_rng(9)
    f = rng.uniform(0.05, 1.0, shape)
    if kind == "tiny":
        f = f * 1e-12
    elif kind == "huge":
        f = f * 1e8
    elif kind == "holes":
        f[rng.uniform(size=shape) < 0.4] = 0.0
        f[:, 10:20, :] = 0.0
    else:
        f = rng.uniform(-1.0, 1.0, shape)
    f = f.astype(np.float32)
    xr, info = oracle.iterate(f, OKf(kern), iters=8)
    fd = torch.from_numpy(f).to(DEV)
    assert P.launch_shape(f.shape, kern)["variant"] >= 0
    _, pf = P.time_chain_step(fd, kern, reps=1)
    x, r = P.power_iterate(fd, kern, iters=8)
    torch.cuda.synchronize()
    err = rel_l2(x.double().cpu().numpy(), xr)
    print(kind, "product form", pf, f"rel L2 {err:.3e}", r["lambda_"], info.lambdas[-1])
    assert pf and err <= 1e-5
    assert abs(r["lambda_"] - info.lambdas[-1]) <= 1e-5 * abs(info.lambdas[-1])
    if kind == "holes":
        assert torch.all(x[torch.from_numpy(f).to(DEV) == 0] == 0)


@pytest.mark.parametrize("kind", ["tiny", "huge", "holes", "signed", "spread"])
def test_product_form_bf16_value_ranges(P, kind):
    """BF16 chains stage the raw bfloat16 values and carry the staging power of
    two in the y-pass taps: f far from 1 on either side (the scales the FP32
    product form is tested at; the power of two then far from 1 too), voxels
    with f = 0, f of both signs and f spread over seven decades (values that
    half precision would hold only as subnormals) match the oracle iterating
    on the rounded f to the storage precision."""
    kern = P.Kernel(5.0, 2.0, 15, 5)
    shape = (10, 50, 90)
    rng = np.random.default_rng(19)
    f = rng.uniform(0.05, 1.0, shape)
    if kind == "tiny":
        f = f * 1e-12
    elif kind == "huge":
        f = f * 1e8
    elif kind == "holes":
        f[rng.uniform(size=shape) < 0.4] = 0.0
        f[:, 10:20, :] = 0.0
    elif kind == "signed":
        f = rng.uniform(-1.0, 1.0, shape)
    else:
        f = 10.0 ** rng.uniform(-7.0, 0.0, shape)
    fb = torch.from_numpy(f.astype(np.float32)).to(torch.bfloat16)
    xr, info = oracle.iterate(fb.double().numpy(), OKf(kern), iters=8)
    fd = fb.to(DEV)
    _, pf = P.time_chain_step(fd, kern, reps=1)
    x, r = P.power_iterate(fd, kern, iters=8)
    torch.cuda.synchronize()
    err = rel_l2(x.double().cpu().numpy(), xr)
    print(kind, "bf16 product form", pf, f"rel L2 {err:.3e}", r["lambda_"], info.lambdas[-1])
    assert pf and err <= 2.0 ** -8
    assert abs(r["lambda_"] - info.lambdas[-1]) <= 2.0 ** -8 * abs(info.lambdas[-1])
    if kind == "holes":
        assert torch.all(x[fd == 0] == 0)


def test_product_form_agrees_with_plain_form(P):
    """Tolerance runs in the two forms: same stopping step, residuals and
    vectors equal to float rounding (warm start with the rise check too)."""
    kern = P.Kernel(4.0, 1.5, 8, 3)
    f, _ = synth.blob_clip(16, 120, 216, 3, 8)
    fd = torch.from_numpy(f).to(DEV)
    xp, rp = P.power_iterate(fd, kern, tol=1e-4, max_iters=300)
    with plain_form():
        _, pf = P.time_chain_step(fd, kern, reps=1)
        assert not pf
        xq, rq = P.power_iterate(fd, kern, tol=1e-4, max_iters=300)
    torch.cuda.synchronize()
    print("tolerance runs", rp["iters"], rq["iters"], rp["residual"], rq["residual"])
    assert abs(rp["iters"] - rq["iters"]) <= 1 and rp["converged"] and rq["converged"]
    assert float((xp.double() - xq.double()).norm()) <= 1e-4
    # a warm start x0 close to the answer, with the rise check
    x0 = (xq + 0.05 * torch.rand_like(xq)).contiguous()
    xw, rw = P.power_iterate(fd, kern, tol=1e-4, max_iters=300, x0=x0.clone(), rise_check=True)
    with plain_form():
        xv, rv = P.power_iterate(fd, kern, tol=1e-4, max_iters=300, x0=x0.clone(), rise_check=True)
    torch.cuda.synchronize()
    print("warm runs", rw["iters"], rv["iters"], (rw["r1"], rw["r2"]), (rv["r1"], rv["r2"]))
    assert abs(rw["iters"] - rv["iters"]) <= 1
    assert abs(rw["r1"] - rv["r1"]) <= 1e-5 and abs(rw["r2"] - rv["r2"]) <= 1e-5
    assert float((xw.double() - xv.double()).norm()) <= 1e-4


def test_product_form_zero_steps_and_failures(P):
    """A chain of no steps keeps the plain form (x is the normalised start);
    f = 0 fails on the first step in either form."""
    from paper_2212_08058_amd import StpiError
    kern = P.Kernel(5.0, 2.0, 15, 5)
    rng = np.random.default_rng(4)
    f = rng.uniform(0.05, 1.0, (4, 40, 60)).astype(np.float32)
    x0 = rng.uniform(0.1, 1.0, f.shape).astype(np.float32)
    x, r = P.power_iterate(torch.from_numpy(f).to(DEV), kern, iters=0, x0=torch.from_numpy(x0).to(DEV))
    assert r["iters"] == 0
    np.testing.assert_allclose(x.double().cpu().numpy(), x0 / np.linalg.norm(x0.astype(np.float64)), rtol=1e-6)
    with pytest.raises(StpiError) as ei:
        P.power_iterate(torch.zeros((2, 40, 60), device=DEV), kern, iters=3)
    assert ei.value.status == 3


@pytest.mark.parametrize("kp", [(5.0, 2.0, 15, 5), (4.0, 1.5, 8, 3)])
def test_product_form_full_frame(P, kp):
    """At 16 x 480 x 854 (full frames, the default variant of each radius) a
    product-form chain agrees with the plain-form chain to float rounding, and
    sampled outputs of its last step match the oracle applied to the GPU's
    previous iterate."""
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(*kp)
    f, _ = synth.blob_clip(16, 480, 854, 5, 6)
    fd = torch.from_numpy(f).to(DEV)
    shape = P.launch_shape(f.shape, kern)
    info = (ctypes.c_int * 9)()
    N.lib.stpi_variant_info(N.STPI_F32, shape["variant"], info)
    assert info[8] == 3, list(info)  # the matrix-core loop is the default at both radii
    x4, _ = P.power_iterate(fd, kern, iters=4)
    x5, r5 = P.power_iterate(fd, kern, iters=5)
    with plain_form():
        xq, rq = P.power_iterate(fd, kern, iters=5)
    torch.cuda.synchronize()
    d = rel_l2(x5.double().cpu().numpy(), xq.double().cpu().numpy())
    print(kp, "variant", list(info), f"product vs plain {d:.3e}", r5["lambda_"], rq["lambda_"])
    assert d <= 1e-5
    assert abs(r5["lambda_"] - rq["lambda_"]) <= 1e-5 * rq["lambda_"]
    assert abs(r5["residual"] - rq["residual"]) <= 1e-4 * rq["residual"] + 1e-6
    # x5 = A x4 / ||A x4||: sampled outputs against the oracle's A applied to x4
    idx = np.random.default_rng(8).integers(0, f.size, 300)
    x4n = x4.double().cpu().numpy()
    ref = oracle.apply_at(f, x4n, OKf(kern), idx) / r5["lambda_"]
    got = x5.double().reshape(-1)[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    e = rel_l2(got, ref)
    print("sampled vs oracle", f"{e:.3e}")
    assert e <= 1e-5


def test_product_form_bf16_chain(P):
    """BF16 storage in product form (w = f x g stored in bfloat16): the chain
    matches the oracle iterating on the bfloat16-rounded f to the storage
    precision, and the plain form to the same bar."""
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(5.0, 2.0, 15, 5)
    rng = np.random.default_rng(12)
    f = torch.from_numpy(rng.uniform(0.05, 1.0, (9, 70, 133)).astype(np.float32)).to(torch.bfloat16)
    fd = f.to(DEV)
    xr, info = oracle.iterate(f.double().numpy(), OKf(kern), iters=6)
    ran = 0
    for i, vi in mfma_variants(N.STPI_BF16):
        if vi[1] < kern.r_t or vi[0] < kern.r_s:
            continue
        with forced(i):
            _, pf = P.time_chain_step(fd, kern, reps=1)
            x, r = P.power_iterate(fd, kern, iters=6)
            with plain_form():
                xq, _ = P.power_iterate(fd, kern, iters=6)
            torch.cuda.synchronize()
        err = rel_l2(x.double().cpu().numpy(), xr)
        errq = rel_l2(xq.double().cpu().numpy(), xr)
        print("bf16 variant", i, vi[:5], "product form", pf, f"rel L2 {err:.3e}, plain form {errq:.3e}",
              r["lambda_"], info.lambdas[-1])
        assert pf and err <= 2.0 ** -8 and errq <= 2.0 ** -8
        assert abs(r["lambda_"] - info.lambdas[-1]) <= 2.0 ** -8 * info.lambdas[-1]
        ran += 1
    assert ran


def _vector_variant(rs, rt):
    """Index of a compiled vector-ALU step variant (float storage) serving (rs, rt)."""
    from paper_2212_08058_amd import _native as N
    for i in range(N.lib.stpi_variant_count(N.STPI_F32)):
        info = (ctypes.c_int * 9)()
        N.lib.stpi_variant_info(N.STPI_F32, i, info)
        if info[8] != 3 and info[0] >= rs and info[1] >= rt:
            return i
    raise AssertionError("no vector variant")


def test_product_form_low_magnitude_tail(P):
    """Per-voxel accuracy where the iterate is small. The split half-precision
    staging is scaled by the iterate's own maximum, so values far below it
    keep float-level relative accuracy down to about 2^-14 of the maximum and
    an absolute error below 2^-33 of it beneath that. One step at full frame
    size from an iterate spanning seven decades (a decayed background under
    the blobs) against the FP64 oracle's full application: relative L2 over the
    whole volume <= 1e-5, over the voxels below 1e-3 of the maximum <= 1e-5,
    and the largest per-voxel relative error above 1e-4 of the maximum <= 2e-5
    (a voxel there stages at >= 2^-5 with 22 significant bits; its output sums
    about ten thousand such products)."""
    kern = P.Kernel(5.0, 2.0, 15, 5)
    mask, rng = synth.blob_mask(4, 480, 854, 5, 61)
    f = np.clip(mask + rng.uniform(0.0, 1e-3, mask.shape), 0.0, 1.0).astype(np.float32)
    x0 = (mask ** 2 + 10.0 ** rng.uniform(-7.0, -3.0, mask.shape)).astype(np.float32)
    print("case: low-magnitude tail, 4x480x854 r=(15,5), seed 61", flush=True)
    fd = torch.from_numpy(f).to(DEV)
    x1, r1 = P.power_iterate(fd, kern, iters=1, x0=torch.from_numpy(x0).to(DEV))
    torch.cuda.synchronize()
    z = oracle.apply(f, x0.astype(np.float64), OKf(kern))
    ref = z / np.linalg.norm(z)
    got = x1.double().cpu().numpy()
    m = np.abs(ref).max()
    low = np.abs(ref) < 1e-3 * m
    above = np.abs(ref) >= 1e-4 * m
    e_all = rel_l2(got, ref)
    e_low = rel_l2(got[low], ref[low])
    e_vox = float(np.max(np.abs(got[above] - ref[above]) / np.abs(ref[above])))
    print(f"low tail: rel L2 {e_all:.3e}, below 1e-3 max ({low.mean():.1%} of voxels, down to "
          f"{np.abs(ref[low]).min() / m:.1e} of max) {e_low:.3e}, max per-voxel above 1e-4 max {e_vox:.3e}")
    assert e_all <= 1e-5 and e_low <= 1e-5 and e_vox <= 2e-5


def test_product_form_long_chain_matches_vector_loop(P):
    """100 product-form iterations on a 16 x 480 x 854 blob clip at r = (15, 5)
    against the same chain on the vector-ALU loop (float arithmetic
    throughout): relative L2 <= 1e-5 overall and over the voxels below 1e-3 of
    the maximum, where the background has decayed."""
    kern = P.Kernel(5.0, 2.0, 15, 5)
    f, _ = synth.blob_clip(16, 480, 854, 5, 62)
    print("case: 100 iterations, 16x480x854 r=(15,5), seed 62", flush=True)
    fd = torch.from_numpy(f).to(DEV)
    x, r = P.power_iterate(fd, kern, iters=100)
    with forced(_vector_variant(15, 5)):
        xv, rv = P.power_iterate(fd, kern, iters=100)
    torch.cuda.synchronize()
    a = x.double().cpu().numpy()
    b = xv.double().cpu().numpy()
    m = np.abs(b).max()
    low = np.abs(b) < 1e-3 * m
    e_all = rel_l2(a, b)
    e_low = rel_l2(a[low], b[low])
    print(f"100 iterations: matrix-core vs vector rel L2 {e_all:.3e}, below 1e-3 max ({low.mean():.1%} of voxels, "
          f"down to {np.abs(b[low]).min() / m:.1e}) {e_low:.3e}; lambda {r['lambda_']:.9g} vs {rv['lambda_']:.9g}")
    assert e_all <= 1e-5 and e_low <= 1e-5
    assert abs(r["lambda_"] - rv["lambda_"]) <= 1e-6 * rv["lambda_"]


SEGMENT_CASES = [
    ((21, 64, 128), (5.0, 2.0, 15, 5)),   # two frame segments
    ((30, 64, 128), (5.0, 2.0, 15, 5)),   # three: the middle one walks forward with both halos
    ((16, 64, 128), (2.0, 1.0, 4, 2)),    # four
    ((12, 32, 64), (4.0, 1.5, 8, 3)),     # one tile, two segments
]


@pytest.mark.parametrize("shape,kp", SEGMENT_CASES)
def test_frame_segments_walk_both_ways(P, shape, kp):
    """When a launch splits the frames, the segment that ends at the last frame
    (and starts after the first) is walked backward, so its last outputs need
    no ring steps past its input. Per compiled variant (matrix-core and vector
    tile loops) that splits this shape: one step against the oracle's direct
    application with every frame's
    error bounded on its own (the frames next to each segment boundary and the
    last r_t frames are where a wrong frame order or a missed output shows),
    and 6-step product-form chains (FP32 and BF16 storage) against the
    oracle's iteration."""
    from paper_2212_08058_amd import _native as N
    kern = P.Kernel(*kp)
    ok = OKf(kern)
    T = shape[0]
    rng = np.random.default_rng(sum(shape) + 7)
    f = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    ref = oracle.apply(f.astype(np.float64), x.astype(np.float64), ok)
    xr, info = oracle.iterate(f, ok, iters=6)
    fb = torch.from_numpy(f).to(torch.bfloat16)
    xrb, infob = oracle.iterate(fb.double().numpy(), ok, iters=6)
    fd, xd, fbd = torch.from_numpy(f).to(DEV), torch.from_numpy(x).to(DEV), fb.to(DEV)
    split = 0
    for code, dt in ((N.STPI_F32, torch.float32), (N.STPI_BF16, torch.bfloat16)):
        for i in range(N.lib.stpi_variant_count(code)):
            info_c = (ctypes.c_int * 9)()
            assert N.lib.stpi_variant_info(code, i, info_c) == 0
            vi = list(info_c)
            if vi[1] < kern.r_t or vi[0] < kern.r_s:
                continue
            nseg = P.launch_shape(shape, kern, dtype=dt, variant=i)["segments"]
            if nseg < 2:
                continue
            split += 1
            with forced(i):
                if dt == torch.float32:
                    z, _ = P.step(fd, xd, kern)
                    xg, r = P.power_iterate(fd, kern, iters=6)
                else:
                    xg, r = P.power_iterate(fbd, kern, iters=6)
                torch.cuda.synchronize()
            if dt == torch.float32:
                zz = z.double().cpu().numpy()
                per_frame = [rel_l2(zz[t], ref[t]) for t in range(T)]
                print(shape, kp, "variant", i, vi[:5], "segments", nseg, f"worst frame {max(per_frame):.2e}")
                assert max(per_frame) <= 1e-5, (i, nseg, per_frame)
                err = rel_l2(xg.double().cpu().numpy(), xr)
                assert r["iters"] == 6 and err <= 1e-5, (i, err)
                assert abs(r["lambda_"] - info.lambdas[-1]) <= 1e-5 * info.lambdas[-1]
                assert abs(r["residual"] - info.residuals[-1]) <= 1e-4 * info.residuals[-1] + 1e-6
            else:
                xx = xg.double().cpu().numpy()
                err = rel_l2(xx, xrb)
                worst = max(rel_l2(xx[t], xrb[t]) for t in range(T))
                print(shape, kp, "bf16 variant", i, vi[:5], "segments", nseg, f"rel L2 {err:.2e}, worst frame {worst:.2e}")
                assert err <= 2.0 ** -8 and worst <= 2.0 ** -7, (i, err, worst)
                assert abs(r["lambda_"] - infob.lambdas[-1]) <= 2.0 ** -8 * infob.lambdas[-1]
    assert split, "no matrix-core variant split the frames of this shape"
