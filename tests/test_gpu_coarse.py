"""Grid transfer kernels (box-average downsampling, nearest / linear
upsampling) against the FP64 oracle, and the two-level start end to end."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
DTYPES = [(torch.float32, 2e-7), (torch.bfloat16, 2.0 ** -8), (torch.float64, 1e-15)]


@pytest.fixture(scope="module")
def P():
    import paper_2212_08058_amd as P
    from paper_2212_08058_amd import api, warmstart
    return P, api, warmstart


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def stored(a, dtype):
    """Device tensor of dtype and the values it holds, in float64."""
    t = torch.from_numpy(np.ascontiguousarray(a)).to(DEV).to(dtype)
    return t, t.double().cpu().numpy()


@pytest.mark.parametrize("dtype,tol", DTYPES)
@pytest.mark.parametrize("shape,sy,st", [((7, 13, 22), 4, 3), ((5, 16, 16), 2, 1), ((3, 9, 10), 1, 1),
                                         ((9, 31, 47), 5, 2), ((1, 1, 3), 4, 2)])
def test_downsample_matches_oracle(P, dtype, tol, shape, sy, st):
    _, api, _ = P
    rng = np.random.default_rng(sum(shape) + sy)
    f, fv = stored(rng.uniform(0, 1, shape), dtype)
    out = api.downsample(f, sy, st)
    torch.cuda.synchronize()
    ref = oracle.downsample(fv, sy, st)
    assert out.shape == ref.shape
    assert rel(out.double().cpu().numpy(), ref) <= tol


@pytest.mark.parametrize("dtype,tol", DTYPES)
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("shape,sy,st", [((7, 13, 22), 4, 3), ((6, 16, 16), 2, 2), ((9, 31, 47), 5, 2)])
def test_upsample_matches_oracle(P, dtype, tol, mode, shape, sy, st):
    _, api, _ = P
    rng = np.random.default_rng(sum(shape) + 10 * mode)
    cs = api.coarse_shape(shape, sy, st)
    xc, xcv = stored(rng.uniform(0, 1, cs), dtype)
    m, mv = stored(rng.uniform(0.5, 1, shape), dtype)
    for mul, mulv in ((None, None), (m, mv)):
        out = api.upsample(xc, shape, sy, st, mode=mode, mul=mul)
        torch.cuda.synchronize()
        ref = oracle.upsample(xcv, shape, sy, st, mode=mode, mul=mulv)
        assert rel(out.double().cpu().numpy(), ref) <= 4 * tol


def test_two_level_start_reaches_the_plain_eigenvector(P):
    """The two-level start (coarse iteration, linear prolongation times f)
    converges to the same eigenvector as the plain method, and the coarse
    eigenvector itself is the oracle's on the coarse grid."""
    Pm, api, W = P
    shape = (12, 60, 100)
    f, _ = synth.blob_clip(*shape, 3, 31)
    kern = Pm.Kernel(4.0, 1.5, 8, 3)
    fd = torch.from_numpy(f).to(DEV)
    tl = W.TwoLevel(shape, kern, sy=4, st=2, tol=1e-5)
    u0 = tl.start(fd)
    torch.cuda.synchronize()
    kc = oracle.coarse_kernel(oracle.Kernel(float(np.float32(4.0)), float(np.float32(1.5)), 8, 3), 4, 2)
    fc = oracle.downsample(f, 4, 2)
    assert rel(tl.fc.double().cpu().numpy(), fc) < 1e-6
    kc32 = oracle.Kernel(float(np.float32(kc.sigma_s)), float(np.float32(kc.sigma_t)), kc.r_s, kc.r_t)
    xc_ref, _ = oracle.iterate(tl.fc.double().cpu().numpy(), kc32, tol=1e-9, cap=20000)
    cos_c = float(np.sum(tl.xc.double().cpu().numpy() * xc_ref))
    assert 1.0 - cos_c < 1e-6
    ref_u0 = oracle.upsample(tl.xc.double().cpu().numpy(), shape, 4, 2, mode=1, mul=f)
    assert rel(u0.double().cpu().numpy(), ref_u0) < 1e-6
    xw, info, _ = W.solve_two_level(tl, fd, kern, tol=1e-4, cap=2000)
    xp, rp = Pm.power_iterate(fd, kern, tol=1e-4, max_iters=2000)
    torch.cuda.synchronize()
    assert info["converged"] and rp["converged"]
    assert 1.0 - float(torch.sum(xw.double() * xp.double())) < 1e-3
    assert info["iters"] <= rp["iters"]


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16, torch.float64])
def test_scale_kernel(P, dtype):
    """stpi_scale: y = x s (times a device double when given), formed in
    double and rounded once to the storage type (bfloat16: from the float
    value, as every store of the library): bit-exact against the same
    rounding on the host; y may be x; n = 0 is a no-op."""
    _, api, _ = P
    rng = np.random.default_rng(5)
    x, xv = stored(rng.standard_normal(10007) * 3.0, dtype)
    sd = torch.tensor([0.37], dtype=torch.float64, device=DEV)
    for s, dev in ((1.7, None), (2.5, sd)):
        m = s * (0.37 if dev is not None else 1.0)
        y = api.scale(x, s, s_dev=dev)
        want = xv * m
        if dtype == torch.float64:
            ref = want
        else:
            ref = torch.from_numpy(want.astype(np.float32)).to(dtype).double().numpy()
        got = y.double().cpu().numpy()
        assert np.array_equal(got, ref), (dtype, s, np.max(np.abs(got - ref)))
    if dtype == torch.bfloat16:
        # x = +-m 2^e with m odd in [129, 169]: 1.5 x = 3m 2^(e-1) has a 9-bit
        # odd significand, exactly halfway between two bfloat16 values, so
        # every element tests the conversion's ties-to-even rule (half of
        # them round up, half down)
        m = np.arange(129, 170, 2, dtype=np.float64)
        e = np.arange(-20, 21, dtype=np.float64)
        tv = (m[:, None] * np.exp2(e)[None, :]).ravel()
        tv = np.concatenate([tv, -tv])
        t = torch.from_numpy(tv).to(torch.bfloat16)
        assert np.array_equal(t.double().numpy(), tv)
        want = (tv * 1.5).astype(np.float32)
        assert np.array_equal(want.astype(np.float64), tv * 1.5)
        ref = torch.from_numpy(want).to(torch.bfloat16).double().numpy()
        up = np.abs(ref) > np.abs(tv * 1.5)
        assert 0 < up.sum() < up.size
        got = api.scale(t.to(DEV), 1.5).double().cpu().numpy()
        assert np.array_equal(got, ref), np.flatnonzero(got != ref)[:8]
    z = x.clone()
    api.scale(z, 3.0, out=z)
    torch.cuda.synchronize()
    ref = xv * 3.0 if dtype == torch.float64 else torch.from_numpy((xv * 3.0).astype(np.float32)).to(dtype).double().numpy()
    assert np.array_equal(z.double().cpu().numpy(), ref)
    e = torch.empty(0, dtype=dtype, device=DEV)
    api.scale(e, 2.0)
