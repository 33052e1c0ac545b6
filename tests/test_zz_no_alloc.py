"""stpi_step_noalloc (the single step for callers that cannot allocate) against
stpi_step on the same inputs: two calls in a row, the second on a smaller
problem, then the first again (the scratch keeps the previous call's
contents), plus the oracle on the small case and the size limit."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def P():
    import paper_2212_08058_amd as P
    return P


def _inputs(shape, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.05, 1.0, shape).astype(np.float32)
    x = rng.uniform(0.0, 1.0, shape).astype(np.float32)
    return f, x


def _both(P, f, x, kern, scale):
    fd = torch.from_numpy(f).to(DEV)
    xd = torch.from_numpy(x).to(DEV)
    z_ref, s_ref = P.step(fd, xd, kern, x_scale=scale)
    z = torch.full_like(fd, float("nan"))
    s = torch.full((2,), float("nan"), dtype=torch.float64, device=DEV)
    P.step_noalloc(fd, xd, kern, scale, z, s)
    torch.cuda.synchronize()
    return z.cpu().numpy(), s.cpu().numpy(), z_ref.cpu().numpy(), s_ref.cpu().numpy()


def test_noalloc_step_matches_stpi_step(P):
    big = (16, 480, 854)
    kb = P.Kernel(5.0, 2.0, 15, 5)  # matrix-core variant: the bound word is used too
    c = synth.CONFIGS["small"]
    small = (c["T"], c["H"], c["W"])
    ks = P.Kernel(c["sigma_s"], c["sigma_t"], c["r_s"], c["r_t"])
    for shape, kern, seed, scale in ((big, kb, 1, 0.3), (small, ks, 2, 0.7), (big, kb, 3, 1.5)):
        print(f"noalloc step {shape} r=({kern.r_s},{kern.r_t}) seed {seed}", flush=True)
        f, x = _inputs(shape, seed)
        z, s, z_ref, s_ref = _both(P, f, x, kern, scale)
        # the same kernels in the same launch shape: bitwise equal outputs and sums
        assert np.array_equal(z, z_ref), np.max(np.abs(z - z_ref))
        assert np.array_equal(s, s_ref), (s, s_ref)
        if shape == small:
            k64 = oracle.Kernel(float(np.float32(kern.sigma_s)), float(np.float32(kern.sigma_t)), kern.r_s, kern.r_t)
            ref = oracle.apply(f.astype(np.float64), x.astype(np.float64) * scale, k64)
            err = float(np.linalg.norm(z - ref) / np.linalg.norm(ref))
            print(f"  rel L2 vs FP64 oracle {err:.3e}")
            assert err <= 1e-5, err


def test_noalloc_rejects_oversized_problems(P):
    from paper_2212_08058_amd import _native as N
    p = N.Problem(1, 4096, 16384, 2.0, 1.0, 4, 2, N.STPI_F32)
    need = N.lib.stpi_step_noalloc_scratch_bytes(ctypes.byref(p))
    assert need > N.STPI_NOALLOC_SCRATCH_BYTES, need
    f = torch.zeros((1, 4096, 16384), device=DEV)
    z = torch.zeros_like(f)
    s = torch.zeros(2, dtype=torch.float64, device=DEV)
    rc = N.lib.stpi_step_noalloc(ctypes.byref(p), f.data_ptr(), f.data_ptr() + 0, 1.0, z.data_ptr(), s.data_ptr(),
                                 None)
    assert rc == N.STPI_EUNSUPPORTED
    assert b"scratch" in N.lib.stpi_last_error()
    # a problem that fits is within the limit
    q = N.Problem(64, 480, 854, 5.0, 2.0, 15, 5, N.STPI_F32)
    assert 0 < N.lib.stpi_step_noalloc_scratch_bytes(ctypes.byref(q)) <= N.STPI_NOALLOC_SCRATCH_BYTES
