"""Online / partial iteration over sub-windows (Sec. 4, "Online vs Offline
processing") on the GPU: the window start vector exactly, every window and the
assembled video against the FP64 oracle's partial iteration (<= 1e-5
relative L2), and the one-window limit against the full iteration."""
import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import Kernel as OK

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def O():
    import paper_2212_08058_amd as P
    from paper_2212_08058_amd import online
    return P, online


def okf(k):
    return OK(float(np.float32(k.sigma_s)), float(np.float32(k.sigma_t)), k.r_s, k.r_t)


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_window_start_vector(O, dtype):
    P, On = O
    kern = P.Kernel(2.0, 1.0, 4, 2)
    q, H, W = 5, 9, 13
    prev = torch.from_numpy(np.random.default_rng(3).standard_normal((q, H, W))).to(DEV).to(dtype)
    for shift in (0, 1, 3, 5):
        x0 = torch.full((q, H, W), float("nan"), dtype=dtype, device=DEV)
        On.window_start(prev, shift, kern, x0)
        ref = np.concatenate([prev.cpu().numpy()[shift:],
                              np.full((shift, H, W), 1.0 / np.sqrt(q * H * W))]).astype(x0.dtype == torch.float32
                                                                                        and np.float32 or np.float64)
        assert np.array_equal(x0.cpu().numpy(), ref), shift


@pytest.mark.parametrize("q,shift,iters", [(4, 2, 5), (5, 1, 3), (6, 6, 4), (7, 3, 6)])
def test_online_matches_oracle(O, q, shift, iters):
    P, On = O
    kern = P.Kernel(2.0, 1.0, 4, 2)
    f, _ = synth.blob_clip(13, 40, 70, 3, 5)
    print(f"case: online q={q} shift={shift} iters={iters}", flush=True)
    x, res = On.online_iterate(torch.from_numpy(f).to(DEV), kern, q, shift, iters=iters)
    torch.cuda.synchronize()
    xr, infos = oracle.online_iterate(f, okf(kern), q, shift, iters=iters)
    assert len(res) == len(infos)
    err = rel_l2(x.double().cpu().numpy(), xr)
    print(f"  windows {len(res)}, rel L2 {err:.3e}")
    assert err <= 1e-5
    for r, info in zip(res, infos):
        assert r["iters"] == iters and abs(r["lambda_"] - info.lambdas[-1]) <= 1e-5 * info.lambdas[-1]


def test_one_window_is_the_full_iteration(O):
    P, On = O
    kern = P.Kernel(4.0, 1.5, 8, 3)
    f, _ = synth.blob_clip(10, 60, 90, 3, 6)
    fd = torch.from_numpy(f).to(DEV)
    x, res = On.online_iterate(fd, kern, 10, 4, iters=8)
    xf, rf = P.power_iterate(fd, kern, iters=8)
    torch.cuda.synchronize()
    assert len(res) == 1
    assert float((x.double() - xf.double()).norm()) <= 1e-6
    assert abs(res[0]["lambda_"] - rf["lambda_"]) <= 1e-6 * rf["lambda_"]
