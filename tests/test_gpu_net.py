"""Warm-start network kernels (BF16 MFMA / FP32 accumulate) against the FP64
oracle's bf16-mirrored convolution, and the warm-start/fallback logic."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def W():
    from paper_2212_08058_amd import warmstart
    return warmstart


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _random_params(W, seed, scale=1.0):
    p = W.init_params(seed=seed)
    rng = np.random.default_rng(seed + 100)
    p = p * scale
    # nonzero biases exercise the bias paths
    flat = p.cpu().numpy()
    return torch.from_numpy(flat).to(DEV)


@pytest.mark.parametrize("shape", [(3, 10, 20), (5, 17, 33), (1, 4, 16)])
def test_forward_matches_bf16_oracle(W, shape):
    rng = np.random.default_rng(1)
    f = rng.uniform(0, 1, shape).astype(np.float32)
    net = W.WarmStartNet(_random_params(W, 3))
    y = net.forward(torch.from_numpy(f).to(DEV)).cpu().numpy()
    y_ref, _ = oracle.net_forward(f, W.unflatten(net.params), bf16=True)
    err = rel(y, y_ref)
    print(shape, "forward rel err", err)
    assert err < 1e-2


def test_shift_kernels_are_exact(W):
    """Delta weights: every layer copies a shifted channel; the output is f shifted (exact in bf16)."""
    shape = (4, 9, 20)
    rng = np.random.default_rng(2)
    f = (rng.integers(0, 64, shape) / 64.0).astype(np.float32)  # exactly representable in bf16
    params = []
    for li in range(4):
        cin, cout = W.CHANNELS[li], W.CHANNELS[li + 1]
        w = np.zeros((cout, cin, 3, 3, 3))
        b = np.zeros(cout)
        for co in range(cout):
            ci = co % cin
            w[co, ci, 1, 1, 2 if li == 1 else 1] = 1.0   # layer 2 shifts by +1 in x
        params += [w.reshape(-1), b]
    flat = torch.from_numpy(np.concatenate(params).astype(np.float32)).to(DEV)
    net = W.WarmStartNet(flat)
    y = net.forward(torch.from_numpy(f).to(DEV)).cpu().numpy()
    ref = np.zeros(shape)
    ref[:, :, :-1] = f[:, :, 1:]
    np.testing.assert_array_equal(y, ref)


def test_backward_matches_oracle(W):
    shape = (4, 12, 21)
    rng = np.random.default_rng(4)
    f = rng.uniform(0, 1, shape).astype(np.float32)
    xs = rng.uniform(0, 1, shape)
    xs = (xs / np.linalg.norm(xs)).astype(np.float32)
    net = W.WarmStartNet(_random_params(W, 5))
    fd = torch.from_numpy(f).to(DEV)
    y = net.forward(fd)
    loss = net.backward(fd, y, torch.from_numpy(xs).to(DEV))
    g = net.grad.cpu().numpy()
    params = W.unflatten(net.params)
    y_ref, cache = oracle.net_forward(f, params, bf16=True)
    lref, gy = oracle.net_loss(y_ref, xs)
    grads = oracle.net_backward(cache, gy)
    assert abs(float(loss) - lref) < 2e-2 * lref
    off = 0
    for li, (gw, gb) in enumerate(grads):
        n = gw.size
        e1 = rel(g[off:off + n], gw.reshape(-1))
        e2 = rel(g[off + n:off + n + gb.size], gb)
        print("layer", li + 1, "dW rel err", e1, "db rel err", e2)
        assert e1 < 3e-2 and e2 < 3e-2
        off += n + gb.size


def test_training_lowers_loss(W):
    from paper_2212_08058_amd import Kernel, power_iterate
    kern = Kernel(4.0, 1.5, 8, 3)
    fs, ts = [], []
    for i in range(4):
        f, _ = synth.blob_clip(8, 60, 100, 3, 700 + i)
        fd = torch.from_numpy(f).to(DEV)
        x, r = power_iterate(fd, kern, tol=1e-6, max_iters=3000)
        fs.append(fd)
        ts.append(x)
    net = W.WarmStartNet(lr=3e-3)
    losses = []
    for ep in range(30):
        tot = 0.0
        for fd, x in zip(fs, ts):
            tot += float(net.train_step(fd, x))
        losses.append(tot)
    print("losses", losses[0], losses[-1])
    assert losses[-1] < 0.5 * losses[0]


def test_warm_start_and_fallback(W):
    from paper_2212_08058_amd import Kernel
    kern = Kernel(2.0, 1.0, 2, 1)
    k = oracle.Kernel(2.0, 1.0, 2, 1)
    # two blobs: the principal eigenvector sits on one, the second on the other
    f = np.full((2, 8, 16), 0.05)
    f[:, 2:6, 1:5] = 1.0
    f[:, 2:6, 10:14] = 0.9
    A = oracle.dense_matrix(f, k)
    w, V = np.linalg.eigh(A)
    v1, v2 = V[:, -1] * np.sign(V[:, -1].sum()), V[:, -2]
    xstar = v1.reshape(f.shape)
    fd = torch.from_numpy(f.astype(np.float32)).to(DEV)

    class Mock:
        def __init__(self, x0):
            self.v = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float32)).to(DEV)

        def x0(self, _f):
            return self.v.clone()

    # exact start: converges at once
    x, info, _ = W.solve_warm(Mock(xstar), fd, kern, tol=1e-4)
    assert info["iters"] == 1 and not info["fallback"]
    # start on the losing blob: the residual rises, the run falls back to uniform and still finds x*
    bad = (v2 + 1e-3 * v1).reshape(f.shape)
    x, info, _ = W.solve_warm(Mock(bad), fd, kern, tol=1e-4, cap=5000)
    print(info)
    assert info["fallback"] and info["r2"] > info["r1"] and info["converged"]
    xg = x.double().cpu().numpy()
    assert 1 - abs(float(np.sum(xg * xstar))) < 1e-3
    assert oracle.fallback(info["r1"], info["r2"])


def test_unusable_warm_start_falls_back(W):
    """A warm start that vanishes wherever f > 0 (A x0 = 0) or holds a
    non-finite value falls back to the uniform start and still finds the
    principal eigenvector (the dense eigh Perron vector)."""
    from paper_2212_08058_amd import Kernel
    kern = Kernel(2.0, 1.0, 2, 1)
    k = oracle.Kernel(2.0, 1.0, 2, 1)
    f = np.zeros((2, 8, 16))
    f[:, 2:6, 1:5] = 1.0
    f[:, 2:6, 10:14] = 0.6
    A = oracle.dense_matrix(f, k)
    _, V = np.linalg.eigh(A)
    xstar = (V[:, -1] * np.sign(V[:, -1].sum())).reshape(f.shape)
    fd = torch.from_numpy(f.astype(np.float32)).to(DEV)

    class Mock:
        def __init__(self, x0):
            self.v = torch.from_numpy(np.ascontiguousarray(x0, dtype=np.float32)).to(DEV)

        def x0(self, _f):
            return self.v.clone()

    off_support = (f == 0).astype(np.float32)   # zero wherever f > 0
    nonfinite = np.ones_like(f, dtype=np.float32)
    nonfinite[0, 0, 0] = np.inf
    for name, x0 in (("zero on supp(f)", off_support), ("non-finite", nonfinite)):
        x, info, _ = W.solve_warm(Mock(x0), fd, kern, tol=1e-6, cap=5000)
        print(name, info)
        assert info["fallback"] and info["converged"], name
        xg = x.double().cpu().numpy()
        assert 1 - float(np.sum(xg * xstar)) < 1e-5, name
