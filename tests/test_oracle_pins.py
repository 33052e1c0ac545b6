"""Pins for the FP64 oracle: checks against mathematics the paper fixes.

None of these re-types the oracle's loops. They use library routines
(scipy.ndimage.correlate, numpy.linalg.eigh, torch CPU ops), closed forms
(Kronecker factorisation, the tridiagonal-Toeplitz sine eigenvector),
invariants (symmetry, scaling, flips, Collatz-Wielandt) and finite
differences, so that a dropped term, a wrong sign or index, or a transposed
operand in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from scipy import ndimage

import oracle
from oracle import Kernel

pytestmark = pytest.mark.filterwarnings("ignore::DeprecationWarning")


def _g1(r, sigma):
    d = np.arange(-r, r + 1, dtype=np.float64)
    return np.exp(-d * d / (2.0 * sigma * sigma))


def _toeplitz_1d(n, r, sigma):
    """n x n truncated-Gaussian Toeplitz matrix (zero outside the band |i-j| <= r)."""
    col = np.zeros(n)
    g = _g1(r, sigma)
    m = min(n, r + 1)
    col[:m] = g[r:r + m]
    return scipy.linalg.toeplitz(col)


def _rand_volume(rng, T, H, W, lo=0.05, hi=1.0):
    return rng.uniform(lo, hi, size=(T, H, W))


@pytest.fixture(autouse=True)
def _built(oracle_mod):
    return oracle_mod


# --- the operator -----------------------------------------------------------

@pytest.mark.parametrize("shape,k", [
    ((3, 7, 9), Kernel(1.3, 0.8, 2, 1)),
    ((5, 12, 10), Kernel(2.0, 1.0, 4, 2)),
    ((2, 5, 6), Kernel(3.0, 2.0, 6, 3)),   # radius larger than the volume
])
def test_apply_matches_library_correlation(shape, k):
    """A x = f * correlate(f x, G3D) with scipy's zero-padded ('constant') correlation."""
    rng = np.random.default_rng(1)
    f = _rand_volume(rng, *shape)
    x = rng.standard_normal(shape)
    G3 = np.einsum("a,b,c->abc", _g1(k.r_t, k.sigma_t), _g1(k.r_s, k.sigma_s), _g1(k.r_s, k.sigma_s))
    ref = f * ndimage.correlate(f * x, G3, mode="constant", cval=0.0)
    z = oracle.apply(f, x, k)
    np.testing.assert_allclose(z, ref, rtol=1e-12, atol=1e-12)


def test_apply_matches_dense_matrix_bruteforce():
    """Tiny volume: the explicit pair-by-pair adjacency times x equals the oracle step."""
    rng = np.random.default_rng(2)
    k = Kernel(1.5, 1.0, 2, 1)
    f = _rand_volume(rng, 3, 4, 5)
    x = rng.standard_normal((3, 4, 5))
    A = oracle.dense_matrix(f, k)
    np.testing.assert_allclose(A, A.T, atol=0)
    np.testing.assert_allclose(oracle.apply(f, x, k).reshape(-1), A @ x.reshape(-1), rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("shape,k", [
    ((16, 120, 216), Kernel(4.0, 1.5, 8, 3)),
    ((7, 33, 41), Kernel(5.0, 2.0, 15, 5)),
])
def test_kronecker_closed_form(shape, k):
    """f = a (x) b (x) c and x = p (x) q (x) r give
    A x = (Da Kt Da p) (x) (Db Ky Db q) (x) (Dc Kx Dc r) exactly (1D Toeplitz factors)."""
    rng = np.random.default_rng(3)
    T, H, W = shape
    a, b, c = (rng.uniform(0.2, 1.0, n) for n in shape)
    p, q, r = (rng.uniform(0.1, 1.0, n) for n in shape)
    f = np.einsum("i,j,l->ijl", a, b, c)
    x = np.einsum("i,j,l->ijl", p, q, r)
    Kt = _toeplitz_1d(T, k.r_t, k.sigma_t)
    Ky = _toeplitz_1d(H, k.r_s, k.sigma_s)
    Kx = _toeplitz_1d(W, k.r_s, k.sigma_s)
    ft = a * (Kt @ (a * p))
    fy = b * (Ky @ (b * q))
    fx = c * (Kx @ (c * r))
    ref = np.einsum("i,j,l->ijl", ft, fy, fx)
    z = oracle.apply(f, x, k)
    np.testing.assert_allclose(z, ref, rtol=1e-11)


def test_one_hot_features_pin_self_loop():
    """f = c e_i gives A = c^2 e_i e_i^T: the centre tap is G(0) = 1."""
    k = Kernel(2.0, 1.0, 3, 2)
    f = np.zeros((4, 6, 7))
    f[2, 3, 4] = 0.7
    x = np.random.default_rng(4).uniform(0.1, 1, f.shape)
    z = oracle.apply(f, x, k)
    expect = np.zeros_like(f)
    expect[2, 3, 4] = 0.49 * x[2, 3, 4]
    np.testing.assert_allclose(z, expect, rtol=1e-15, atol=0)


def test_symmetry_scaling_and_flips():
    rng = np.random.default_rng(5)
    k = Kernel(2.5, 1.2, 4, 2)
    f = _rand_volume(rng, 6, 11, 13)
    x = rng.standard_normal(f.shape)
    y = rng.standard_normal(f.shape)
    Ax, Ay = oracle.apply(f, x, k), oracle.apply(f, y, k)
    # zero padding and an even kernel make A symmetric
    assert abs(np.sum(y * Ax) - np.sum(Ay * x)) < 1e-11 * np.sum(np.abs(y * Ax))
    # f -> c f gives z -> c^2 z; linear in x
    np.testing.assert_allclose(oracle.apply(3.0 * f, x, k), 9.0 * Ax, rtol=1e-13, atol=1e-13 * np.abs(Ax).max())
    np.testing.assert_allclose(oracle.apply(f, 2 * x - y, k), 2 * Ax - Ay, rtol=1e-11, atol=1e-11)
    # flipping any axis commutes with the operator
    for ax in range(3):
        np.testing.assert_allclose(oracle.apply(np.flip(f, ax), np.flip(x, ax), k), np.flip(Ax, ax),
                                   rtol=1e-12, atol=1e-12)
    # swapping the two spatial axes commutes (isotropic spatial kernel)
    ft, xt = np.ascontiguousarray(f.transpose(0, 2, 1)), np.ascontiguousarray(x.transpose(0, 2, 1))
    np.testing.assert_allclose(oracle.apply(ft, xt, k), Ax.transpose(0, 2, 1), rtol=1e-12, atol=1e-12)


def test_apply_at_matches_apply():
    rng = np.random.default_rng(6)
    k = Kernel(2.0, 1.0, 4, 2)
    f = _rand_volume(rng, 5, 17, 19)
    x = rng.standard_normal(f.shape)
    idx = rng.integers(0, f.size, 200)
    np.testing.assert_array_equal(oracle.apply_at(f, x, k, idx), oracle.apply(f, x, k).reshape(-1)[idx])
    with pytest.raises(ValueError):
        oracle.apply_at(f, x, k, [f.size])


def test_invalid_arguments_rejected():
    with pytest.raises(ValueError):
        oracle.apply(np.ones((2, 2, 2)), np.ones((2, 2, 2)), Kernel(0.0, 1.0, 1, 1))
    with pytest.raises(ValueError):
        oracle.apply(np.ones((2, 2, 2)), np.ones((2, 2, 2)), Kernel(1.0, 1.0, -1, 1))


# --- the converged limit -----------------------------------------------------

@pytest.mark.parametrize("shape,k,seed", [
    ((2, 8, 8), Kernel(1.5, 1.0, 2, 1), 0),
    ((4, 8, 16), Kernel(2.0, 1.0, 3, 2), 1),
    ((8, 8, 8), Kernel(1.0, 1.0, 1, 1), 2),
])
def test_power_iteration_reaches_dense_perron_vector(shape, k, seed):
    """<= 512 nodes: converged oracle iterate = numpy.linalg.eigh top eigenvector (Eq. 3)."""
    rng = np.random.default_rng(seed)
    f = _rand_volume(rng, *shape, lo=0.05, hi=0.5)
    # a bright space-time blob makes the spectral gap comfortable
    f[: min(3, shape[0]), 2:5, 2:5] += 1.5
    A = oracle.dense_matrix(f, k)
    lam, v, w = oracle.perron(A)
    assert w[-2] / lam < 0.9
    x, info = oracle.iterate(f, k, tol=1e-13, cap=5000)
    assert info.converged
    xf = x.reshape(-1)
    cosd = 1.0 - abs(float(np.dot(xf, v)))
    assert cosd < 1e-12
    assert float(xf.min()) >= -1e-15
    assert np.linalg.norm(A @ xf - info.lambdas[-1] * xf) / lam < 1e-10
    assert abs(info.lambdas[-1] - lam) / lam < 1e-12
    assert abs(info.rayleigh[-1] - lam) / lam < 1e-12


def test_sine_closed_form_eigenvector():
    """r = 1, f = 1: each axis is tridiagonal Toeplitz [q, 1, q] with q = exp(-1/(2 sigma^2));
    the Perron vector is sin(pi i/(n+1)) per axis and lambda = prod(1 + 2 q cos(pi/(n+1)))."""
    T, H, W = 4, 6, 7
    k = Kernel(1.1, 0.9, 1, 1)
    f = np.ones((T, H, W))
    x, info = oracle.iterate(f, k, tol=1e-13, cap=20000)
    assert info.converged

    def axis(n, sigma):
        i = np.arange(1, n + 1)
        q = math.exp(-1.0 / (2 * sigma * sigma))
        return np.sin(math.pi * i / (n + 1)), 1 + 2 * q * math.cos(math.pi / (n + 1))

    (vt, lt), (vy, ly), (vx, lx) = axis(T, k.sigma_t), axis(H, k.sigma_s), axis(W, k.sigma_s)
    v = np.einsum("i,j,l->ijl", vt, vy, vx)
    v /= np.linalg.norm(v)
    assert np.max(np.abs(x - v)) < 1e-10
    assert abs(info.lambdas[-1] - lt * ly * lx) < 1e-10


def test_collatz_wielandt_bracket():
    """For positive x: min (Ax)_i/x_i <= lambda_1 <= max (Ax)_i/x_i, tightening as x converges."""
    rng = np.random.default_rng(7)
    k = Kernel(2.0, 1.0, 2, 1)
    f = _rand_volume(rng, 3, 7, 8, lo=0.3)
    lam, v, _ = oracle.perron(oracle.dense_matrix(f, k))
    widths = []
    for it in (1, 5, 40):
        x, _ = oracle.iterate(f, k, iters=it)
        ratio = oracle.apply(f, x, k) / x
        assert ratio.min() <= lam * (1 + 1e-12) and ratio.max() >= lam * (1 - 1e-12)
        widths.append(ratio.max() - ratio.min())
    assert widths[0] > widths[1] > widths[2]


def test_iteration_counts_and_residual_definition():
    rng = np.random.default_rng(8)
    k = Kernel(2.0, 1.0, 4, 2)
    f = _rand_volume(rng, 4, 16, 20)
    x10, info10 = oracle.iterate(f, k, iters=10)
    assert info10.iters == 10 and len(info10.residuals) == 10 and not info10.converged
    # the fixed-count run equals the trajectory of the tolerance run
    xs = oracle.iterate(f, k, iters=3, keep=True)[2]
    assert len(xs) == 4
    np.testing.assert_allclose(info10.residuals[2], np.linalg.norm(xs[3] - xs[2]), rtol=1e-14)
    # tolerance mode stops at the first residual below tol
    x, info = oracle.iterate(f, k, tol=1e-3, cap=500)
    assert info.converged and info.residuals[-1] < 1e-3 and all(r >= 1e-3 for r in info.residuals[:-1])
    # zero features: A x = 0 is reported, not divided by
    _, info0 = oracle.iterate(np.zeros((2, 3, 4)), k, iters=3)
    assert info0.status == "zero_norm" and info0.iters == 0


# --- channel combination, loss and the reverse mode -------------------------

def test_softmax_and_combine_against_library():
    import scipy.special
    rng = np.random.default_rng(9)
    w = rng.standard_normal(8)
    np.testing.assert_allclose(oracle.softmax(w), scipy.special.softmax(w), rtol=1e-14)
    fc = rng.uniform(0, 1, (8, 2, 3, 4))
    f = oracle.combine(fc, w)
    a = scipy.special.softmax(w)
    np.testing.assert_allclose(f, sum(a[c] * fc[c] for c in range(8)), rtol=1e-14)


def test_combine_bwd_finite_differences():
    rng = np.random.default_rng(10)
    w = rng.standard_normal(5)
    fc = rng.uniform(0, 1, (5, 2, 3, 4))
    gf = rng.standard_normal((2, 3, 4))
    g = oracle.combine_bwd(fc, w, gf)
    h = 1e-6
    for c in range(5):
        e = np.zeros(5)
        e[c] = h
        fd = (np.sum(gf * oracle.combine(fc, w + e)) - np.sum(gf * oracle.combine(fc, w - e))) / (2 * h)
        assert abs(fd - g[c]) < 1e-8


def test_bce_against_torch_and_finite_differences():
    import torch
    rng = np.random.default_rng(11)
    x = rng.uniform(0.0, 1.0, (2, 5, 6))
    x[0, 0, 0] = 0.0   # clipped at eps
    gt = rng.uniform(size=x.shape) < 0.4
    loss, g = oracle.bce(x, gt)
    xt = torch.tensor(x, dtype=torch.float64)
    yt = torch.clamp(xt / xt.max(), oracle.BCE_EPS, 1 - oracle.BCE_EPS)
    ref = torch.nn.functional.binary_cross_entropy(yt, torch.tensor(gt, dtype=torch.float64))
    assert abs(loss - float(ref)) < 1e-12
    h = 1e-7
    for i in rng.integers(1, x.size, 12):   # skip the clipped entry
        e = np.zeros(x.size)
        e[i] = h
        e = e.reshape(x.shape)
        fd = (oracle.bce(x + e, gt)[0] - oracle.bce(x - e, gt)[0]) / (2 * h)
        assert abs(fd - g.reshape(-1)[i]) < 1e-6 * max(1.0, abs(fd))
    # the max entry's derivative includes the max-normalisation term
    a = int(np.argmax(x))
    e = np.zeros(x.size)
    e[a] = h
    e = e.reshape(x.shape)
    fd = (oracle.bce(x + e, gt)[0] - oracle.bce(x - e, gt)[0]) / (2 * h)
    assert abs(fd - g.reshape(-1)[a]) < 1e-6 * max(1.0, abs(fd))


def test_adjoint_finite_differences_end_to_end():
    """dL/dw through combine -> 6 normalised steps -> BCE, against central differences in FP64."""
    rng = np.random.default_rng(12)
    k = Kernel(1.5, 1.0, 2, 1)
    C, shape = 4, (3, 8, 9)
    fc = rng.uniform(0.05, 1.0, (C,) + shape)
    gt = rng.uniform(size=shape) < 0.3
    w = rng.standard_normal(C) * 0.5
    loss, gw, _ = oracle.loss_and_grad(fc, w, gt, k, iters=6)
    h = 1e-6
    for c in range(C):
        e = np.zeros(C)
        e[c] = h
        lp = oracle.loss_and_grad(fc, w + e, gt, k, 6)[0]
        lm = oracle.loss_and_grad(fc, w - e, gt, k, 6)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gw[c]) <= 1e-6 * max(abs(fd), 1e-3), (c, fd, gw[c])


def test_adjoint_df_finite_differences():
    """dL/df for a linear functional L = <c, x_K>, checked voxel by voxel."""
    rng = np.random.default_rng(13)
    k = Kernel(1.7, 1.1, 2, 1)
    f = rng.uniform(0.1, 1.0, (3, 5, 6))
    cvec = rng.standard_normal(f.shape)
    tape = oracle.forward_train(f, k, 4)
    gf = oracle.adjoint(f, k, tape, cvec)
    h = 1e-6
    for i in rng.integers(0, f.size, 10):
        e = np.zeros(f.size)
        e[i] = h
        e = e.reshape(f.shape)
        lp = np.sum(cvec * oracle.forward_train(f + e, k, 4)["xs"][-1])
        lm = np.sum(cvec * oracle.forward_train(f - e, k, 4)["xs"][-1])
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gf.reshape(-1)[i]) < 1e-7, (i, fd, gf.reshape(-1)[i])


# --- the warm-start network ---------------------------------------------------

def test_conv3d_against_torch():
    import torch
    rng = np.random.default_rng(14)
    x = rng.standard_normal((3, 4, 5, 6))
    w = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    out = oracle.conv3d(x, w, b)
    ref = torch.nn.functional.conv3d(torch.tensor(x)[None], torch.tensor(w), torch.tensor(b), padding=1)[0]
    np.testing.assert_allclose(out, ref.numpy(), rtol=1e-12, atol=1e-12)
    go = rng.standard_normal(out.shape)
    xt = torch.tensor(x, requires_grad=True)
    wt = torch.tensor(w, requires_grad=True)
    bt = torch.tensor(b, requires_grad=True)
    torch.nn.functional.conv3d(xt[None], wt, bt, padding=1)[0].backward(torch.tensor(go))
    gi, gw, gb = oracle.conv3d_bwd(x, w, go)
    np.testing.assert_allclose(gi, xt.grad.numpy(), rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(gw, wt.grad.numpy(), rtol=1e-12, atol=1e-11)
    np.testing.assert_allclose(gb, bt.grad.numpy(), rtol=1e-12, atol=1e-12)


def test_conv3d_delta_kernel_is_a_shift():
    rng = np.random.default_rng(15)
    x = rng.standard_normal((1, 4, 5, 6))
    w = np.zeros((1, 1, 3, 3, 3))
    w[0, 0, 2, 1, 0] = 1.0   # out[t,y,x] = in[t+1, y, x-1]
    out = oracle.conv3d(x, w, np.zeros(1))[0]
    ref = np.zeros((4, 5, 6))
    ref[:-1, :, 1:] = x[0, 1:, :, :-1]
    np.testing.assert_array_equal(out, ref)


def test_net_backward_finite_differences():
    rng = np.random.default_rng(16)
    chans = (1, 2, 2, 1)
    params = [(rng.standard_normal((chans[i + 1], chans[i], 3, 3, 3)) * 0.4, rng.standard_normal(chans[i + 1]) * 0.1)
              for i in range(3)]
    f = rng.uniform(0, 1, (3, 4, 5))
    tgt = rng.uniform(0, 1, f.shape)
    tgt /= np.linalg.norm(tgt)
    y, cache = oracle.net_forward(f, params)
    loss, gy = oracle.net_loss(y, tgt)
    grads = oracle.net_backward(cache, gy)
    h = 1e-6
    for li in range(3):
        for flat in rng.integers(0, params[li][0].size, 3):
            pp = [(w.copy(), b.copy()) for w, b in params]
            pm = [(w.copy(), b.copy()) for w, b in params]
            pp[li][0].reshape(-1)[flat] += h
            pm[li][0].reshape(-1)[flat] -= h
            fd = (oracle.net_loss(oracle.net_forward(f, pp)[0], tgt)[0]
                  - oracle.net_loss(oracle.net_forward(f, pm)[0], tgt)[0]) / (2 * h)
            assert abs(fd - grads[li][0].reshape(-1)[flat]) < 1e-7 * max(1, abs(fd))
        pp = [(w.copy(), b.copy()) for w, b in params]
        pm = [(w.copy(), b.copy()) for w, b in params]
        pp[li][1][0] += h
        pm[li][1][0] -= h
        fd = (oracle.net_loss(oracle.net_forward(f, pp)[0], tgt)[0]
              - oracle.net_loss(oracle.net_forward(f, pm)[0], tgt)[0]) / (2 * h)
        assert abs(fd - grads[li][1][0]) < 1e-7 * max(1, abs(fd))


def test_bf16_rounding_against_torch():
    import torch
    rng = np.random.default_rng(17)
    a = np.concatenate([rng.standard_normal(1000) * 10.0 ** rng.integers(-8, 8, 1000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38]])
    ref = torch.tensor(a, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(oracle.bf16_round(a), ref)


def test_adamw_against_torch():
    import torch
    rng = np.random.default_rng(18)
    w0 = rng.standard_normal(7)
    wt = torch.tensor(w0, requires_grad=True)
    opt = torch.optim.AdamW([wt], lr=3e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.05, amsgrad=True)
    w, m, v, vm = w0.copy(), np.zeros(7), np.zeros(7), np.zeros(7)
    for step in range(1, 6):
        g = rng.standard_normal(7) * (0.1 if step == 3 else 1.0)
        wt.grad = torch.tensor(g)
        opt.step()
        w, m, v, vm = oracle.adamw_step(w, g, m, v, vm, step, lr=3e-3, weight_decay=0.05)
        np.testing.assert_allclose(w, wt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_fallback_rule():
    assert oracle.fallback(0.1, 0.2)
    assert not oracle.fallback(0.2, 0.1)
    assert not oracle.fallback(0.1, 0.1)
    assert oracle.fallback(0.1, float("nan"))


# ---- two-level start: grid transfer ------------------------------------------

def test_downsample_divisible_is_block_mean(oracle_mod):
    """On divisible sizes the box average is numpy's reshape-and-mean."""
    rng = np.random.default_rng(40)
    f = rng.uniform(0, 1, (6, 12, 20))
    ref = f.reshape(3, 2, 3, 4, 5, 4).mean(axis=(1, 3, 5))
    assert np.allclose(oracle_mod.downsample(f, 4, 2), ref, rtol=0, atol=1e-15)


def test_downsample_ragged_conserves_mass_and_constants(oracle_mod):
    """Partial edge blocks average what exists: constants stay constant and
    sum(coarse * block size) = sum(fine)."""
    rng = np.random.default_rng(41)
    f = rng.uniform(0, 1, (7, 13, 22))
    sy, st = 4, 3
    c = oracle_mod.downsample(f, sy, st)
    assert c.shape == (3, 4, 6)
    sizes = np.einsum("i,j,k->ijk", [3, 3, 1], [4, 4, 4, 1], [4, 4, 4, 4, 4, 2])
    assert abs(float((c * sizes).sum()) - float(f.sum())) < 1e-12 * f.size
    assert np.allclose(oracle_mod.downsample(np.full(f.shape, 0.37), sy, st), 0.37, rtol=0, atol=1e-15)


def test_upsample_nearest_is_replication(oracle_mod):
    rng = np.random.default_rng(42)
    xc = rng.uniform(0, 1, (3, 4, 6))
    ref = np.repeat(np.repeat(np.repeat(xc, 3, 0), 4, 1), 4, 2)[:7, :13, :22]
    assert np.array_equal(oracle_mod.upsample(xc, (7, 13, 22), 4, 3, mode=0), ref)


def test_upsample_linear_reproduces_affine_functions(oracle_mod):
    """Trilinear interpolation between cell centres is exact for affine data
    away from the clamped borders, and exact for constants everywhere; at a
    cell centre (odd factor) it returns the cell's value."""
    sy, st = 3, 3
    Tc, Hc, Wc = 4, 5, 6
    tc, yc, xc_ = np.meshgrid(np.arange(Tc), np.arange(Hc), np.arange(Wc), indexing="ij")
    coarse = 0.5 + 0.25 * tc - 0.125 * yc + 0.0625 * xc_
    shape = (Tc * st, Hc * sy, Wc * sy)
    up = oracle_mod.upsample(coarse, shape, sy, st, mode=1)
    t, y, x = np.meshgrid(np.arange(shape[0]), np.arange(shape[1]), np.arange(shape[2]), indexing="ij")
    affine = 0.5 + 0.25 * ((t + 0.5) / st - 0.5) - 0.125 * ((y + 0.5) / sy - 0.5) + 0.0625 * ((x + 0.5) / sy - 0.5)
    inner = (slice(1, shape[0] - 1), slice(1, shape[1] - 1), slice(1, shape[2] - 1))
    assert np.allclose(up[inner], affine[inner], rtol=0, atol=1e-14)
    assert np.allclose(up[1::3, 1::3, 1::3], coarse, rtol=0, atol=1e-14)
    assert np.allclose(oracle_mod.upsample(np.full((Tc, Hc, Wc), 2.5), (11, 14, 17), sy, st, mode=1), 2.5,
                       rtol=0, atol=1e-14)


def test_upsample_multiplies_by_field(oracle_mod):
    rng = np.random.default_rng(43)
    xc = rng.uniform(0, 1, (2, 3, 3))
    m = rng.uniform(0, 1, (4, 6, 6))
    for mode in (0, 1):
        assert np.allclose(oracle_mod.upsample(xc, m.shape, 2, 2, mode=mode, mul=m),
                           oracle_mod.upsample(xc, m.shape, 2, 2, mode=mode) * m, rtol=0, atol=1e-15)


def test_coarse_kernel_units(oracle_mod):
    k = oracle_mod.coarse_kernel(oracle_mod.Kernel(4.0, 1.5, 8, 3), 4, 2)
    assert (k.sigma_s, k.sigma_t, k.r_s, k.r_t) == (1.0, 0.75, 2, 2)


# ---- pins for the training tape, the bf16 net mirror and the net loss ----------

@pytest.mark.parametrize("x0", [None, "random"])
def test_forward_train_matches_iterate_trajectory(x0):
    """forward_train's tape is the plain iteration: its iterates and norms are
    iterate(keep=True)'s trajectory and lambdas (which the dense Perron,
    Kronecker and sine pins fix), and each saved v is G (f x_k), checked
    against scipy's zero-padded correlation (Eq. 4 split as f * (G * (f x)))."""
    rng = np.random.default_rng(21)
    k = Kernel(1.7, 0.9, 3, 2)
    f = _rand_volume(rng, 5, 9, 11)
    start = None if x0 is None else rng.uniform(0.1, 1.0, f.shape)
    tape = oracle.forward_train(f, k, 6, x0=start)
    _, info, traj = oracle.iterate(f, k, x0=start, iters=6, keep=True)
    assert len(tape["xs"]) == len(traj) == 7
    for a, b in zip(tape["xs"], traj):
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-13)
    np.testing.assert_allclose(tape["ns"], info.lambdas, rtol=1e-13, atol=0)
    G3 = np.einsum("a,b,c->abc", _g1(k.r_t, k.sigma_t), _g1(k.r_s, k.sigma_s), _g1(k.r_s, k.sigma_s))
    for j, v in enumerate(tape["vs"]):
        ref = ndimage.correlate(f * traj[j], G3, mode="constant", cval=0.0)
        np.testing.assert_allclose(v, ref, rtol=1e-12, atol=1e-14)
        # x_{k+1} = f v / ||f v||
        np.testing.assert_allclose(tape["xs"][j + 1], f * v / np.linalg.norm(f * v), rtol=0, atol=1e-14)


def test_net_forward_bf16_mirror_against_torch():
    """The bf16 mirror rounds the weights and every layer's input activation to
    bfloat16 (torch's own float32 -> bfloat16 cast) and convolves in FP64 with
    unrounded outputs, bias added in FP64, ReLU between layers."""
    import torch
    rng = np.random.default_rng(22)
    chans = oracle.NET_CHANNELS
    params = [(rng.standard_normal((chans[i + 1], chans[i], 3, 3, 3)) * 0.3, rng.standard_normal(chans[i + 1]) * 0.1)
              for i in range(4)]
    f = rng.uniform(0, 1, (3, 6, 7))
    y, _ = oracle.net_forward(f, params, bf16=True)

    def q(a):  # torch bfloat16 rounding, back to float64
        return a.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    h = torch.tensor(f)[None, None]
    for li, (w, b) in enumerate(params):
        h = torch.nn.functional.conv3d(q(h), q(torch.tensor(w)), torch.tensor(b), padding=1)
        if li < 3:
            h = torch.relu(h)
    np.testing.assert_allclose(y, h[0, 0].numpy(), rtol=1e-12, atol=1e-12)
    # the mirror differs from the unrounded net (so the rounding is really applied)
    y_exact, _ = oracle.net_forward(f, params, bf16=False)
    assert np.max(np.abs(y - y_exact)) > 1e-4


def test_net_loss_and_warm_start_against_torch():
    """net_loss is torch's mse_loss against x* sqrt(N), with torch's gradient;
    warm_start_x0 is torch's normalize(relu(y) + eps)."""
    import torch
    rng = np.random.default_rng(23)
    y = rng.standard_normal((3, 5, 4))
    xs = rng.uniform(0, 1, y.shape)
    xs /= np.linalg.norm(xs)
    loss, g = oracle.net_loss(y, xs)
    yt = torch.tensor(y, requires_grad=True)
    lt = torch.nn.functional.mse_loss(yt, torch.tensor(xs) * math.sqrt(y.size))
    lt.backward()
    assert abs(loss - lt.item()) <= 1e-14 * max(1.0, lt.item())
    np.testing.assert_allclose(g, yt.grad.numpy(), rtol=1e-13, atol=1e-16)
    x0 = oracle.warm_start_x0(y, eps=1e-3)
    ref = torch.nn.functional.normalize((torch.relu(torch.tensor(y)) + 1e-3).reshape(-1), dim=0).reshape(y.shape)
    np.testing.assert_allclose(x0, ref.numpy(), rtol=1e-14, atol=1e-16)


# --- the full SFSeg operator (Eq. 2 Taylor affinity, Eq. 5-7) -----------------

def _sfseg_case(seed, shape=(3, 6, 7)):
    rng = np.random.default_rng(seed)
    s = rng.uniform(0.05, 1.0, shape)
    f = rng.uniform(0.0, 1.0, shape)
    x = rng.standard_normal(shape)
    return s, f, x


@pytest.mark.parametrize("alpha", [1.0, 0.3, 2.5])
def test_sfseg_apply_matches_pairwise_matrix(alpha):
    """The direct loop equals the explicit matrix built pair by pair from
    Eq. 2's affinity s_i s_j [1 - alpha (f_i - f_j)^2] G_ij, divided by alpha."""
    k = Kernel(1.7, 0.9, 2, 1)
    s, f, x = _sfseg_case(3)
    M = oracle.sfseg_dense(s, f, alpha, k)
    z = oracle.sfseg_apply(s, f, x, alpha, k)
    ref = (M @ x.reshape(-1)).reshape(x.shape)
    assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("k", [Kernel(1.7, 0.9, 2, 1), Kernel(3.0, 1.5, 5, 2)])
def test_sfseg_apply_matches_three_library_correlations(k):
    """Eq. 7: S (1/alpha - F^2) G*(S X) - S G*(F^2 S X) + 2 S F G*(F S X), each
    G* computed with scipy's zero-padded correlation."""
    s, f, x = _sfseg_case(4, (4, 9, 11))
    alpha = 0.7
    G3 = np.einsum("a,b,c->abc", _g1(k.r_t, k.sigma_t), _g1(k.r_s, k.sigma_s), _g1(k.r_s, k.sigma_s))

    def conv(v):
        return ndimage.correlate(v, G3, mode="constant", cval=0.0)

    u = s * x
    ref = s * (1 / alpha - f * f) * conv(u) - s * conv(f * f * u) + 2 * s * f * conv(f * u)
    z = oracle.sfseg_apply(s, f, x, alpha, k)
    assert np.max(np.abs(z - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert np.max(np.abs(oracle.sfseg_apply_conv(s, f, x, alpha, k) - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_sfseg_special_cases():
    """Constant f: every pairwise difference vanishes and the operator is the
    single-field one on s, divided by alpha. alpha -> 0: alpha times the
    operator tends to the single-field one (the Taylor term is O(alpha))."""
    k = Kernel(2.0, 1.0, 3, 2)
    s, f, x = _sfseg_case(5, (3, 8, 9))
    fc = np.full_like(f, 0.37)
    for alpha in (1.0, 0.25):
        z = oracle.sfseg_apply(s, fc, x, alpha, k)
        ref = oracle.apply(s, x, k) / alpha
        assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))
    a = 1e-9
    z = a * oracle.sfseg_apply(s, f, x, a, k)
    ref = oracle.apply(s, x, k)
    assert np.max(np.abs(z - ref)) <= 1e-7 * np.max(np.abs(ref))


def test_sfseg_symmetry_and_scaling():
    """M is symmetric (<y, M x> = <M y, x>); z is quadratic in s and linear in x."""
    k = Kernel(2.0, 1.0, 3, 1)
    s, f, x = _sfseg_case(6, (3, 7, 10))
    y = np.random.default_rng(60).standard_normal(x.shape)
    a = float(np.sum(y * oracle.sfseg_apply(s, f, x, 0.8, k)))
    b = float(np.sum(oracle.sfseg_apply(s, f, y, 0.8, k) * x))
    assert abs(a - b) <= 1e-12 * abs(a)
    z1 = oracle.sfseg_apply(s, f, x, 0.8, k)
    z2 = oracle.sfseg_apply(2.0 * s, f, 3.0 * x, 0.8, k)
    assert np.max(np.abs(z2 - 12.0 * z1)) <= 1e-12 * np.max(np.abs(z2))


def test_sfseg_perron_vector_and_negative_affinity():
    """With f in [0, 1] and alpha <= 1 every affinity is >= 0 and the power
    iteration reaches the nonnegative principal eigenvector of the dense
    matrix (eigh). With alpha (max f - min f)^2 > 1 some affinities are negative."""
    k = Kernel(2.0, 1.0, 2, 1)
    rng = np.random.default_rng(7)
    s = rng.uniform(0.1, 1.0, (3, 6, 8))
    f = rng.uniform(0.0, 1.0, s.shape)
    M = oracle.sfseg_dense(s, f, 1.0, k)
    assert M.min() >= 0.0
    lam, v, w = oracle.perron(M)
    assert w[-1] - w[-2] > 1e-3 * w[-1]
    x, info = oracle.sfseg_iterate(s, f, 1.0, k, tol=1e-13, cap=20000)
    assert info.converged
    xf = x.reshape(-1)
    assert 1.0 - float(xf @ v) < 1e-12
    assert xf.min() >= -1e-15
    assert abs(info.lambdas[-1] - lam) <= 1e-10 * lam
    Mneg = oracle.sfseg_dense(s, f, 4.0, k)
    assert Mneg.min() < 0.0


# --- online / partial iteration over sub-windows ----------------------------

def test_online_iterate_limits():
    """One window covering the video is the full iteration; windows that do
    not overlap are independent iterations from the uniform start; the start
    of an overlapping window carries the previous solution's shared frames
    (checked on a case whose windows shift by one frame: frame t of window
    w + 1 starts at frame t + 1 of window w's solution)."""
    rng = np.random.default_rng(71)
    f = rng.uniform(0.05, 1.0, (6, 5, 7))
    k = Kernel(1.5, 1.0, 2, 1)
    x_full, info = oracle.iterate(f, k, iters=7)
    x_one, infos = oracle.online_iterate(f, k, q=6, shift=3, iters=7)
    assert len(infos) == 1 and np.array_equal(x_one, x_full)
    x_sep, infos = oracle.online_iterate(f, k, q=3, shift=3, iters=5)
    for a in (0, 3):
        xa, _ = oracle.iterate(f[a:a + 3], k, iters=5)
        assert np.max(np.abs(x_sep[a:a + 3] - xa)) <= 1e-15
    # shift 1, one iteration per window: the second window's start is the
    # first window's solution moved by one frame plus a uniform last frame
    w0, _ = oracle.iterate(f[0:3], k, iters=1)
    start = np.concatenate([w0[1:3], np.full((1, 5, 7), 1.0 / math.sqrt(3 * 5 * 7))])
    w1, _ = oracle.iterate(f[1:4], k, x0=start, iters=1)
    x4, infos = oracle.online_iterate(f[:4], k, q=3, shift=1, iters=1)
    assert len(infos) == 2 and np.max(np.abs(x4[1:4] - w1)) <= 1e-15 and np.array_equal(x4[0], w0[0])


# --- exact exponential affinity (Eq. 1) ---------------------------------------

def test_exp_apply_matches_pairwise_matrix_and_limits():
    """The direct loop equals the explicit matrix of Eq. 1 built pair by pair;
    alpha = 0 is the single-field operator on s; for small alpha the exact
    affinity and alpha times the Taylor operator of Eq. 7 differ by O(alpha^2)
    (exp(-a d^2) = 1 - a d^2 + O(a^2)), checked by the ratio of the errors at
    alpha and alpha / 2."""
    k = Kernel(1.7, 0.9, 2, 1)
    rng = np.random.default_rng(81)
    s = rng.uniform(0.05, 1.0, (3, 6, 7))
    f = rng.uniform(0.0, 1.0, s.shape)
    x = rng.standard_normal(s.shape)
    for alpha in (0.0, 0.8, 3.0):
        E = oracle.exp_dense(s, f, alpha, k)
        z = oracle.exp_apply(s, f, x, alpha, k)
        ref = (E @ x.reshape(-1)).reshape(x.shape)
        assert np.max(np.abs(z - ref)) <= 1e-13 * np.max(np.abs(ref))
    z0 = oracle.exp_apply(s, f, x, 0.0, k)
    assert np.max(np.abs(z0 - oracle.apply(s, x, k))) <= 1e-13 * np.max(np.abs(z0))
    errs = []
    for a in (1e-2, 5e-3):
        d = oracle.exp_apply(s, f, x, a, k) - a * oracle.sfseg_apply(s, f, x, a, k)
        errs.append(np.max(np.abs(d)))
    assert 3.5 <= errs[0] / errs[1] <= 4.5


def test_exp_iterate_perron():
    """The exact-affinity iteration reaches the principal eigenvector of E (eigh)."""
    k = Kernel(2.0, 1.0, 2, 1)
    rng = np.random.default_rng(82)
    s = rng.uniform(0.1, 1.0, (3, 6, 8))
    f = rng.uniform(0.0, 1.0, s.shape)
    lam, v, w = oracle.perron(oracle.exp_dense(s, f, 2.0, k))
    x, info = oracle.exp_iterate(s, f, 2.0, k, tol=1e-13, cap=20000)
    assert info.converged and 1.0 - float(x.reshape(-1) @ v) < 1e-12
    assert abs(info.lambdas[-1] - lam) <= 1e-10 * lam


# --- the SFSeg++ learning objective ---------------------------------------------

def test_pp_pieces_match_torch_autograd():
    """Eq. 9's combination, the soft-binarisation and the per-frame Focal-Dice
    loss and their derivatives against torch (float64, CPU autograd)."""
    import torch
    rng = np.random.default_rng(91)
    fc = rng.uniform(0.0, 1.0, (4, 3, 5, 6))
    w = rng.standard_normal(4)
    b = 0.3
    g_f = rng.standard_normal((3, 5, 6))
    tw = torch.tensor(w, requires_grad=True)
    tb = torch.tensor(b, dtype=torch.float64, requires_grad=True)
    tf = torch.sigmoid((tw[:, None, None, None] * torch.tensor(fc)).sum(0) + tb)
    assert np.max(np.abs(tf.detach().numpy() - oracle.combine_sigmoid(fc, w, b))) <= 1e-15
    (tf * torch.tensor(g_f)).sum().backward()
    gw, gb = oracle.combine_sigmoid_bwd(fc, w, b, g_f)
    assert np.max(np.abs(gw - tw.grad.numpy())) <= 1e-13 and abs(gb - float(tb.grad)) <= 1e-13
    y = rng.standard_normal((3, 5, 6))
    y /= np.linalg.norm(y)
    ty = torch.tensor(y)
    ref = torch.sigmoid(2.5 * (ty * math.sqrt(y.size) - 0.7))
    assert np.max(np.abs(oracle.softbin(y, 2.5, 0.7) - ref.numpy())) <= 1e-15
    x = rng.uniform(0.0, 1.0, (3, 5, 6))
    gt = (rng.uniform(size=x.shape) > 0.5).astype(np.float64)
    tx = torch.tensor(x, requires_grad=True)
    tg = torch.tensor(gt)
    inter = (tx * tg).sum(dim=(1, 2))
    dice = (2 * inter + 1.0) / (tx.sum(dim=(1, 2)) + tg.sum(dim=(1, 2)) + 1.0)
    J = ((1 - dice) ** 0.75).sum()
    J.backward()
    Jo, gxo = oracle.focal_dice(x, gt, 0.75, 1.0)
    assert abs(Jo - float(J)) <= 1e-13 and np.max(np.abs(gxo - tx.grad.numpy())) <= 1e-13


def test_pp_gradient_matches_finite_differences():
    """The whole objective (combination, continuous and soft-binarised
    iterations, Focal-Dice): dJ/dw and dJ/db against central differences."""
    rng = np.random.default_rng(92)
    k = Kernel(2.0, 1.0, 2, 1)
    fc = rng.uniform(0.0, 1.0, (3, 3, 6, 7))
    gt = (rng.uniform(size=fc.shape[1:]) > 0.6).astype(np.float64)
    w = np.array([0.8, -0.4, 1.1])
    b = -0.2
    args = dict(k=k, n_iter=6, n_cont=3, kappa=2.0, theta=1.0)
    J, gw, gb, _ = oracle.loss_and_grad_pp(fc, w, b, gt, **args)
    h = 1e-6
    for c in range(3):
        wp, wm = w.copy(), w.copy()
        wp[c] += h
        wm[c] -= h
        fd = (oracle.loss_and_grad_pp(fc, wp, b, gt, **args)[0] - oracle.loss_and_grad_pp(fc, wm, b, gt, **args)[0]) / (2 * h)
        assert abs(fd - gw[c]) <= 1e-6 * max(1.0, abs(fd)), (c, fd, gw[c])
    fd = (oracle.loss_and_grad_pp(fc, w, b + h, gt, **args)[0] - oracle.loss_and_grad_pp(fc, w, b - h, gt, **args)[0]) / (2 * h)
    assert abs(fd - gb) <= 1e-6 * max(1.0, abs(fd))
    # with no soft-binarised iteration the tape is the plain normalised iteration
    tape = oracle.forward_train_pp(oracle.combine_sigmoid(fc, w, b), k, 5, 5, 2.0, 1.0)
    x_plain, _ = oracle.iterate(oracle.combine_sigmoid(fc, w, b), k, iters=5)
    assert np.max(np.abs(tape["xs"][-1] - x_plain)) <= 1e-14
