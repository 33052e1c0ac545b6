"""FP64 CPU oracle for the space-time power iteration (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package. It shares no code with the HIP
library and never imports it; the two meet only through the seeded inputs of
the ``synth`` module.

What it computes, each function citing the passage it restates:

* ``apply``/``apply_at``: one application of the affinity matrix
  A = diag(f) G diag(f) as a direct 3D neighbourhood sum (C, ``stpi_oracle.c``)
  -- Eq. 2 with alpha = 0, Eq. 4, first convolution term of Eq. 7.
* ``iterate``: power iteration with global L2 normalisation after every
  application (Eq. 4 + Eq. 8, Alg. 1 outer loop).
* ``sfseg_apply``/``sfseg_apply_at``/``sfseg_iterate``/``sfseg_dense``: the
  full SFSeg operator with the first-order Taylor affinity of Eq. 2
  (alpha > 0, unary map s = S^p distinct from the pairwise feature f), in the
  scaling of the update of Eq. 7 (M / alpha), as a direct neighbourhood sum
  (C) and as an explicit matrix; ``sfseg_apply_conv`` restates Eq. 7 itself
  (three Gaussian filterings of s x, f^2 s x and f s x, recombined per voxel).
* ``exp_apply``/``exp_dense``/``exp_iterate``: the exact exponential pairwise
  affinity of Eq. 1 (before the Taylor approximation), direct loop and
  explicit matrix, for the exact-vs-approximate comparison of Sec. 4
  ("Quantitative analysis").
* ``online_iterate``: partial iterations over moving sub-windows, each
  started from the previous window's solution on the shared frames (Sec. 4,
  "Online vs Offline processing").
* ``dense_matrix``/``perron``: the explicit N x N adjacency on tiny volumes and
  its principal eigenvector (Eq. 3, Perron-Frobenius).
* ``combine``/``combine_bwd``: softmax-weighted channel sum f = sum_c
  softmax(w)_c f_c (the multi-channel combination of Eq. 9, in the
  convex-combination form used for learning the channel weights).
* ``forward_train``/``adjoint``: reverse-mode derivative of the normalised
  iteration (gradient through the full spectral algorithm, Sec. 3.4).
* ``bce``: binary cross-entropy on x / max(x).
* ``combine_sigmoid``/``softbin``/``focal_dice``/``forward_train_pp``/
  ``adjoint_pp``/``loss_and_grad_pp``: the paper's learning objective on the
  single-field operator: the sigmoid-affine combination with bias (Eq. 9),
  soft-binarised iterations after the first N_cont (Alg. 1, step 3) and the
  Focal-Dice loss (Eq. 12), with the reverse mode through all of them.
* ``net_forward``/``net_backward``: 4-layer 3x3x3 'same' conv net (C).
* ``adamw_step``: AdamW with AMSGrad (Eq. 13).
* ``fallback``: warm-start fallback rule.
* ``downsample``/``upsample``/``coarse_kernel``: grid transfer for the
  two-level start (box average; nearest-cell or cell-centred trilinear
  prolongation) and the coarse filter. Not from the paper (its warm start is
  the previous sub-window's solution, Sec. 4, "Online vs Offline processing"): restated from the textbook
  definitions, each per output voxel.

Readings of points the paper leaves open (unnormalised Gaussian with G(0)=1,
the 2*sigma^2 convention, box support, zero padding, global normalisation,
residual = ||x_{k+1} - x_k||_2 between unit vectors) are fixed here and
listed in the design notes.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "stpi_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ci, cd = ctypes.c_int, ctypes.c_double
        lib.oracle_apply.argtypes = [ci, ci, ci, dp, dp, cd, cd, ci, ci, dp]
        lib.oracle_apply_at.argtypes = [ci, ci, ci, dp, dp, cd, cd, ci, ci, i64p, ctypes.c_int64, dp]
        lib.oracle_sfseg_apply.argtypes = [ci, ci, ci, dp, dp, dp, cd, cd, cd, ci, ci, dp]
        lib.oracle_sfseg_apply_at.argtypes = [ci, ci, ci, dp, dp, dp, cd, cd, cd, ci, ci, i64p, ctypes.c_int64, dp]
        lib.oracle_exp_apply.argtypes = [ci, ci, ci, dp, dp, dp, cd, cd, cd, ci, ci, dp]
        lib.oracle_conv3d_fwd.argtypes = [ci, ci, ci, ci, ci, dp, dp, dp, dp]
        lib.oracle_conv3d_bwd.argtypes = [ci, ci, ci, ci, ci, dp, dp, dp, dp, dp, dp]
        lib.oracle_num_threads.restype = ci
        lib.oracle_set_threads.argtypes = [ci]
        _lib = lib
    return _lib


def num_threads() -> int:
    return _load().oracle_num_threads()


def set_threads(n: int) -> None:
    _load().oracle_set_threads(int(n))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass(frozen=True)
class Kernel:
    """Truncated space-time Gaussian: sigmas in pixels / frames, box radii."""
    sigma_s: float
    sigma_t: float
    r_s: int
    r_t: int


# ---------------------------------------------------------------------------
# Operator and power iteration
# ---------------------------------------------------------------------------

def apply(f, x, k: Kernel) -> np.ndarray:
    """z = A x with A_ij = f_i f_j G_ij (direct neighbourhood loop, FP64)."""
    f = _f64(f)
    x = _f64(x)
    assert f.ndim == 3 and f.shape == x.shape
    T, H, W = f.shape
    z = np.empty_like(f)
    rc = _load().oracle_apply(T, H, W, _dptr(f), _dptr(x), k.sigma_s, k.sigma_t, k.r_s, k.r_t, _dptr(z))
    if rc != 0:
        raise ValueError("oracle_apply: invalid arguments")
    return z


def apply_at(f, x, k: Kernel, idx) -> np.ndarray:
    """(A x)_i for the flat indices ``idx`` only."""
    f = _f64(f)
    x = _f64(x)
    T, H, W = f.shape
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.shape, dtype=np.float64)
    rc = _load().oracle_apply_at(T, H, W, _dptr(f), _dptr(x), k.sigma_s, k.sigma_t, k.r_s, k.r_t,
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.size, _dptr(out))
    if rc != 0:
        raise ValueError("oracle_apply_at: invalid arguments or index out of range")
    return out


@dataclass
class IterInfo:
    iters: int = 0
    converged: bool = False
    residuals: list = None
    lambdas: list = None        # ||A x_k|| for each application (x_k unit)
    rayleigh: list = None       # <x_k, A x_k>
    status: str = "ok"          # "ok" | "zero_norm" | "nonfinite"


def iterate(f, k: Kernel, x0=None, iters: int | None = None, tol: float | None = None,
            cap: int | None = None, keep=False):
    """Power iteration x_{k+1} = A x_k / ||A x_k|| (Eq. 4, Eq. 8).

    x0 defaults to the uniform unit vector 1/sqrt(N) (Sec. 4: uniform or the
    unary map). It is normalised before the first application. With ``iters``
    the loop runs exactly that many applications; with ``tol`` it stops at the
    first k whose residual ||x_k - x_{k-1}|| < tol, or at ``cap``. The
    residual is taken directly on the difference of the two unit vectors.
    Returns (x, IterInfo) or, with keep=True, (x, IterInfo, [x_0 .. x_K]).
    """
    f = _f64(f)
    return _power(lambda v: apply(f, v, k), f.shape, x0, iters, tol, cap, keep)


def _power(apply_fn, shape, x0, iters, tol, cap, keep):
    """The loop of ``iterate`` for any operator ``apply_fn``."""
    N = int(np.prod(shape))
    x = np.full(shape, 1.0 / math.sqrt(N)) if x0 is None else _f64(x0).copy()
    nx = math.sqrt(float(np.sum(x * x)))
    if not nx > 0:
        raise ValueError("x0 has zero norm")
    x = x / nx
    limit = iters if iters is not None else (cap if cap is not None else 1000)
    info = IterInfo(residuals=[], lambdas=[], rayleigh=[])
    traj = [x.copy()] if keep else None
    for _ in range(limit):
        z = apply_fn(x)
        n = math.sqrt(float(np.sum(z * z)))
        if not math.isfinite(n):
            info.status = "nonfinite"
            break
        if n == 0.0:
            info.status = "zero_norm"
            break
        info.rayleigh.append(float(np.sum(x * z)))
        x1 = z / n
        r = math.sqrt(float(np.sum((x1 - x) ** 2)))
        info.iters += 1
        info.residuals.append(r)
        info.lambdas.append(n)
        x = x1
        if keep:
            traj.append(x.copy())
        if iters is None and tol is not None and r < tol:
            info.converged = True
            break
    if keep:
        return x, info, traj
    return x, info


def sfseg_apply(s, f, x, alpha: float, k: Kernel) -> np.ndarray:
    """z = (M x) / alpha with M_ij = s_i s_j [1 - alpha (f_i - f_j)^2] G_ij
    (Eq. 2, Taylor affinity; the update of Eq. 5-7), direct loop in FP64."""
    s, f, x = _f64(s), _f64(f), _f64(x)
    assert s.ndim == 3 and s.shape == f.shape == x.shape
    T, H, W = s.shape
    z = np.empty_like(s)
    rc = _load().oracle_sfseg_apply(T, H, W, _dptr(s), _dptr(f), _dptr(x), float(alpha), k.sigma_s, k.sigma_t,
                                    k.r_s, k.r_t, _dptr(z))
    if rc != 0:
        raise ValueError("oracle_sfseg_apply: invalid arguments")
    return z


def sfseg_apply_at(s, f, x, alpha: float, k: Kernel, idx) -> np.ndarray:
    """(M x)_i / alpha for the flat indices ``idx`` only."""
    s, f, x = _f64(s), _f64(f), _f64(x)
    T, H, W = s.shape
    idx = np.ascontiguousarray(np.asarray(idx, dtype=np.int64))
    out = np.empty(idx.shape, dtype=np.float64)
    rc = _load().oracle_sfseg_apply_at(T, H, W, _dptr(s), _dptr(f), _dptr(x), float(alpha), k.sigma_s, k.sigma_t,
                                       k.r_s, k.r_t, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), idx.size,
                                       _dptr(out))
    if rc != 0:
        raise ValueError("oracle_sfseg_apply_at: invalid arguments or index out of range")
    return out


def sfseg_apply_conv(s, f, x, alpha: float, k: Kernel) -> np.ndarray:
    """Eq. 7 as written: S (1/alpha - F^2) G*(S X) - S G*(F^2 S X) + 2 S F G*(F S X),
    each G* a plain Gaussian filtering (``apply`` with a unit feature)."""
    s, f, x = _f64(s), _f64(f), _f64(x)
    one = np.ones_like(s)
    u = s * x
    g1 = apply(one, u, k)
    g2 = apply(one, f * f * u, k)
    g3 = apply(one, f * u, k)
    return s * (1.0 / alpha - f * f) * g1 - s * g2 + 2.0 * s * f * g3


def sfseg_iterate(s, f, alpha: float, k: Kernel, x0=None, iters: int | None = None, tol: float | None = None,
                  cap: int | None = None):
    """Power iteration with the full operator (Eq. 7 then the normalisation of
    Eq. 8), the same loop, start and stopping rule as ``iterate``."""
    return _power(lambda v: sfseg_apply(s, f, v, alpha, k), _f64(s).shape, x0, iters, tol, cap, False)


def sfseg_dense(s, f, alpha: float, k: Kernel) -> np.ndarray:
    """Explicit M / alpha (tiny volumes only), built pair by pair from Eq. 2."""
    s, f = _f64(s), _f64(f)
    T, H, W = s.shape
    N = s.size
    if N > 4096:
        raise ValueError("sfseg_dense is for tiny volumes")
    coords = [(t, y, x) for t in range(T) for y in range(H) for x in range(W)]
    sf, ff = s.reshape(-1), f.reshape(-1)
    M = np.zeros((N, N))
    for i, (ti, yi, xi) in enumerate(coords):
        for j, (tj, yj, xj) in enumerate(coords):
            dt, dy, dx = tj - ti, yj - yi, xj - xi
            if abs(dt) <= k.r_t and abs(dy) <= k.r_s and abs(dx) <= k.r_s:
                g = math.exp(-(dt * dt) / (2 * k.sigma_t ** 2) - (dy * dy + dx * dx) / (2 * k.sigma_s ** 2))
                M[i, j] = sf[i] * sf[j] * (1.0 - alpha * (ff[i] - ff[j]) ** 2) * g
    return M / alpha


def exp_apply(s, f, x, alpha: float, k: Kernel) -> np.ndarray:
    """z = E x with the exact pairwise affinity of Eq. 1,
    E_ij = s_i s_j exp(-alpha (f_i - f_j)^2) G_ij (direct loop, FP64)."""
    s, f, x = _f64(s), _f64(f), _f64(x)
    T, H, W = s.shape
    z = np.empty_like(s)
    rc = _load().oracle_exp_apply(T, H, W, _dptr(s), _dptr(f), _dptr(x), float(alpha), k.sigma_s, k.sigma_t,
                                  k.r_s, k.r_t, _dptr(z))
    if rc != 0:
        raise ValueError("oracle_exp_apply: invalid arguments")
    return z


def exp_dense(s, f, alpha: float, k: Kernel) -> np.ndarray:
    """Explicit E (tiny volumes only), built pair by pair from Eq. 1."""
    s, f = _f64(s), _f64(f)
    T, H, W = s.shape
    N = s.size
    if N > 4096:
        raise ValueError("exp_dense is for tiny volumes")
    coords = [(t, y, x) for t in range(T) for y in range(H) for x in range(W)]
    sf, ff = s.reshape(-1), f.reshape(-1)
    E = np.zeros((N, N))
    for i, (ti, yi, xi) in enumerate(coords):
        for j, (tj, yj, xj) in enumerate(coords):
            dt, dy, dx = tj - ti, yj - yi, xj - xi
            if abs(dt) <= k.r_t and abs(dy) <= k.r_s and abs(dx) <= k.r_s:
                E[i, j] = sf[i] * sf[j] * math.exp(-alpha * (ff[i] - ff[j]) ** 2 - (dt * dt) / (2 * k.sigma_t ** 2)
                                                   - (dy * dy + dx * dx) / (2 * k.sigma_s ** 2))
    return E


def exp_iterate(s, f, alpha: float, k: Kernel, x0=None, iters: int | None = None, tol: float | None = None,
                cap: int | None = None):
    """Power iteration with the exact affinity (the loop of ``iterate``)."""
    return _power(lambda v: exp_apply(s, f, v, alpha, k), _f64(s).shape, x0, iters, tol, cap, False)


def online_iterate(f, k: Kernel, q: int, shift: int, iters: int | None = None, tol: float | None = None,
                   cap: int | None = None):
    """Partial iterations over q-frame sub-windows (Sec. 4, "Online vs Offline
    processing"): windows start at frames 0, shift, 2 shift, ... (the last one
    ends at the last frame); a window's start vector takes the previous
    window's final solution on the frames the two share and the uniform value
    1/sqrt(q H W) on its new frames; each frame keeps the value of the last
    window that contains it. Returns (x, [IterInfo per window])."""
    f = _f64(f)
    T = f.shape[0]
    starts = list(range(0, T - q + 1, shift))
    if starts[-1] != T - q:
        starts.append(T - q)
    out = np.zeros_like(f)
    infos = []
    prev, prev_a = None, None
    c = 1.0 / math.sqrt(q * f.shape[1] * f.shape[2])
    for a in starts:
        x0 = np.full((q,) + f.shape[1:], c)
        if prev is not None:
            m = a - prev_a
            for t in range(q - m):
                x0[t] = prev[t + m]
        x, info = iterate(f[a:a + q], k, x0=x0, iters=iters, tol=tol, cap=cap)
        out[a:a + q] = x
        infos.append(info)
        prev, prev_a = x, a
    return out, infos


def dense_matrix(f, k: Kernel) -> np.ndarray:
    """Explicit adjacency (tiny volumes only): A_ij = f_i f_j G_ij, built pair by pair."""
    f = _f64(f)
    T, H, W = f.shape
    N = f.size
    if N > 4096:
        raise ValueError("dense_matrix is for tiny volumes")
    coords = [(t, y, x) for t in range(T) for y in range(H) for x in range(W)]
    flat = f.reshape(-1)
    A = np.zeros((N, N))
    for i, (ti, yi, xi) in enumerate(coords):
        for j, (tj, yj, xj) in enumerate(coords):
            dt, dy, dx = tj - ti, yj - yi, xj - xi
            if abs(dt) <= k.r_t and abs(dy) <= k.r_s and abs(dx) <= k.r_s:
                g = math.exp(-(dt * dt) / (2 * k.sigma_t ** 2) - (dy * dy + dx * dx) / (2 * k.sigma_s ** 2))
                A[i, j] = flat[i] * flat[j] * g
    return A


def perron(A: np.ndarray):
    """Principal eigenpair of a symmetric nonnegative matrix via numpy.linalg.eigh.

    The eigenvector's sign is fixed so that it sums to a nonnegative value
    (Perron-Frobenius: the principal eigenvector is nonnegative, Eq. 3).
    """
    w, V = np.linalg.eigh(A)
    v = V[:, -1]
    if v.sum() < 0:
        v = -v
    return float(w[-1]), v, w


# ---------------------------------------------------------------------------
# Channel combination (learned weights) and loss
# ---------------------------------------------------------------------------

def softmax(w) -> np.ndarray:
    w = _f64(w)
    e = np.exp(w - w.max())
    return e / e.sum()


def combine(fc, w) -> np.ndarray:
    """f = sum_c softmax(w)_c * fc[c]."""
    fc = _f64(fc)
    a = softmax(w)
    return np.tensordot(a, fc, axes=(0, 0))


def combine_bwd(fc, w, g_f) -> np.ndarray:
    """dL/dw from dL/df: g_a_c = <g_f, fc_c>, then the softmax Jacobian."""
    fc = _f64(fc)
    g_f = _f64(g_f)
    a = softmax(w)
    g_a = np.array([float(np.sum(g_f * fc[c])) for c in range(fc.shape[0])])
    return a * (g_a - float(np.dot(a, g_a)))


BCE_EPS = 1e-7


def bce(x, gt):
    """BCE(y, gt) with y = clip(x / max(x), eps, 1 - eps), mean over voxels.

    Returns (loss, dL/dx). The max term's derivative goes to the first argmax;
    clipped entries pass no gradient.
    """
    x = _f64(x)
    g = np.asarray(gt, dtype=np.float64)
    m = float(x.max())
    y_raw = x / m
    y = np.clip(y_raw, BCE_EPS, 1.0 - BCE_EPS)
    N = x.size
    loss = -float(np.mean(g * np.log(y) + (1.0 - g) * np.log(1.0 - y)))
    g_y = (y - g) / (y * (1.0 - y)) / N
    g_y = np.where((y_raw > BCE_EPS) & (y_raw < 1.0 - BCE_EPS), g_y, 0.0)
    g_x = g_y / m
    a = int(np.argmax(x.reshape(-1)))
    g_x.reshape(-1)[a] -= float(np.sum(g_y * x)) / (m * m)
    return loss, g_x


# ---------------------------------------------------------------------------
# Reverse mode through the normalised iteration
# ---------------------------------------------------------------------------

def forward_train(f, k: Kernel, iters: int, x0=None):
    """Run `iters` steps keeping everything the derivative needs.

    Per step (x_k unit): u = f x_k, v = G u, z = f v, n = ||z||, x_{k+1} = z / n.
    Returns dict(xs=[x_0..x_K], vs=[v_0..v_{K-1}], ns=[n_1..n_K]).
    """
    f = _f64(f)
    N = f.size
    x = np.full(f.shape, 1.0 / math.sqrt(N)) if x0 is None else _f64(x0) / np.linalg.norm(x0)
    xs, vs, ns = [x], [], []
    ones = np.ones_like(f)
    for _ in range(iters):
        # G u through the direct loop: A with unit features applied to u.
        v = apply(ones, f * x, k)
        z = f * v
        n = math.sqrt(float(np.sum(z * z)))
        x = z / n
        xs.append(x)
        vs.append(v)
        ns.append(n)
    return dict(xs=xs, vs=vs, ns=ns)


def adjoint(f, k: Kernel, tape, g_xK):
    """dL/df given dL/dx_K, by the chain rule through every step in reverse.

    For x_{k+1} = z / ||z||, z = f (G (f x_k)):
      g_z = (g - x_{k+1} <x_{k+1}, g>) / n
      g_f += v g_z ;  g_u = G (f g_z) ;  g_f += x_k g_u ;  g_{x_k} = f g_u
    x_0 is a constant (uniform start), so the chain stops there.
    """
    f = _f64(f)
    ones = np.ones_like(f)
    g = _f64(g_xK).copy()
    g_f = np.zeros_like(f)
    K = len(tape["ns"])
    for j in range(K - 1, -1, -1):
        x1 = tape["xs"][j + 1]
        x0 = tape["xs"][j]
        n = tape["ns"][j]
        v = tape["vs"][j]
        g_z = (g - x1 * float(np.sum(x1 * g))) / n
        g_f += v * g_z
        g_u = apply(ones, f * g_z, k)
        g_f += x0 * g_u
        g = f * g_u
    return g_f


def loss_and_grad(fc, w, gt, k: Kernel, iters: int):
    """End to end: f = combine(fc, w); x = iterate(f); L = bce(x, gt); dL/dw."""
    f = combine(fc, w)
    tape = forward_train(f, k, iters)
    loss, g_x = bce(tape["xs"][-1], gt)
    g_f = adjoint(f, k, tape, g_x)
    return loss, combine_bwd(fc, w, g_f), tape


# ---------------------------------------------------------------------------
# The paper's learning objective (SFSeg++): sigmoid-affine channel
# combination (Eq. 9), soft-binarised iterations after N_cont continuous ones
# (Alg. 1, step 3), Focal-Dice loss (Eq. 12)
# ---------------------------------------------------------------------------

def sigmoid(a):
    """The standard logistic 1 / (1 + exp(-a)) (Eq. 9 prints exp(+x): a sign slip)."""
    a = _f64(a)
    return 0.5 * (1.0 + np.tanh(0.5 * a))


def combine_sigmoid(fc, w, b: float) -> np.ndarray:
    """Eq. 9: f = sigmoid(sum_c w_c fc_c + b)."""
    fc = _f64(fc)
    w = np.asarray(w, dtype=np.float64)
    a = np.tensordot(w, fc, axes=(0, 0)) + b
    return sigmoid(a)


def combine_sigmoid_bwd(fc, w, b: float, g_f):
    """(dL/dw, dL/db) of Eq. 9 given dL/df: f' = f (1 - f)."""
    f = combine_sigmoid(fc, w, b)
    ga = _f64(g_f) * f * (1.0 - f)
    return np.tensordot(_f64(fc), ga, axes=([1, 2, 3], [0, 1, 2])), float(np.sum(ga))


def softbin(y, kappa: float, theta: float) -> np.ndarray:
    """Soft-binarisation of a unit iterate (Alg. 1, step 3, with the sigmoid's
    parameter made explicit): sigmoid(kappa (sqrt(N) y - theta))."""
    y = _f64(y)
    return sigmoid(kappa * (math.sqrt(y.size) * y - theta))


def focal_dice(x, gt, gamma: float = 0.75, eps: float = 1.0):
    """Eq. 12 per frame with the soft Dice 2 sum(x gt) / (sum x + sum gt),
    smoothed by eps: J = sum_t (1 - D_t)^gamma, D_t = (2 P_t + eps) / (X_t + Y_t + eps).
    Returns (J, dJ/dx)."""
    x = _f64(x)
    y = _f64(gt)
    P = np.sum(x * y, axis=(1, 2))
    X = np.sum(x, axis=(1, 2))
    Y = np.sum(y, axis=(1, 2))
    den = X + Y + eps
    D = (2.0 * P + eps) / den
    J = float(np.sum((1.0 - D) ** gamma))
    dJ_dD = -gamma * (1.0 - D) ** (gamma - 1.0)
    dD_dx = (2.0 * y * den[:, None, None] - (2.0 * P + eps)[:, None, None]) / (den ** 2)[:, None, None]
    return J, dJ_dD[:, None, None] * dD_dx


def forward_train_pp(f, k: Kernel, n_iter: int, n_cont: int, kappa: float, theta: float):
    """Alg. 1's loop on the single-field operator: every iteration applies A and
    normalises (y = A x / ||A x||); iterations after the first n_cont are then
    soft-binarised (x = softbin(y)). Returns dict(xs=[inputs x_0..x_K], ys=[y_1..y_K],
    ns=[||A x_k||], vs=[G (f x_k / ||x_k||)], soft=[bool per iteration]); xs[K] is the output."""
    f = _f64(f)
    N = f.size
    x = np.full(f.shape, 1.0 / math.sqrt(N))
    ones = np.ones_like(f)
    xs, ys, ns, vs, soft = [x], [], [], [], []
    for it in range(n_iter):
        xu = x / np.linalg.norm(x)
        v = apply(ones, f * xu, k)
        z = f * v
        n = math.sqrt(float(np.sum(z * z)))
        y = z / n
        sb = it >= n_cont
        x = softbin(y, kappa, theta) if sb else y
        xs.append(x)
        ys.append(y)
        ns.append(n)
        vs.append(v)
        soft.append(sb)
    return dict(xs=xs, ys=ys, ns=ns, vs=vs, soft=soft)


def adjoint_pp(f, k: Kernel, tape, kappa: float, g_out):
    """dL/df through forward_train_pp in reverse: the soft-binarisation
    (g_y = g_x sigmoid' kappa sqrt(N)), the normalisation of the step's output
    and of its input, and the step itself (as ``adjoint``)."""
    f = _f64(f)
    N = f.size
    ones = np.ones_like(f)
    g = _f64(g_out).copy()  # gradient w.r.t. xs[K]
    g_f = np.zeros_like(f)
    for j in range(len(tape["ns"]) - 1, -1, -1):
        x_out = tape["xs"][j + 1]
        if tape["soft"][j]:
            g = g * x_out * (1.0 - x_out) * kappa * math.sqrt(N)
        y = tape["ys"][j]
        g_z = (g - y * float(np.sum(y * g))) / tape["ns"][j]
        x_in = tape["xs"][j]
        nx = float(np.linalg.norm(x_in))
        xu = x_in / nx
        g_f += tape["vs"][j] * g_z
        g_u = apply(ones, f * g_z, k)
        g_f += xu * g_u
        g_xu = f * g_u
        g = (g_xu - xu * float(np.sum(xu * g_xu))) / nx
    return g_f


def loss_and_grad_pp(fc, w, b: float, gt, k: Kernel, n_iter: int, n_cont: int, kappa: float, theta: float,
                     gamma: float = 0.75):
    """End to end (SFSeg++ objective): f = combine_sigmoid(fc, w, b); Alg. 1's
    loop with soft-binarisation; Focal-Dice on the output. Returns (J, dJ/dw, dJ/db, tape)."""
    f = combine_sigmoid(fc, w, b)
    tape = forward_train_pp(f, k, n_iter, n_cont, kappa, theta)
    J, g_x = focal_dice(tape["xs"][-1], gt, gamma)
    g_f = adjoint_pp(f, k, tape, kappa, g_x)
    g_w, g_b = combine_sigmoid_bwd(fc, w, b, g_f)
    return J, g_w, g_b, tape


# ---------------------------------------------------------------------------
# Warm-start network (4 x conv3d 3x3x3, ReLU between layers)
# ---------------------------------------------------------------------------

def bf16_round(a) -> np.ndarray:
    """Round float values to bfloat16 (round to nearest, ties to even), returned as float64."""
    a32 = np.asarray(a, dtype=np.float32)
    bits = a32.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) >> 16) << 16
    nan = np.isnan(a32)
    out = rounded.astype(np.uint32).view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out


def conv3d(x, wgt, bias):
    """'same' 3x3x3 conv with zero padding. x [Cin][T][H][W], wgt [Cout][Cin][3][3][3]."""
    x = _f64(x)
    wgt = _f64(wgt)
    bias = _f64(bias)
    Cin, T, H, W = x.shape
    Cout = wgt.shape[0]
    assert wgt.shape == (Cout, Cin, 3, 3, 3)
    out = np.empty((Cout, T, H, W))
    rc = _load().oracle_conv3d_fwd(Cin, Cout, T, H, W, _dptr(x), _dptr(wgt), _dptr(bias), _dptr(out))
    if rc:
        raise ValueError("oracle_conv3d_fwd: bad arguments")
    return out


def conv3d_bwd(x, wgt, g_out, need_input_grad=True):
    x = _f64(x)
    wgt = _f64(wgt)
    g_out = _f64(g_out)
    Cin, T, H, W = x.shape
    Cout = wgt.shape[0]
    g_in = np.empty_like(x) if need_input_grad else None
    g_w = np.empty_like(wgt)
    g_b = np.empty(Cout)
    null = ctypes.POINTER(ctypes.c_double)()
    rc = _load().oracle_conv3d_bwd(Cin, Cout, T, H, W, _dptr(x), _dptr(wgt), _dptr(g_out),
                                   _dptr(g_in) if g_in is not None else null, _dptr(g_w), _dptr(g_b))
    if rc:
        raise ValueError("oracle_conv3d_bwd: bad arguments")
    return g_in, g_w, g_b


NET_CHANNELS = (1, 16, 16, 16, 1)


def net_forward(f, params, bf16: bool = False):
    """y = L4(relu(L3(relu(L2(relu(L1(f))))))); params = [(w1,b1),..,(w4,b4)].

    With bf16=True the weights and each layer's input activations are rounded
    to bfloat16 before the (FP64-accumulated) convolution, and the output is
    left unrounded. Returns (y [T][H][W], cache for net_backward).
    """
    h = _f64(f)[None]
    cache = []
    nl = len(params)
    for li, (w, b) in enumerate(params):
        hin = bf16_round(h) if bf16 else h
        wq = bf16_round(w) if bf16 else _f64(w)
        pre = conv3d(hin, wq, b)
        cache.append((hin, wq, pre))
        h = np.maximum(pre, 0.0) if li < nl - 1 else pre
    return h[0], cache


def net_backward(cache, g_y):
    """Gradients [(g_w, g_b)] of the loss w.r.t. each layer's (rounded) weights."""
    g = _f64(g_y)[None]
    grads = [None] * len(cache)
    for li in range(len(cache) - 1, -1, -1):
        hin, wq, pre = cache[li]
        if li < len(cache) - 1:
            g = g * (pre > 0)
        g_in, g_w, g_b = conv3d_bwd(hin, wq, g, need_input_grad=li > 0)
        grads[li] = (g_w, g_b)
        g = g_in
    return grads


def warm_start_x0(y, eps: float = 1e-6) -> np.ndarray:
    """Initial vector from the net output: normalize(max(y, 0) + eps)."""
    x = np.maximum(_f64(y), 0.0) + eps
    return x / np.linalg.norm(x)


def net_loss(y, x_star):
    """MSE between the net output and the target eigenvector scaled by sqrt(N)."""
    y = _f64(y)
    tgt = _f64(x_star) * math.sqrt(y.size)
    d = y - tgt
    return float(np.mean(d * d)), 2.0 * d / y.size


def adamw_step(w, g, m, v, vmax, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
               weight_decay=0.01, amsgrad=True):
    """AdamW (Eq. 13) with decoupled weight decay and AMSGrad; returns new (w, m, v, vmax).

    step is 1-based. Decay first (w <- w (1 - lr wd)), then the moment
    updates, bias corrections and w <- w - lr m_hat / (sqrt(v_hat) + eps).
    """
    w = _f64(w) * (1.0 - lr * weight_decay)
    g = _f64(g)
    m = beta1 * _f64(m) + (1.0 - beta1) * g
    v = beta2 * _f64(v) + (1.0 - beta2) * g * g
    vmax = np.maximum(_f64(vmax), v) if amsgrad else v
    m_hat = m / (1.0 - beta1 ** step)
    v_hat = vmax / (1.0 - beta2 ** step)
    w = w - lr * m_hat / (np.sqrt(v_hat) + eps)
    return w, m, v, vmax


def fallback(r1: float, r2: float) -> bool:
    """Warm-start fallback: restart from uniform when the residual rises (r2 > r1)."""
    return not (r2 <= r1)


def _coarse_size(n: int, s: int) -> int:
    return (n + s - 1) // s


def downsample(f, sy: int, st: int) -> np.ndarray:
    """Box average over sy x sy pixels and st frames; partial blocks at the
    far edges average the voxels that exist."""
    f = _f64(f)
    T, H, W = f.shape
    Tc, Hc, Wc = _coarse_size(T, st), _coarse_size(H, sy), _coarse_size(W, sy)
    out = np.empty((Tc, Hc, Wc))
    for tc in range(Tc):
        for yc in range(Hc):
            for xc in range(Wc):
                blk = f[tc * st:(tc + 1) * st, yc * sy:(yc + 1) * sy, xc * sy:(xc + 1) * sy]
                out[tc, yc, xc] = blk.sum() / blk.size
    return out


def _linear_axis(n_fine: int, s: int, n_coarse: int):
    """Cell-centred coordinate c = (i + 1/2) / s - 1/2 clamped to [0, n - 1]:
    lower index, upper index and weight of the upper one, per fine index."""
    i0 = np.empty(n_fine, dtype=np.int64)
    i1 = np.empty(n_fine, dtype=np.int64)
    w = np.empty(n_fine)
    for i in range(n_fine):
        c = min(max((i + 0.5) / s - 0.5, 0.0), n_coarse - 1.0)
        i0[i] = int(math.floor(c))
        i1[i] = min(i0[i] + 1, n_coarse - 1)
        w[i] = c - i0[i]
    return i0, i1, w


def upsample(xc, shape, sy: int, st: int, mode: int = 1, mul=None) -> np.ndarray:
    """Fine volume of the given shape from the coarse one: mode 0 takes the
    coarse cell holding each voxel, mode 1 interpolates trilinearly between
    cell centres (clamped at the edges). Multiplied by mul if given."""
    xc = _f64(xc)
    T, H, W = shape
    Tc, Hc, Wc = xc.shape
    if mode == 0:
        out = np.empty(shape)
        for t in range(T):
            for y in range(H):
                out[t, y, :] = xc[t // st, y // sy, np.arange(W) // sy]
    else:
        at0, at1, wt = _linear_axis(T, st, Tc)
        ay0, ay1, wy = _linear_axis(H, sy, Hc)
        ax0, ax1, wx = _linear_axis(W, sy, Wc)
        out = np.zeros(shape)
        for ti, tw in ((at0, 1.0 - wt), (at1, wt)):
            for yi, yw in ((ay0, 1.0 - wy), (ay1, wy)):
                for xi, xw in ((ax0, 1.0 - wx), (ax1, wx)):
                    out += (tw[:, None, None] * yw[None, :, None] * xw[None, None, :]) * \
                        xc[np.ix_(ti, yi, xi)]
    if mul is not None:
        out = out * _f64(mul)
    return out


def coarse_kernel(k: Kernel, sy: int, st: int) -> Kernel:
    """The filter on the coarse grid: sigmas and radii in coarse units (radii
    rounded up so the support covers the fine one)."""
    return Kernel(k.sigma_s / sy, k.sigma_t / st, -(-k.r_s // sy), -(-k.r_t // st))
