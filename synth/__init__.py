"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module only draws inputs. It holds none of the method's arithmetic (no
Gaussian affinity, no iteration, no normalisation): both the HIP path and the
FP64 oracle receive the arrays it returns.

Workload recipe (stands in for the paper's DAVIS-2016 soft masks, which are
not available): soft segmentation masks in [0, 1] built from moving Gaussian
blobs, corrupted with the paper's additive uniform noise U[0, 0.1] and
salt-and-pepper noise (Sec. 5, noise models U / SP), at the paper's frame size
480x854 and clip lengths around the DAVIS average of ~69 frames.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "blob_clip",
    "channel_stack",
    "ClipSpec",
    "batch_specs",
    "CONFIGS",
]


def _blob_params(rng: np.random.Generator, nblobs: int, H: int, W: int):
    out = []
    for _ in range(nblobs):
        sigma = rng.uniform(6.0, 15.0)
        speed = rng.uniform(1.0, 3.0)
        angle = rng.uniform(0.0, 2.0 * math.pi)
        cy0 = rng.uniform(0.0, H)
        cx0 = rng.uniform(0.0, W)
        out.append((sigma, speed, angle, cy0, cx0))
    return out


def blob_mask(T: int, H: int, W: int, nblobs: int, seed: int):
    """Noise-free soft mask (float64, [T][H][W]) of linearly moving Gaussian blobs.

    Returns (mask, rng) so that callers keep drawing from the same stream.
    """
    rng = np.random.default_rng(seed)
    params = _blob_params(rng, nblobs, H, W)
    yy = np.arange(H, dtype=np.float64)
    xx = np.arange(W, dtype=np.float64)
    mask = np.zeros((T, H, W), dtype=np.float64)
    for t in range(T):
        m = mask[t]
        for sigma, speed, angle, cy0, cx0 in params:
            cy = cy0 + speed * math.sin(angle) * t
            cx = cx0 + speed * math.cos(angle) * t
            # isotropic Gaussian = product of its row and column profiles
            gy = np.exp(-((yy - cy) ** 2) / (2.0 * sigma * sigma))
            gx = np.exp(-((xx - cx) ** 2) / (2.0 * sigma * sigma))
            np.maximum(m, np.multiply.outer(gy, gx), out=m)
    return mask, rng


def blob_clip(T: int, H: int, W: int, nblobs: int, seed: int, noise: float = 0.1):
    """Return (f, gt): f float32 in [0, 1], gt bool mask (blob >= 0.5).

    f = clip(mask + U[0, noise), 0, 1), the noise drawn as one C-order
    float64 array from the same generator right after the blob parameters.
    """
    mask, rng = blob_mask(T, H, W, nblobs, seed)
    f = mask + rng.uniform(0.0, noise, size=(T, H, W))
    np.clip(f, 0.0, 1.0, out=f)
    return f.astype(np.float32), mask >= 0.5


def _disk(radius: int) -> np.ndarray:
    r = np.arange(-radius, radius + 1)
    return (r[:, None] ** 2 + r[None, :] ** 2) <= radius * radius


def channel_stack(C: int, T: int, H: int, W: int, seed: int, nblobs: int = 3):
    """C noisy, randomly dilated/eroded copies of one ground-truth blob mask.

    Returns (fc float32 [C][T][H][W], gt bool [T][H][W]). Channels 0..2 get
    additive U[0, 0.1] noise, the others 20% salt-and-pepper noise, then all
    are clipped to [0, 1].
    """
    from scipy import ndimage

    mask, rng = blob_mask(T, H, W, nblobs, seed)
    gt = mask >= 0.5
    fc = np.empty((C, T, H, W), dtype=np.float32)
    for c in range(C):
        ch = np.empty((T, H, W), dtype=np.float64)
        for t in range(T):
            radius = int(rng.integers(1, 5))
            if rng.uniform() < 0.5:
                m = ndimage.binary_dilation(gt[t], structure=_disk(radius))
            else:
                m = ndimage.binary_erosion(gt[t], structure=_disk(radius))
            ch[t] = m
        if c < 3:
            ch += rng.uniform(0.0, 0.1, size=ch.shape)
        else:
            hit = rng.uniform(size=ch.shape) < 0.2
            salt = rng.uniform(size=ch.shape) < 0.5
            ch[hit] = salt[hit].astype(np.float64)
        np.clip(ch, 0.0, 1.0, out=ch)
        fc[c] = ch
    return fc, gt


@dataclasses.dataclass(frozen=True)
class ClipSpec:
    T: int
    H: int
    W: int
    seed: int
    nblobs: int = 3


def batch_specs(n: int = 48, seed: int = 3000, t_range=(8, 96),
                sizes=((240, 432), (360, 640), (480, 854))) -> list[ClipSpec]:
    """Uneven batch: T ~ U{t_range}, (H, W) uniform over `sizes`; clip i seeded seed+i."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        T = int(rng.integers(t_range[0], t_range[1] + 1))
        H, W = sizes[int(rng.integers(0, len(sizes)))]
        out.append(ClipSpec(T, H, W, seed + i))
    return out


# Named workloads. Kernel radii/sigmas: the single-clip and channel workloads
# use sigma_s=2, sigma_t=1, r_s=4, r_t=2; the full-resolution one sigma_s=5,
# sigma_t=2, r_s=15, r_t=5; the batched and warm-start ones r_s=8, r_t=3 with
# sigma = r/2 (sigma_s=4, sigma_t=1.5).
CONFIGS = {
    "small": dict(T=8, H=64, W=112, nblobs=3, seed=0, sigma_s=2.0, sigma_t=1.0, r_s=4, r_t=2, iters=10),
    "full": dict(T=64, H=480, W=854, nblobs=5, seed=1, sigma_s=5.0, sigma_t=2.0, r_s=15, r_t=5, iters=20),
    "channels": dict(C=8, T=32, H=240, W=432, seed=2, sigma_s=2.0, sigma_t=1.0, r_s=4, r_t=2, iters=15, ckpt=5),
    "batch": dict(n=48, seed=3000, sigma_s=4.0, sigma_t=1.5, r_s=8, r_t=3, tol=1e-4, cap=50),
    "warm": dict(train_n=2000, train_T=16, train_H=240, train_W=432, train_seed=40000,
                 eval_n=200, eval_T=32, eval_H=480, eval_W=854, eval_seed=50000,
                 sigma_s=4.0, sigma_t=1.5, r_s=8, r_t=3, tol=1e-4),
}
