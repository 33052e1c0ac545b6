"""Seeded input generators: determinism, shapes and value ranges."""
import numpy as np

import synth


def test_blob_clip_deterministic_and_in_range():
    f1, g1 = synth.blob_clip(4, 32, 48, 3, seed=5)
    f2, g2 = synth.blob_clip(4, 32, 48, 3, seed=5)
    f3, _ = synth.blob_clip(4, 32, 48, 3, seed=6)
    assert f1.dtype == np.float32 and f1.shape == (4, 32, 48)
    assert f1.tobytes() == f2.tobytes() and np.array_equal(g1, g2)
    assert not np.array_equal(f1, f3)
    assert f1.min() >= 0.0 and f1.max() <= 1.0
    # additive U[0, 0.1] noise keeps every feature strictly positive almost surely
    assert f1.min() > 0.0


def test_blob_clip_small_workload_shape():
    c = synth.CONFIGS["small"]
    f, gt = synth.blob_clip(c["T"], c["H"], c["W"], c["nblobs"], c["seed"])
    assert f.shape == (8, 64, 112) and gt.shape == f.shape and gt.dtype == bool


def test_channel_stack():
    fc, gt = synth.channel_stack(8, 3, 40, 56, seed=2)
    fc2, _ = synth.channel_stack(8, 3, 40, 56, seed=2)
    assert fc.shape == (8, 3, 40, 56) and fc.tobytes() == fc2.tobytes()
    assert fc.min() >= 0 and fc.max() <= 1
    # salt-and-pepper channels contain exact zeros and ones, the uniform-noise ones do not hit 0
    assert (fc[3:] == 0).any() and (fc[3:] == 1).any()
    assert fc[:3].min() >= 0.0


def test_batch_specs():
    specs = synth.batch_specs()
    assert len(specs) == 48
    assert all(8 <= s.T <= 96 for s in specs)
    assert {(s.H, s.W) for s in specs} <= {(240, 432), (360, 640), (480, 854)}
    assert specs == synth.batch_specs()
