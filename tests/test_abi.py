"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "stpi.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(stpi_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def native():
    from paper_2212_08058_amd import _native
    return _native


def test_every_declared_symbol_is_exported(native):
    syms = declared_symbols()
    assert len(syms) >= 6
    for s in syms:
        assert hasattr(native.lib, s), s
    # and the binding prototypes cover the header
    bound = {name for name, _, _ in native.PROTOTYPES}
    assert set(syms) <= bound, set(syms) - bound


def test_status_strings(native):
    for code in range(7):
        assert native.lib.stpi_status_string(code)
    assert native.lib.stpi_status_string(99) == b"unknown status"


def _prob(native, **kw):
    d = dict(T=8, H=64, W=112, sigma_s=2.0, sigma_t=1.0, r_s=4, r_t=2, dtype=0)
    d.update(kw)
    return native.Problem(d["T"], d["H"], d["W"], d["sigma_s"], d["sigma_t"], d["r_s"], d["r_t"], d["dtype"])


def test_workspace_bytes_and_validation(native):
    ws = native.lib.stpi_workspace_bytes(ctypes.byref(_prob(native)))
    assert ws >= 8 * 64 * 112 * 4
    bf = native.lib.stpi_workspace_bytes(ctypes.byref(_prob(native, dtype=1)))
    assert bf < ws
    for bad in (dict(T=0), dict(W=-1), dict(sigma_s=0.0), dict(sigma_t=float("nan")), dict(r_s=-1),
                dict(r_s=17), dict(r_t=9), dict(dtype=7)):
        assert native.lib.stpi_workspace_bytes(ctypes.byref(_prob(native, **bad))) == 0, bad


def test_invalid_calls_fail_before_any_launch(native):
    p = _prob(native)
    res = native.Result()
    # NULL buffers
    assert native.lib.stpi_step(ctypes.byref(p), None, None, 1.0, None, None, None, 0, None) == native.STPI_EINVAL
    assert b"NULL" in native.lib.stpi_last_error()
    rc = native.lib.stpi_iterate(ctypes.byref(p), 16, 32, 1, 10, 0.0, None, 0, ctypes.byref(res), None)
    assert rc == native.STPI_EWORKSPACE
    rc = native.lib.stpi_iterate(ctypes.byref(p), 16, 16, 1, 10, 0.0, 64, 1 << 30, ctypes.byref(res), None)
    assert rc == native.STPI_EINVAL   # x aliases f
    rc = native.lib.stpi_iterate(ctypes.byref(p), 16, 32, 3, 10, 0.0, 64, 1 << 30, ctypes.byref(res), None)
    assert rc == native.STPI_EINVAL   # bad init
    rc = native.lib.stpi_iterate(ctypes.byref(p), 16, 32, 1, -1, 0.0, 64, 1 << 30, ctypes.byref(res), None)
    assert rc == native.STPI_EINVAL   # negative count
    big = _prob(native, r_s=20)
    rc = native.lib.stpi_iterate(ctypes.byref(big), 16, 32, 1, 1, 0.0, 64, 1 << 30, ctypes.byref(res), None)
    assert rc == native.STPI_EUNSUPPORTED
    # the chain-step timer validates before touching the device
    ms, pf = ctypes.c_double(), ctypes.c_int()
    tc = native.lib.stpi_time_chain_step
    assert tc(ctypes.byref(p), None, 32, 64, 1 << 30, -1, 5, None, ctypes.byref(ms), None) == native.STPI_EINVAL
    assert tc(ctypes.byref(p), 16, 16, 64, 1 << 30, -1, 5, None, ctypes.byref(ms), None) == native.STPI_EINVAL
    assert tc(ctypes.byref(p), 16, 32, 64, 1 << 30, -1, 0, None, ctypes.byref(ms), ctypes.byref(pf)) == native.STPI_EINVAL
    assert tc(ctypes.byref(p), 16, 32, 64, 0, -1, 5, None, ctypes.byref(ms), None) == native.STPI_EWORKSPACE


def test_grid_transfer_rejects_bad_arguments(native):
    """stpi_downsample / stpi_upsample validate before any launch."""
    L = native.lib
    assert L.stpi_downsample(0, 4, 4, 2, 1, 0, 16, 32, None) == native.STPI_EINVAL      # empty volume
    assert L.stpi_downsample(4, 4, 4, 0, 1, 0, 16, 32, None) == native.STPI_EINVAL      # factor < 1
    assert L.stpi_downsample(4, 4, 4, 2, 1, 9, 16, 32, None) == native.STPI_EINVAL      # dtype
    assert L.stpi_downsample(4, 4, 4, 2, 1, 0, None, 32, None) == native.STPI_EINVAL    # NULL
    assert L.stpi_downsample(4, 4, 4, 2, 1, 0, 16, 16, None) == native.STPI_EINVAL      # alias
    assert L.stpi_upsample(4, 4, 4, 2, 1, 2, 0, 16, None, 32, None) == native.STPI_EINVAL  # mode
    assert L.stpi_upsample(4, 4, 4, 2, 1, 1, 0, 16, 32, 32, None) == native.STPI_EINVAL    # out aliases mul
    assert b"alias" in L.stpi_last_error()


def test_coarse_problem_host_only(native):
    """stpi_coarse_problem (host arithmetic, no device work): sizes rounded
    up, sigmas divided by the factors, radii rounded up, dtype kept; bad
    arguments rejected."""
    P = native.Problem
    fine = P(64, 480, 854, 5.0, 2.0, 15, 5, native.STPI_F32)
    c = P()
    assert native.lib.stpi_coarse_problem(ctypes.byref(fine), 4, 2, ctypes.byref(c)) == native.STPI_OK
    assert (c.T, c.H, c.W) == (32, 120, 214)
    assert (c.sigma_s, c.sigma_t, c.r_s, c.r_t, c.dtype) == (1.25, 1.0, 4, 3, native.STPI_F32)
    fine = P(5, 7, 9, 3.0, 1.5, 8, 3, native.STPI_BF16)
    assert native.lib.stpi_coarse_problem(ctypes.byref(fine), 3, 1, ctypes.byref(c)) == native.STPI_OK
    assert (c.T, c.H, c.W, c.r_s, c.r_t, c.dtype) == (5, 3, 3, 3, 3, native.STPI_BF16)
    assert c.sigma_s == 1.0 and c.sigma_t == 1.5
    for bad in (dict(sy=0), dict(st=0)):
        assert native.lib.stpi_coarse_problem(ctypes.byref(fine), bad.get("sy", 2), bad.get("st", 2),
                                              ctypes.byref(c)) == native.STPI_EINVAL
    assert native.lib.stpi_coarse_problem(None, 2, 2, ctypes.byref(c)) == native.STPI_EINVAL
    zero = P(0, 7, 9, 3.0, 1.5, 8, 3, native.STPI_F32)
    assert native.lib.stpi_coarse_problem(ctypes.byref(zero), 2, 2, ctypes.byref(c)) == native.STPI_EINVAL


def _walk_phases(T, RT, k):
    """Phases of the slowest of k frame segments: each segment stages RT frames
    beyond an inner boundary, the last one (starting after frame 0) walks
    backward so it has no epilogue-only ring steps at the clip's end, plus 2
    phases to fill the pipeline."""
    worst = 0
    for s in range(k):
        t0, t1 = s * T // k, (s + 1) * T // k
        ts, te = max(t0 - RT, 0), min(t1 + RT, T)
        n = (te - t0 if (t1 == T and t0 > 0) else t1 - ts) + RT + 2
        worst = max(worst, n)
    return worst


def test_short_clips_split_their_frames(native):
    """stpi_launch_shape (host logic): a clip whose tiles would leave most CUs
    idle splits its frames when that saves at least two phases of its slowest
    segment (a 16-frame window at 480 x 854, r = (15, 5): 15 phases against
    23 whole); a 3-frame clip stays whole; the full 64-frame clip keeps its
    two segments."""
    P = native.Problem
    info = (ctypes.c_int32 * 5)()
    cases = [((16, 480, 854), (5.0, 2.0, 15, 5), 2), ((64, 480, 854), (5.0, 2.0, 15, 5), 2),
             ((3, 45, 108), (4.0, 1.5, 8, 3), 1), ((4, 45, 108), (4.0, 1.5, 8, 3), 2)]
    for (T, H, W), (ss, st, rs, rt), want in cases:
        p = P(T, H, W, ss, st, rs, rt, native.STPI_F32)
        assert native.lib.stpi_launch_shape(ctypes.byref(p), -1, info) == native.STPI_OK
        variant, tiles, nseg = info[0], info[1], info[2]
        assert nseg == want, ((T, H, W), list(info))
        vi = (ctypes.c_int * 9)()
        assert native.lib.stpi_variant_info(native.STPI_F32, variant, vi) == native.STPI_OK
        RT = vi[1]
        if nseg > 1 and T < 4 * RT:
            # split only by the phase rule: it saves at least two phases
            assert _walk_phases(T, RT, nseg) + 1 < _walk_phases(T, RT, 1)
    assert _walk_phases(16, 5, 2) == 15 and _walk_phases(16, 5, 1) == 23
