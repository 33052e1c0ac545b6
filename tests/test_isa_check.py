"""The build-time device-code checker recognises a barrier inside a loop that
lanes leave one by one (the shape that livelocks a persistent tile loop) and
accepts the same loop with a wave-uniform exit."""
import importlib.util
import os

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CHECKER = os.path.join(HERE, "..", "paper_2212_08058_amd", "isa_check.py")

LANE_EXIT = """_Z6kernelv:                              ; @_Z6kernelv
; %bb.0:
	s_branch .LBB0_2
.LBB0_1:                                ;   in Loop: Header=BB0_2 Depth=1
	s_andn2_b64 exec, exec, s[4:5]
	s_cbranch_execz .LBB0_3
.LBB0_2:                                ; =>This Loop Header: Depth=1
	s_barrier
	ds_read_b32 v0, v1
	s_branch .LBB0_1
.LBB0_3:
	s_endpgm
.Lfunc_end0:
"""

UNIFORM_EXIT = LANE_EXIT.replace("s_andn2_b64 exec, exec, s[4:5]\n\ts_cbranch_execz", "s_cmp_ge_i32 s6, s7\n\ts_cbranch_scc1")


@pytest.fixture(scope="module")
def checker():
    if not os.path.exists(CHECKER):
        pytest.skip("device-code checker not present in this tree")
    spec = importlib.util.spec_from_file_location("stpi_isa_check_test", CHECKER)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_flags_barrier_in_lane_divergent_loop(checker):
    assert checker._loops_with_barrier_and_lane_exit(LANE_EXIT) == [("_Z6kernelv", "BB0_2")]


def test_accepts_uniform_loop_exit(checker):
    assert checker._loops_with_barrier_and_lane_exit(UNIFORM_EXIT) == []


def test_accepts_lane_divergent_loop_without_barrier(checker):
    assert checker._loops_with_barrier_and_lane_exit(LANE_EXIT.replace("\ts_barrier\n", "")) == []
