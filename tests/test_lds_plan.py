"""The hop kernel's LDS planner on the CPU (host arithmetic only): requests
that a compute unit cannot hold are refused before any dispatch, and an
accepted wave cap admits exactly the intended number of resident blocks."""
import ctypes

import pytest

KIB = 1024
UNIT = 2560


@pytest.fixture(scope="module")
def plan():
    from paper_1311_4462_amd import _lib
    L = _lib.lib()

    def f(bs, wcap, staging, cu, blk, static):
        out = ctypes.c_uint(0)
        rc = L.tm_plan_hop_lds(bs, wcap, staging, cu, blk, static, ctypes.byref(out))
        return rc, out.value
    return f


def test_no_cap_no_staging_asks_nothing(plan):
    assert plan(256, 0, 0, 160 * KIB, 160 * KIB, 32) == (0, 0)


@pytest.mark.parametrize("bs", [64, 128, 256])
@pytest.mark.parametrize("wcap", [1, 2, 3, 4])
@pytest.mark.parametrize("static", [0, 8, 32, 1000])
def test_wave_cap_admits_exactly_its_blocks(plan, bs, wcap, static):
    cu = 160 * KIB
    rc, dyn = plan(bs, wcap, 0, cu, cu, static)
    assert rc == 0
    foot = dyn + static
    assert foot % UNIT == 0                      # no rounding up at dispatch
    assert foot <= cu                            # never beyond the compute unit
    blocks = max(1, 4 * wcap * 64 // bs)
    assert cu // foot == blocks                  # exactly `blocks` resident blocks


def test_whole_compute_unit_block_keeps_room_for_static_lds(plan):
    # the case that once asked for 160 KiB of dynamic LDS on top of the
    # kernel's static LDS: one 256-thread block per compute unit
    rc, dyn = plan(256, 1, 0, 160 * KIB, 160 * KIB, 48)
    assert rc == 0 and dyn + 48 <= 160 * KIB


def test_refusals(plan):
    cu = 160 * KIB
    # staging beyond what one block may use
    assert plan(256, 0, cu, cu, cu, 16)[0] == -9
    assert plan(256, 0, 65 * KIB, cu, 64 * KIB, 0)[0] == -9
    # a per-block limit below the footprint the cap needs: one resident
    # block per compute unit cannot be expressed when a block may use at most
    # 64 KiB (two such blocks fit)
    assert plan(256, 1, 0, cu, 64 * KIB, 0)[0] == -9
    # while two blocks of at most 64 KiB each can
    rc, dyn = plan(256, 2, 0, cu, 64 * KIB, 0)
    assert rc == 0 and cu // dyn == 2
    # static LDS larger than the footprint of the cap
    assert plan(64, 4, 0, cu, cu, 11 * KIB)[0] == -9
    # bad arguments
    assert plan(100, 1, 0, cu, cu, 0)[0] == -1
    assert plan(256, 9, 0, cu, cu, 0)[0] == -1
    assert plan(256, 1, 0, 0, cu, 0)[0] == -1
    from paper_1311_4462_amd import _lib
    assert _lib.lib().tm_plan_hop_lds(256, 1, 0, cu, cu, 0, None) == -1


def test_staging_and_cap_take_the_larger(plan):
    cu = 160 * KIB
    rc, dyn = plan(256, 4, 50 * KIB, cu, cu, 0)     # cap wants 40 KiB, staging 50 KiB
    assert rc == 0 and dyn == 50 * KIB
