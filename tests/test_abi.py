"""CPU checks of the C ABI: the library loads, exports every entry point
that include/rtg.h declares, and its host-side plan logic (sizes, layout,
argument checks) works without touching a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rtg.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(rtg_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_2404_19706_amd._lib import LIB_PATH, lib
    if not os.path.exists(LIB_PATH):
        pytest.fail("librtg.so not built: run __graft_entry__.build()")
    return lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    from paper_2404_19706_amd._lib import SIGNATURES
    assert sorted(s[0] for s in SIGNATURES) == names


def test_plan_sizes_and_layout(L):
    from paper_2404_19706_amd._lib import Intrinsics, default_config, RTG_OK
    cfg = default_config()
    assert (cfg.tile_w, cfg.tile_h, cfg.cutoff2, cfg.z_near) == (16, 16, 9.0, pytest.approx(0.2))
    assert (cfg.fwd_items_per_pop, cfg.fwd_static_share) == (-1, -1)
    intr = Intrinsics(525.0, 525.0, 320.0, 240.0, 640, 480)
    plan = ctypes.c_void_p()
    assert L.rtg_plan_create(ctypes.byref(cfg), ctypes.byref(intr), 100000, 2, 1 << 20, ctypes.byref(plan)) == RTG_OK
    nbytes = L.rtg_plan_workspace_bytes(plan)
    slots = 2 * 100000
    assert nbytes >= slots * (48 + 16 + 4 + 8 + 64) + 20 * (1 << 20)
    lay = (ctypes.c_int64 * 10)()
    assert L.rtg_plan_layout(plan, lay, 10) == 10
    offs = list(lay)
    assert all(o % 256 == 0 for o in offs) and len(set(offs)) == 10
    assert max(offs) < nbytes
    L.rtg_plan_destroy(plan)


@pytest.mark.parametrize("kw", [dict(tile_w=12, tile_h=12), dict(cutoff2=0.0), dict(items_per_pop=-1), dict(items_per_pop=2000),
                                dict(sort_cap=10 ** 6), dict(t_eps=-1.0), dict(stage_cap=-1), dict(stage_cap=4001),
                                dict(fwd_items_per_pop=-2), dict(fwd_items_per_pop=2000), dict(fwd_static_share=-2),
                                dict(fwd_static_share=101)])
def test_plan_rejects_bad_config(L, kw):
    from paper_2404_19706_amd._lib import Intrinsics, default_config, RTG_E_INVALID
    cfg = default_config(**kw)
    intr = Intrinsics(100.0, 100.0, 64.0, 48.0, 128, 96)
    plan = ctypes.c_void_p()
    assert L.rtg_plan_create(ctypes.byref(cfg), ctypes.byref(intr), 10, 1, 1000, ctypes.byref(plan)) == RTG_E_INVALID


@pytest.mark.parametrize("args", [(10, 0, 1000), (10, 33, 1000), (-1, 1, 1000), (10, 1, 0),
                                  (1 << 28, 32, 1000), (10, 1, 1 << 31), (1 << 30, 1, 1000)])
def test_plan_rejects_bad_sizes(L, args):
    from paper_2404_19706_amd._lib import Intrinsics, default_config, RTG_E_INVALID
    cfg = default_config()
    intr = Intrinsics(100.0, 100.0, 64.0, 48.0, 128, 96)
    plan = ctypes.c_void_p()
    n, f, mp = args
    assert L.rtg_plan_create(ctypes.byref(cfg), ctypes.byref(intr), n, f, mp, ctypes.byref(plan)) == RTG_E_INVALID


def test_bad_intrinsics_and_null_workspace(L):
    from paper_2404_19706_amd._lib import Intrinsics, default_config, RTG_E_INVALID, RTG_OK
    cfg = default_config()
    plan = ctypes.c_void_p()
    for intr in (Intrinsics(0.0, 100.0, 64.0, 48.0, 128, 96), Intrinsics(100.0, 100.0, 64.0, 48.0, 0, 96),
                 Intrinsics(float("nan"), 100.0, 64.0, 48.0, 128, 96)):
        assert L.rtg_plan_create(ctypes.byref(cfg), ctypes.byref(intr), 10, 1, 1000, ctypes.byref(plan)) == RTG_E_INVALID
    intr = Intrinsics(100.0, 100.0, 64.0, 48.0, 128, 96)
    assert L.rtg_plan_create(ctypes.byref(cfg), ctypes.byref(intr), 10, 1, 1000, ctypes.byref(plan)) == RTG_OK
    # NULL / misaligned workspace is rejected before anything is enqueued
    assert L.rtg_bin(plan, None, None, None) == RTG_E_INVALID
    assert L.rtg_project(plan, ctypes.c_void_p(8), *([None] * 8)) == RTG_E_INVALID
    assert L.rtg_read_status(plan, None, None, None) == RTG_E_INVALID
    assert L.rtg_backward_raster_l1(plan, None, *([None] * 7)) == RTG_E_INVALID
    # the L1 projection backward rejects a null loss output and a null workspace
    assert L.rtg_backward_project_l1(plan, ctypes.c_void_p(256), *([None] * 6), 1.0, 1.0,
                                     *([None] * 7)) == RTG_E_INVALID
    assert L.rtg_backward_project_l1(plan, None, *([None] * 6), 1.0, 1.0, *([None] * 5),
                                     ctypes.c_void_p(256), None) == RTG_E_INVALID
    assert L.rtg_status_string(-2) == b"pair capacity exceeded"
    assert b"gfx950" in L.rtg_version()
    L.rtg_plan_destroy(plan)


def test_static_forward_rejects_plans_beyond_its_scratch(L):
    """rtg_forward_static checks the plan's workspace against the fixed
    scratch before it touches any device (here: pair capacity of 2^30)."""
    from paper_2404_19706_amd._lib import (Intrinsics, default_config, RTG_E_INVALID, RTG_E_TOO_LARGE, RTG_OK,
                                           STATIC_SCRATCH_BYTES)
    cfg = default_config()
    intr = Intrinsics(100.0, 100.0, 64.0, 48.0, 128, 96)
    plan = ctypes.c_void_p()
    assert L.rtg_plan_create(ctypes.byref(cfg), ctypes.byref(intr), 1000, 1, 1 << 30, ctypes.byref(plan)) == RTG_OK
    assert L.rtg_plan_workspace_bytes(plan) > STATIC_SCRATCH_BYTES
    dummy = [ctypes.c_void_p(256)] * 13
    assert L.rtg_forward_static(plan, *dummy, None) == RTG_E_TOO_LARGE
    assert L.rtg_status_string(RTG_E_TOO_LARGE).startswith(b"plan workspace exceeds")
    L.rtg_plan_destroy(plan)
    assert L.rtg_forward_static(None, *dummy, None) == RTG_E_INVALID


def test_mapping_iteration_calls_check_their_arguments(L):
    from paper_2404_19706_amd._lib import RTG_E_INVALID
    assert L.rtg_select_workspace_bytes(0, 10, 10) == 0
    assert L.rtg_select_workspace_bytes(2, 10, 10) >= 2 * 10 * 10 * 4 + 2 * 256 * 4
    ws = ctypes.c_void_p(256)
    p = ctypes.c_void_p(512)
    # frac outside [0, 1], a misaligned or short workspace, a null buffer
    assert L.rtg_select_top_error(1, 8, 8, 1.5, p, p, p, ws, 1 << 20, None) == RTG_E_INVALID
    assert L.rtg_select_top_error(1, 8, 8, 0.4, p, p, p, ctypes.c_void_p(8), 1 << 20, None) == RTG_E_INVALID
    assert L.rtg_select_top_error(1, 8, 8, 0.4, p, p, p, ws, 16, None) == RTG_E_INVALID
    assert L.rtg_select_top_error(1, 8, 8, 0.4, p, None, p, ws, 1 << 20, None) == RTG_E_INVALID
    assert L.rtg_fuse(10, 0, *([p] * 10), None) == RTG_E_INVALID
    assert L.rtg_fuse(10, 49, *([p] * 10), None) == RTG_E_INVALID
    assert L.rtg_reg_l2(10, 1000.0, *([p] * 11), None, None) == RTG_E_INVALID
    assert L.rtg_reg_l2(-1, 1000.0, *([p] * 12), None) == RTG_E_INVALID
    assert L.rtg_confidence_count(10, 0, p, p, p, None) == RTG_E_INVALID
