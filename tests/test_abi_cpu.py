"""The C ABI library loads and exports every symbol ``include/gs.h`` declares,
and its host-side argument checks reject bad calls before touching a device
(so these run without a GPU).  No compute call is made here."""
import ctypes
import os
import re

import pytest

from paper_2503_18402_amd import gsmi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not gsmi.is_available():
        from paper_2503_18402_amd import build
        build.build()
    return gsmi.lib()


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "gs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    syms = declared_symbols()
    assert len(syms) >= 12
    for s in syms:
        assert hasattr(L, s), s
    # and the binding exposes the same names
    for s in syms:
        assert hasattr(gsmi, s), s


def test_version_and_status_strings(L):
    assert gsmi.gs_version() == 1
    assert gsmi.gs_status_str(0) == "ok"
    assert "argument" in gsmi.gs_status_str(1)


def _cam(w=64, h=48):
    from paper_2503_18402_amd import scenes
    return scenes.look_at((0, 0, -3), (0, 0, 0), w, h, 60.0)


def test_sizes(L):
    assert gsmi.gs_proj_bytes(1, 0) >= 0
    assert gsmi.gs_proj_bytes(2, 1000) >= 2 * 56 * 1000
    assert gsmi.gs_proj_bytes(0, 10) == 0
    assert gsmi.gs_proj_bytes(33, 10) == 0
    cams = gsmi.make_cameras([_cam(64, 48), _cam(20, 9)])
    assert gsmi.gs_total_tiles(cams, gsmi.make_cfg(16)) == 4 * 3 + 2 * 1
    assert gsmi.gs_total_tiles(cams, gsmi.make_cfg(8)) == 8 * 6 + 3 * 2
    assert gsmi.gs_total_tiles(cams, gsmi.make_cfg(12)) == -1
    assert gsmi.gs_bin_sort_workspace_bytes(1, 100, 1000) > 0
    assert gsmi.gs_bin_sort_workspace_bytes(1, 100, -1) == 0
    assert gsmi.gs_render_bwd_workspace_bytes(1, 100, 1000) >= 9 * 4 * 1000


def _call_pre(L, n_views, cams, cfg, n, sh_degree, ptr=16):
    return L.gs_preprocess(n_views, cams, ctypes.byref(cfg), n, ptr, ptr, ptr, ptr, ptr,
                           sh_degree, ptr, None)


def test_argument_errors(L):
    cams = gsmi.make_cameras([_cam()])
    good = gsmi.make_cfg(16, 256)
    # bad tile, bad batch, bad degree, bad n, null pointers: GS_ERR_ARG, nothing enqueued
    assert _call_pre(L, 1, cams, gsmi.make_cfg(12, 256), 10, 3) == 1
    assert _call_pre(L, 1, cams, gsmi.make_cfg(16, 100), 10, 3) == 1
    assert _call_pre(L, 1, cams, good, 10, 4) == 1
    assert _call_pre(L, 1, cams, good, -1, 3) == 1
    assert _call_pre(L, 0, cams, good, 10, 3) == 1
    assert L.gs_preprocess(1, cams, ctypes.byref(good), 10, None, 16, 16, 16, 16, 3, 16, None) == 1
    # misaligned quaternions
    assert L.gs_preprocess(1, cams, ctypes.byref(good), 10, 16, 16, 20, 16, 16, 3, 16, None) == 1
    bad = gsmi.make_cameras([_cam(0, 10)])
    assert _call_pre(L, 1, bad, good, 10, 3) == 1
    cams_near = gsmi.make_cameras([_cam()])
    cams_near[0].near_plane = 0.0
    assert _call_pre(L, 1, cams_near, good, 10, 3) == 1
    # workspace too small -> GS_ERR_CAPACITY
    need = gsmi.gs_bin_sort_workspace_bytes(1, 10, 100)
    assert L.gs_bin_sort(1, cams, ctypes.byref(good), 10, 16, 100, 256, need - 1, None, 16, 16,
                         16, None) == 2
    # the no-allocation binning: capacity or items beyond its array -> GS_ERR_CAPACITY,
    # a negative capacity -> GS_ERR_ARG (checked before anything touches a device)
    mx = gsmi.GS_BIN_SORT_NOALLOC_MAX_PAIRS
    assert L.gs_bin_sort_noalloc(1, cams, ctypes.byref(good), 10, 16, mx + 1, None, 16, 16, 16,
                                 None) == 2
    assert L.gs_bin_sort_noalloc(1, cams, ctypes.byref(good), gsmi.GS_BIN_SORT_NOALLOC_MAX_ITEMS
                                 + 1, 16, 100, None, 16, 16, 16, None) == 2
    assert L.gs_bin_sort_noalloc(1, cams, ctypes.byref(good), 10, 16, -1, None, 16, 16, 16,
                                 None) == 1
    # adam: step 0, too many groups, bad beta
    grp = (gsmi.GsAdamGroup * 1)()
    grp[0].numel = 0
    assert L.gs_adam_step(grp, 1, 0, 0.9, 0.999, 1e-15, None) == 1
    assert L.gs_adam_step(grp, 9, 1, 0.9, 0.999, 1e-15, None) == 1
    assert L.gs_adam_step(grp, 1, 1, 1.0, 0.999, 1e-15, None) == 1
    assert L.gs_l1_loss_grad(-1, 16, 16, 1.0, 16, None, None) == 1
    # forward with the L1 gradient: a null target or gradient, a bad tile
    assert L.gs_render_fwd_l1(1, cams, ctypes.byref(good), 10, 256, 256, 256, 256, 256, 256,
                              None, 1.0, 256, None, None) == 1
    assert L.gs_render_fwd_l1(1, cams, ctypes.byref(good), 10, 256, 256, 256, 256, 256, 256,
                              256, 1.0, None, None, None) == 1
    assert L.gs_render_fwd_l1(1, cams, ctypes.byref(gsmi.make_cfg(12, 256)), 10, 256, 256, 256,
                              256, 256, 256, 256, 1.0, 256, None, None) == 1
    # fused backward + Adam: null moment table, a null moment, bad beta, misaligned SH moments
    ptrs = (ctypes.c_void_p * 5)(*([256] * 5))
    lrs = (ctypes.c_float * 6)(*([1e-3] * 6))
    ws_need = gsmi.gs_render_bwd_workspace_bytes(1, 10, 100)
    for entry in (L.gs_render_bwd_adam, L.gs_render_bwd_sparse_adam):
        def fused(m, v, b1=0.9, ws_bytes=ws_need):
            return entry(1, cams, ctypes.byref(good), 10, 256, 256, 256, 256, 256, 3,
                         256, 256, 256, 256, 256, 256, m, v, lrs, 256, b1, 0.999,
                         1e-15, None, 100, 256, ws_bytes, None)
        assert fused(None, ptrs) == 1
        nul = (ctypes.c_void_p * 5)(256, 256, 256, None, 256)
        assert fused(nul, ptrs) == 1
        assert fused(ptrs, ptrs, b1=1.0) == 1
        mis = (ctypes.c_void_p * 5)(256, 256, 256, 256, 260)
        assert fused(ptrs, mis) == 1
        assert fused(ptrs, ptrs, ws_bytes=ws_need - 1) == 2


def test_header_mentions_every_entry_point_in_binding():
    text = open(os.path.join(ROOT, "include", "gs.h")).read()
    for name in ("gs_preprocess", "gs_bin_sort", "gs_render_fwd", "gs_render_bwd", "gs_adam_step"):
        assert name in text
