"""Thin ctypes binding of ``include/gs.h``: same names, argument marshalling only.

Every function here converts torch tensors to device pointers, calls the C
entry point of ``libgsmi.so`` on the current HIP stream and raises
``GsError`` on a non-OK status.  All arithmetic runs in the HIP kernels; if
the library is missing this module raises instead of falling back.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_float, c_int32, c_int64, c_size_t, c_uint32, c_uint64, c_void_p

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgsmi.so")

GS_MAX_VIEWS = 32
GS_MAX_ADAM_GROUPS = 8
STATUS = {0: "GS_OK", 1: "GS_ERR_ARG", 2: "GS_ERR_CAPACITY", 3: "GS_ERR_DEVICE",
          4: "GS_ERR_UNSUPPORTED"}


class GsError(RuntimeError):
    def __init__(self, fn: str, status: int):
        super().__init__(f"{fn} returned {STATUS.get(status, status)}")
        self.status = status


class GsCamera(ctypes.Structure):
    _fields_ = [("R", c_float * 9), ("t", c_float * 3), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("width", c_int32), ("height", c_int32),
                ("near_plane", c_float)]


class GsRasterCfg(ctypes.Structure):
    _fields_ = [("tile", c_int32), ("lds_batch", c_int32), ("bg", c_float * 3),
                ("mip2d", c_int32), ("filter3d", c_void_p), ("cam_table", c_void_p),
                ("cam_index", c_void_p), ("adam_lr", c_void_p)]


class GsKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", c_int64), ("total_ms", ctypes.c_double)]


class GsAdamGroup(ctypes.Structure):
    _fields_ = [("p", c_void_p), ("g", c_void_p), ("m", c_void_p), ("v", c_void_p),
                ("numel", c_int64), ("lr", c_float)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libgsmi.so (built by ``__graft_entry__.build()``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_2503_18402_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, sz = c_void_p, c_int32, c_int64, c_size_t
        cam_p, cfg_p = POINTER(GsCamera), POINTER(GsRasterCfg)
        sig = {
            "gs_version": (i32, []),
            "gs_status_str": (ctypes.c_char_p, [i32]),
            "gs_proj_bytes": (sz, [i32, i32]),
            "gs_total_tiles": (i64, [i32, cam_p, cfg_p]),
            "gs_preprocess": (i32, [i32, cam_p, cfg_p, i32, vp, vp, vp, vp, vp, i32, vp, vp]),
            "gs_bin_sort_workspace_bytes": (sz, [i32, i32, i64]),
            "gs_bin_sort": (i32, [i32, cam_p, cfg_p, i32, vp, i64, vp, sz, vp, vp, vp, vp, vp]),
            "gs_bin_sort_noalloc": (i32, [i32, cam_p, cfg_p, i32, vp, i64, vp, vp, vp, vp, vp]),
            "gs_spatial_order_workspace_bytes": (sz, [i32]),
            "gs_spatial_order": (i32, [i32, vp, vp, sz, vp, vp]),
            "gs_gather_rows": (i32, [i32, vp, i32, vp, vp, vp, vp]),
            "gs_bin_sort_radix_workspace_bytes": (sz, [i32, i32, i64]),
            "gs_bin_sort_radix": (i32, [i32, cam_p, cfg_p, i32, vp, i64, vp, sz, vp, vp, vp, vp,
                                        vp]),
            "gs_render_fwd": (i32, [i32, cam_p, cfg_p, i32, vp, vp, vp, vp, vp, vp, vp]),
            "gs_render_fwd_l1": (i32, [i32, cam_p, cfg_p, i32, vp, vp, vp, vp, vp, vp, vp,
                                       c_float, vp, vp, vp]),
            "gs_render_bwd_workspace_bytes": (sz, [i32, i32, i64]),
            "gs_render_bwd": (i32, [i32, cam_p, cfg_p, i32, vp, vp, vp, vp, vp, i32, vp, vp, vp,
                                    vp, vp, vp, vp, vp, vp, vp, vp, vp, i32, i64, vp, sz, vp]),
            "gs_adam_step": (i32, [POINTER(GsAdamGroup), i32, i32, c_float, c_float, c_float, vp]),
            "gs_adam_step_device": (i32, [POINTER(GsAdamGroup), i32, vp, c_float, c_float,
                                          c_float, vp]),
            "gs_render_bwd_adam": (i32, [i32, cam_p, cfg_p, i32, vp, vp, vp, vp, vp, i32, vp,
                                         vp, vp, vp, vp, vp, POINTER(c_void_p),
                                         POINTER(c_void_p), POINTER(c_float), vp, c_float,
                                         c_float, c_float, vp, i64, vp, sz, vp]),
            "gs_render_bwd_sparse_adam": (i32, [i32, cam_p, cfg_p, i32, vp, vp, vp, vp, vp, i32,
                                                vp, vp, vp, vp, vp, vp, POINTER(c_void_p),
                                                POINTER(c_void_p), POINTER(c_float), vp, c_float,
                                                c_float, c_float, vp, i64, vp, sz, vp]),
            "gs_filter3d_variance": (i32, [i32, cam_p, i32, vp, c_float, vp, vp, vp]),
            "gs_frequency_map_workspace_bytes": (sz, [i32, i32]),
            "gs_frequency_map": (i32, [i32, i32, i32, vp, vp, vp, sz, vp]),
            "gs_resolution_schedule": (i32, [POINTER(c_double), i32, i32, c_double, c_double, i32,
                                             c_double, i32, POINTER(c_double), POINTER(c_double)]),
            "gs_schedule_resolution": (c_double, [c_double, i32, POINTER(c_double),
                                                  POINTER(c_double)]),
            "gs_downsample_aa": (i32, [i32, i32, i32, i32, i32, vp, vp, vp]),
            "gs_primitive_target": (c_double, [c_double, c_double, c_double, c_double,
                                               c_double]),
            "gs_primitive_budget": (c_double, [c_double, c_double, c_double, c_double]),
            "gs_densify_workspace_bytes": (sz, [i32]),
            "gs_densify_stats": (i32, [i32, i32, vp, vp, c_float, vp, vp, vp]),
            "gs_densify_classify": (i32, [i32, vp, vp, vp, c_float, c_float, vp, sz, vp, vp]),
            "gs_densify_plan": (i32, [i32, i64, i64, vp, c_float, vp, sz, vp, vp]),
            "gs_densify_apply": (i32, [i32, POINTER(c_void_p), POINTER(c_void_p),
                                       POINTER(c_void_p), vp, vp, sz, POINTER(c_void_p),
                                       POINTER(c_void_p), POINTER(c_void_p), vp]),
            "gs_l1_loss_grad": (i32, [i64, vp, vp, c_float, vp, vp, vp]),
            "gs_profile_enable": (None, [i32]),
            "gs_profile_collect": (i32, [POINTER(GsKernelTime), i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def is_available() -> bool:
    return os.path.exists(LIB_PATH)


# ----------------------------------------------------------------- helpers

def _ptr(t):
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


def _check(fn: str, status: int):
    if status != 0:
        raise GsError(fn, status)


def make_cameras(cams) -> ctypes.Array:
    """Camera objects (attributes R, t, fx, fy, cx, cy, width, height, near) -> C array."""
    arr = (GsCamera * len(cams))()
    for k, c in enumerate(cams):
        R = [float(x) for x in (c.R.reshape(-1) if hasattr(c.R, "reshape") else c.R)]
        t = [float(x) for x in (c.t.reshape(-1) if hasattr(c.t, "reshape") else c.t)]
        arr[k].R[:] = R
        arr[k].t[:] = t
        arr[k].fx, arr[k].fy, arr[k].cx, arr[k].cy = float(c.fx), float(c.fy), float(c.cx), float(c.cy)
        arr[k].width, arr[k].height = int(c.width), int(c.height)
        arr[k].near_plane = float(getattr(c, "near", 0.2))
    return arr


def make_cfg(tile: int = 16, lds_batch: int = 256, bg=(0.0, 0.0, 0.0), mip2d: bool = False,
             filter3d=None, cam_table=None, cam_index=None, adam_lr=None) -> GsRasterCfg:
    """filter3d: device float32 [n] 3D filter variances or None; cam_table
    (from camera_table), cam_index (device int32 [1]) and adam_lr (device
    float32 [6]): the device-side step parameters of gs_raster_cfg.  The caller
    keeps every tensor alive while the cfg is in use."""
    c = GsRasterCfg()
    c.tile, c.lds_batch = int(tile), int(lds_batch)
    c.bg[:] = [float(x) for x in bg]
    c.mip2d = 1 if mip2d else 0
    c.filter3d = _ptr(filter3d)
    c.cam_table = _ptr(cam_table)
    c.cam_index = _ptr(cam_index)
    c.adam_lr = _ptr(adam_lr)
    return c


def camera_table(cams, device="cuda") -> torch.Tensor:
    """The cameras as a device array of gs_camera structs (uint8 tensor)."""
    arr = make_cameras(cams)
    raw = torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8)
    return raw.to(device)


# ------------------------------------------------------ the C entry points

def gs_version() -> int:
    return int(lib().gs_version())


def gs_status_str(status: int) -> str:
    return lib().gs_status_str(int(status)).decode()


def gs_proj_bytes(n_views: int, n: int) -> int:
    return int(lib().gs_proj_bytes(n_views, n))


def gs_total_tiles(cams_c, cfg) -> int:
    return int(lib().gs_total_tiles(len(cams_c), cams_c, ctypes.byref(cfg)))


def gs_preprocess(cams_c, cfg, n, means, log_scales, quats, opacity_logits, sh, sh_degree,
                  proj, stream=None):
    _check("gs_preprocess", lib().gs_preprocess(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(means), _ptr(log_scales),
        _ptr(quats), _ptr(opacity_logits), _ptr(sh), int(sh_degree), _ptr(proj), _stream(stream)))


def gs_bin_sort_workspace_bytes(n_views: int, n: int, capacity: int) -> int:
    return int(lib().gs_bin_sort_workspace_bytes(n_views, n, capacity))


def gs_bin_sort(cams_c, cfg, n, proj, capacity, ws, keys, vals, ranges, n_pairs_dev,
                stream=None):
    _check("gs_bin_sort", lib().gs_bin_sort(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(proj), int(capacity), _ptr(ws),
        ws.numel() * ws.element_size(), _ptr(keys), _ptr(vals), _ptr(ranges), _ptr(n_pairs_dev),
        _stream(stream)))


GS_BIN_SORT_NOALLOC_MAX_PAIRS = 1 << 22
GS_BIN_SORT_NOALLOC_MAX_ITEMS = 1 << 23


def gs_bin_sort_noalloc(cams_c, cfg, n, proj, capacity, keys, vals, ranges, n_pairs_dev,
                        stream=None):
    _check("gs_bin_sort_noalloc", lib().gs_bin_sort_noalloc(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(proj), int(capacity), _ptr(keys),
        _ptr(vals), _ptr(ranges), _ptr(n_pairs_dev), _stream(stream)))


def gs_spatial_order_workspace_bytes(n: int) -> int:
    return int(lib().gs_spatial_order_workspace_bytes(int(n)))


def gs_spatial_order(n, means, ws, perm, stream=None):
    _check("gs_spatial_order", lib().gs_spatial_order(
        int(n), _ptr(means), _ptr(ws), ws.numel() * ws.element_size(), _ptr(perm),
        _stream(stream)))


def gs_gather_rows(n, perm, src, dst, stream=None):
    """src, dst: lists of device float tensors of n rows each (row = numel / n)."""
    k = len(src)
    rows = [(t.numel() // n) if n else 1 for t in src]
    _check("gs_gather_rows", lib().gs_gather_rows(
        int(n), _ptr(perm), k, (c_void_p * k)(*[_ptr(t) for t in src]),
        (c_void_p * k)(*[_ptr(t) for t in dst]), (c_int32 * k)(*rows), _stream(stream)))


def gs_bin_sort_radix_workspace_bytes(n_views: int, n: int, capacity: int) -> int:
    return int(lib().gs_bin_sort_radix_workspace_bytes(n_views, n, capacity))


def gs_bin_sort_radix(cams_c, cfg, n, proj, capacity, ws, keys, vals, ranges, n_pairs_dev,
                      stream=None):
    """gs_bin_sort's result by a stable LSD radix sort (its own workspace size)."""
    _check("gs_bin_sort_radix", lib().gs_bin_sort_radix(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(proj), int(capacity), _ptr(ws),
        ws.numel() * ws.element_size(), _ptr(keys), _ptr(vals), _ptr(ranges), _ptr(n_pairs_dev),
        _stream(stream)))


def gs_render_fwd(cams_c, cfg, n, proj, ranges, vals, image, final_T, last_contrib,
                  stream=None):
    _check("gs_render_fwd", lib().gs_render_fwd(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(proj), _ptr(ranges), _ptr(vals),
        _ptr(image), _ptr(final_T), _ptr(last_contrib), _stream(stream)))


def gs_render_fwd_l1(cams_c, cfg, n, proj, ranges, vals, image, final_T, last_contrib, target,
                     scale, dL_dimage, loss_sum=None, stream=None):
    _check("gs_render_fwd_l1", lib().gs_render_fwd_l1(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(proj), _ptr(ranges), _ptr(vals),
        _ptr(image), _ptr(final_T), _ptr(last_contrib), _ptr(target), float(scale),
        _ptr(dL_dimage), _ptr(loss_sum), _stream(stream)))


def gs_render_bwd_workspace_bytes(n_views: int, n: int, capacity: int) -> int:
    return int(lib().gs_render_bwd_workspace_bytes(n_views, n, capacity))


def gs_render_bwd(cams_c, cfg, n, means, log_scales, quats, opacity_logits, sh, sh_degree, proj,
                  ranges, vals, final_T, last_contrib, dL_dimage, d_means, d_log_scales, d_quats,
                  d_opacity_logits, d_sh, d_mean2d_abs, capacity, ws, stream=None,
                  accumulate=True):
    _check("gs_render_bwd", lib().gs_render_bwd(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(means), _ptr(log_scales),
        _ptr(quats), _ptr(opacity_logits), _ptr(sh), int(sh_degree), _ptr(proj), _ptr(ranges),
        _ptr(vals), _ptr(final_T), _ptr(last_contrib), _ptr(dL_dimage), _ptr(d_means),
        _ptr(d_log_scales), _ptr(d_quats), _ptr(d_opacity_logits), _ptr(d_sh),
        _ptr(d_mean2d_abs), 1 if accumulate else 0, int(capacity), _ptr(ws),
        ws.numel() * ws.element_size(), _stream(stream)))


def gs_adam_step(groups, step: int, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """groups: list of (p, g, m, v, lr) float32 device tensors (same numel per group)."""
    arr = (GsAdamGroup * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        arr[k].p, arr[k].g, arr[k].m, arr[k].v = _ptr(p), _ptr(g), _ptr(m), _ptr(v)
        arr[k].numel = p.numel()
        arr[k].lr = float(lr)
    _check("gs_adam_step", lib().gs_adam_step(arr, len(groups), int(step), float(beta1),
                                              float(beta2), float(eps), _stream(stream)))


def gs_adam_step_device(groups, step_dev, beta1=0.9, beta2=0.999, eps=1e-15, stream=None):
    """Like gs_adam_step, the step count living in the device int32 ``step_dev``."""
    arr = (GsAdamGroup * len(groups))()
    for k, (p, g, m, v, lr) in enumerate(groups):
        arr[k].p, arr[k].g, arr[k].m, arr[k].v = _ptr(p), _ptr(g), _ptr(m), _ptr(v)
        arr[k].numel = p.numel()
        arr[k].lr = float(lr)
    _check("gs_adam_step_device", lib().gs_adam_step_device(
        arr, len(groups), _ptr(step_dev), float(beta1), float(beta2), float(eps),
        _stream(stream)))


def gs_render_bwd_adam(cams_c, cfg, n, means, log_scales, quats, opacity_logits, sh, sh_degree,
                       proj, ranges, vals, final_T, last_contrib, dL_dimage, m, v, lr, step_dev,
                       beta1, beta2, eps, d_mean2d_abs, capacity, ws, stream=None, sparse=False):
    """m, v: five entries each, in the order means, log_scales, quats,
    opacity_logits, sh; lr: those five learning rates (the SH one for every
    coefficient) or six (the last for the SH coefficients above degree 0).
    sparse: call gs_render_bwd_sparse_adam instead (Gaussians with no pair in
    any view left untouched)."""
    name = "gs_render_bwd_sparse_adam" if sparse else "gs_render_bwd_adam"
    lr = list(lr)
    if len(lr) == 5:
        lr.append(lr[4])
    mp = (c_void_p * 5)(*[_ptr(t) for t in m])
    vp_ = (c_void_p * 5)(*[_ptr(t) for t in v])
    lr_ = (c_float * 6)(*[float(x) for x in lr])
    _check(name, getattr(lib(), name)(
        len(cams_c), cams_c, ctypes.byref(cfg), int(n), _ptr(means), _ptr(log_scales),
        _ptr(quats), _ptr(opacity_logits), _ptr(sh), int(sh_degree), _ptr(proj), _ptr(ranges),
        _ptr(vals), _ptr(final_T), _ptr(last_contrib), _ptr(dL_dimage), mp, vp_, lr_,
        _ptr(step_dev), float(beta1), float(beta2), float(eps), _ptr(d_mean2d_abs),
        int(capacity), _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))


def gs_render_bwd_sparse_adam(*args, **kw):
    """gs_render_bwd_adam's arguments; Gaussians with no pair in any view keep
    their parameters and moments."""
    kw["sparse"] = True
    gs_render_bwd_adam(*args, **kw)


def gs_filter3d_variance(cams_c, n, means, scale, variance, scratch, stream=None):
    """Mip-Splatting's 3D filter variances of n Gaussians [n] from the
    training views; scratch: device int32/uint32 [1]."""
    _check("gs_filter3d_variance", lib().gs_filter3d_variance(
        len(cams_c), cams_c, int(n), _ptr(means), float(scale), _ptr(variance), _ptr(scratch),
        _stream(stream)))


def gs_frequency_map_workspace_bytes(H: int, W: int) -> int:
    return int(lib().gs_frequency_map_workspace_bytes(int(H), int(W)))


def gs_frequency_map(images, H, W, mag, ws, stream=None):
    """images: device float32 [n,3,H,W] (contiguous); mag: device float64 [H,W]."""
    n = images.numel() // (3 * H * W)
    _check("gs_frequency_map", lib().gs_frequency_map(
        int(n), int(H), int(W), _ptr(images), _ptr(mag), _ptr(ws), ws.numel() * ws.element_size(),
        _stream(stream)))


def gs_resolution_schedule(mag_host, S, a=4.0, m=4, r_max=0.0, norm="sum"):
    """mag_host: numpy float64 [H,W] frequency map; norm "sum" (X(F_r) scaled by
    1/r^2) or "mean" (by 1/(H W)); returns (r_knots, s_knots)."""
    if norm not in ("sum", "mean"):
        raise ValueError(norm)
    import numpy as np
    mag = np.ascontiguousarray(mag_host, dtype=np.float64)
    H, W = mag.shape
    r = (c_double * (m + 1))()
    s = (c_double * (m + 1))()
    _check("gs_resolution_schedule", lib().gs_resolution_schedule(
        mag.ctypes.data_as(POINTER(c_double)), int(H), int(W), float(S), float(a), int(m),
        float(r_max), 1 if norm == "mean" else 0, r, s))
    return np.array(r[:]), np.array(s[:])


def gs_schedule_resolution(k, r_knots, s_knots) -> float:
    m = len(r_knots) - 1
    r = (c_double * (m + 1))(*[float(x) for x in r_knots])
    s = (c_double * (m + 1))(*[float(x) for x in s_knots])
    return float(lib().gs_schedule_resolution(float(k), int(m), r, s))


def gs_downsample_aa(src, n_planes, H, W, h, w, dst, stream=None):
    _check("gs_downsample_aa", lib().gs_downsample_aa(
        int(n_planes), int(H), int(W), int(h), int(w), _ptr(src), _ptr(dst), _stream(stream)))


def gs_primitive_target(i, S, r, p_init, p_fin) -> float:
    return float(lib().gs_primitive_target(float(i), float(S), float(r), float(p_init),
                                           float(p_fin)))


def gs_primitive_budget(p_fin_prev, p_add, gamma=0.98, eta=1.0) -> float:
    return float(lib().gs_primitive_budget(float(p_fin_prev), float(p_add), float(gamma),
                                           float(eta)))


def gs_densify_workspace_bytes(n: int) -> int:
    return int(lib().gs_densify_workspace_bytes(int(n)))


def gs_densify_stats(n_views, n, proj, d_mean2d_abs, accum, count, scale=1.0, stream=None):
    _check("gs_densify_stats", lib().gs_densify_stats(
        int(n_views), int(n), _ptr(proj), _ptr(d_mean2d_abs), float(scale), _ptr(accum),
        _ptr(count), _stream(stream)))


def gs_densify_classify(n, accum, count, opacity_logits, grad_thr, min_opacity, ws, counts_dev,
                        stream=None):
    _check("gs_densify_classify", lib().gs_densify_classify(
        int(n), _ptr(accum), _ptr(count), _ptr(opacity_logits), float(grad_thr),
        float(min_opacity), _ptr(ws), ws.numel() * ws.element_size(), _ptr(counts_dev),
        _stream(stream)))


def gs_densify_plan(n, k, n_candidates, log_scales, max_scale, ws, n_new_dev, stream=None):
    _check("gs_densify_plan", lib().gs_densify_plan(
        int(n), int(k), int(n_candidates), _ptr(log_scales), float(max_scale), _ptr(ws),
        ws.numel() * ws.element_size(), _ptr(n_new_dev), _stream(stream)))


def gs_densify_apply(n, params, m, v, z, ws, params_out, m_out, v_out, stream=None):
    """params, m, v, params_out, m_out, v_out: five tensors each (means,
    log_scales, quats, opacity_logits, sh)."""
    arr = lambda ts: (c_void_p * 5)(*[_ptr(t) for t in ts])
    _check("gs_densify_apply", lib().gs_densify_apply(
        int(n), arr(params), arr(m), arr(v), _ptr(z), _ptr(ws), ws.numel() * ws.element_size(),
        arr(params_out), arr(m_out), arr(v_out), _stream(stream)))


def gs_l1_loss_grad(image, target, scale, dL_dimage, loss_sum=None, stream=None):
    _check("gs_l1_loss_grad", lib().gs_l1_loss_grad(
        image.numel(), _ptr(image), _ptr(target), float(scale), _ptr(dL_dimage), _ptr(loss_sum),
        _stream(stream)))


def gs_profile_enable(on: bool = True):
    lib().gs_profile_enable(1 if on else 0)


def gs_profile_collect(max_entries: int = 64) -> dict:
    """{kernel name: (launches, total_ms)} for the launches recorded since the last collect."""
    arr = (GsKernelTime * max_entries)()
    n = lib().gs_profile_collect(arr, max_entries)
    if n < 0:
        raise GsError("gs_profile_collect", 3)
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n)}
