"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and decode its opaque per-view records for comparison with the oracle."""
from __future__ import annotations

import math

import numpy as np
import torch

from paper_2503_18402_amd import gsmi, raster

LOG2E = 1.0 / math.log(2.0)


def align256(x: int) -> int:
    return (x + 255) & ~255


def decode_proj(frame, view: int = 0, tile: int | None = None) -> dict:
    """Per-Gaussian records of one view, in the documented layout of the
    projected-record buffer (rec: 3 float4, then tiles touched, then flags);
    the record holds log2 of the opacity."""
    n = frame.n
    stride = align256(48 * n) + 2 * align256(4 * n)
    raw = frame.proj.cpu().numpy()[view * stride:(view + 1) * stride]
    rec = raw[:48 * n].view(np.float32).reshape(n, 12)
    tt_off = align256(48 * n)
    tt = raw[tt_off:tt_off + 4 * n].view(np.uint32)
    fl_off = tt_off + align256(4 * n)
    flags = raw[fl_off:fl_off + 4 * n].view(np.uint32)
    box_lo = rec[:, 10].view(np.uint32)
    box_hi = rec[:, 11].view(np.uint32)
    A, B, C = rec[:, 2].astype(np.float64), rec[:, 3].astype(np.float64), rec[:, 4].astype(np.float64)
    conic = np.stack([-2.0 * A / LOG2E, -B / LOG2E, -2.0 * C / LOG2E], 1)
    px_box = np.stack([box_lo & 0xFFFF, box_lo >> 16, box_hi & 0xFFFF, box_hi >> 16], 1).astype(np.int64)
    T = frame.cfg.tile if tile is None else tile
    origin = np.stack([(box_lo & 0xFFFF) // T * T, (box_lo >> 16) // T * T], 1).astype(np.float64)
    origin[tt == 0] = 0.0
    return dict(mean2d=rec[:, 0:2].astype(np.float64) + origin, conic=conic,
                opacity=np.where(tt > 0, np.exp2(rec[:, 5].astype(np.float64)), 0.0),
                rgb=rec[:, [6, 7, 8]].astype(np.float64),
                depth=rec[:, 9].copy(), tt=tt.astype(np.int64), flags=flags, px_box=px_box)


def gpu_rect(d: dict, tile: int) -> np.ndarray:
    return np.where(d["tt"][:, None] > 0, d["px_box"] // tile, 0)


def grads_np(g: dict) -> dict:
    return {k: v.detach().cpu().numpy().astype(np.float64) for k, v in g.items()}


def run(scene: dict, cams, tile=16, lds_batch=256, bg=(0.0, 0.0, 0.0), sh_degree=3,
        upstream=None, want_keys=True, capacity=None, mip2d=False, filter3d=None):
    """Forward (and backward if ``upstream`` is given, one [3,H,W] array per view).
    filter3d: numpy [N] 3D filter variances or None."""
    params = raster.to_device(scene, "cuda")
    f3 = None if filter3d is None else torch.from_numpy(
        np.ascontiguousarray(filter3d, np.float32)).cuda()
    frame = raster.render(params, cams, tile=tile, lds_batch=lds_batch, bg=bg,
                          sh_degree=sh_degree, want_keys=want_keys, capacity=capacity,
                          mip2d=mip2d, filter3d=f3)
    grads = None
    if upstream is not None:
        dL = torch.cat([torch.from_numpy(np.ascontiguousarray(u, np.float32)).reshape(-1)
                        for u in upstream]).cuda()
        grads = grads_np(raster.render_backward(params, frame, dL))
    torch.cuda.synchronize()
    return params, frame, grads


def grad_violations(g, ref, rel=1e-3, abs_=1e-6, mask=None):
    """Elements breaking |g - ref| <= rel |ref| + abs (rows in ``mask`` are skipped)."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    bad = np.abs(g - ref) > rel * np.abs(ref) + abs_
    if mask is not None:
        bad = bad & mask.reshape(mask.shape + (1,) * (bad.ndim - 1))
    return bad


def check_grads(g, ref, bound, mask=None, rel=1e-3, abs_=1e-6, cond=1e-3, max_frac=1e-3):
    """Gradient parity.  Every element must satisfy
        |g - ref| <= rel |ref| + abs + cond * S
    where S is the oracle's scale of the terms summed into that element (a
    float32 result that cancels down from large terms carries an error
    proportional to S); and the elements breaking the plain rule
    |g - ref| <= rel |ref| + abs must be at most ``max_frac`` of the checked
    ones.  Returns the number of plain-rule violations."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(g - ref)
    m = np.ones(g.shape, bool) if mask is None else np.broadcast_to(
        mask.reshape(mask.shape + (1,) * (g.ndim - 1)), g.shape)
    loose = (err > rel * np.abs(ref) + abs_ + cond * np.asarray(bound)) & m
    assert not loose.any(), ("gradient outside the conditioned bound", int(loose.sum()),
                             np.argwhere(loose)[:5].tolist())
    strict = (err > rel * np.abs(ref) + abs_) & m
    assert strict.sum() <= max_frac * m.sum(), ("too many plain-rule violations",
                                                int(strict.sum()), int(m.sum()))
    return int(strict.sum())
