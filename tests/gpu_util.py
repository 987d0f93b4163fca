"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and decode its opaque per-view records for comparison with the oracle."""
from __future__ import annotations

import math
import os

import numpy as np
import torch

from paper_2503_18402_amd import gsmi, raster

LOG2E = 1.0 / math.log(2.0)


def align256(x: int) -> int:
    return (x + 255) & ~255


def decode_proj(frame, view: int = 0, tile: int | None = None) -> dict:
    """Per-Gaussian records of one view, in the documented layout of the
    projected-record buffer (rec: 3 float4, then tiles touched, then flags,
    then the first pair position binning writes, then the pair total in a
    256-byte slot); the record holds log2 of the opacity."""
    n = frame.n
    stride = align256(48 * n) + 3 * align256(4 * n) + 256
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


def zero_flagged(w, F):
    """The upstream dL/dC (a [3,H,W] image, or [3,P] at the oracle's sampled
    pixels) with zeros at every pixel the oracle flags: one whose float32
    decisions (alpha vs 1/255, T vs 1e-4, the 0.99 clamp) sit inside the guard
    band.  Each pixel's part of every gradient is proportional to its
    upstream, so with dL/dC = 0 there both sides take nothing from those
    pixels and every Gaussian stays in the gradient check."""
    w = np.array(w, dtype=np.float32, copy=True)
    w.reshape(3, -1)[:, np.asarray(F["flag"]).reshape(-1)] = 0.0
    return w


def gaussian_flags(P):
    """Gaussians with a per-Gaussian float32 decision in its guard band, which no
    upstream can neutralise: a colour channel at the clamp at 0 (the SH
    gradient is zeroed on one side only) or the opacity at the 1/255 cull."""
    return P["flag_rgb"].any(1) | P["flag_opacity"]


# Every check_grads call of the session: test, parameter, elements checked,
# plain-rule violations and the worst error relative to each bound.
RECORDS: list[dict] = []


# Some mean-gradient elements cancel down to 1e-4 of the terms summed into them
# (pixels on both sides of the centre, with upstreams of both signs); their
# float32 accumulation error, a few ulps of the term scale S, can then exceed
# 1e-3 of the result.  Tests where the plain rule failed for such an element
# allow this fraction of the mean gradients to fall back on the 1e-5 S bound.
MEANS_CANCELLATION_FRAC = 1e-3


def check_grads(g, ref, bound, mask=None, rel=1e-3, abs_=1e-6, cond=1e-5, max_frac=0.0,
                name=""):
    """Gradient parity.  The plain rule is |g - ref| <= rel |ref| + abs for every
    element; up to ``max_frac`` of the checked elements may break it, and those
    must still satisfy
        |g - ref| <= rel |ref| + abs + cond * S,
    S the oracle's scale of the terms summed into that element (a float32
    result that cancels down from large terms carries an error proportional
    to S; 1e-5 S is about 80 ulps of it).  Every call is recorded in RECORDS;
    returns the number of plain-rule violations."""
    g = np.asarray(g, np.float64)
    ref = np.asarray(ref, np.float64)
    err = np.abs(g - ref)
    m = np.ones(g.shape, bool) if mask is None else np.broadcast_to(
        mask.reshape(mask.shape + (1,) * (g.ndim - 1)), g.shape)
    plain = rel * np.abs(ref) + abs_
    strict = (err > plain) & m
    loose = (err > plain + cond * np.asarray(bound)) & m
    RECORDS.append(dict(test=os.environ.get("PYTEST_CURRENT_TEST", "").split(" ")[0],
                        param=name, checked=int(m.sum()), plain_violations=int(strict.sum()),
                        worst_plain=float((err / plain)[m].max(initial=0.0)),
                        worst_conditioned=float((err / (plain + cond * np.asarray(bound)))[m]
                                                .max(initial=0.0))))
    assert not loose.any(), ("gradient outside the conditioned bound", name, int(loose.sum()),
                             np.argwhere(loose)[:5].tolist())
    assert strict.sum() <= max_frac * m.sum(), ("plain-rule violations", name, int(strict.sum()),
                                                int(m.sum()), np.argwhere(strict)[:5].tolist())
    return int(strict.sum())
