"""Per-Gaussian projection to the image plane (FP64), the 3D->2D splatting step.

The paper names this step (Sec. 3: each 3D Gaussian with centre p_i and
covariance Sigma_i is splatted to a 2D Gaussian G2D_i on the image plane)
but prints no formula for it.  This follows the EWA splatting reading used by
3DGS-family rasterizers, with the choices below (each is a reading where the
paper is silent):

* camera space x_c = R m + t; cull when the float32 depth z_f32 <= near;
* Sigma = M M^T with M = R(q/|q|) diag(exp(log_scale));
* Sigma' = J W Sigma W^T J^T + 0.3 I (W = R, J the perspective Jacobian at
  x_c, no field-of-view clamp); cull when det(Sigma') <= 0;
* conic (a, b, c) = inverse of Sigma' stored as (S11, -S01, S00)/det;
* mean2D = (fx x/z + cx, fy y/z + cy); pixel centres at (px+0.5, py+0.5);
* colour = max(0, sum_k sh_k Y_k(d) + 0.5) with d the unit vector from the
  camera centre to the mean;
* opacity o = sigmoid(logit); cull when o < 1/255;
* an opacity-aware, conservative footprint: every pixel whose centre lies
  outside the axis-aligned box of the ellipse {D : D^T Q D <= 2 ln(255 o)}
  has alpha < 1/255, so binning by that box never changes a pixel.  The box
  half-widths sqrt(2 ln(255 o) Sigma'_00), sqrt(2 ln(255 o) Sigma'_11) are
  widened by EXT_REL (relative) and EXT_ABS (pixels) so that float32
  evaluation on the device stays inside them;
* depth key: z_f32 = (((R20*mx) + (R21*my)) + (R22*mz)) + tz with every
  product and sum rounded to float32 in that order (no fused multiply-add);
  its IEEE bits, which order like the values for z > 0, are the sort key.

Mip-Splatting's filters (the second backbone family the paper equips, Sec. 5
and the supplementary), both optional:

* 3D smoothing filter: a per-Gaussian variance f (world units squared, from
  ``filter3d_variance``) is added to Sigma, Sigma_f = Sigma + f I, and the
  opacity is scaled by sqrt(det Sigma / det Sigma_f) = prod_i s_i /
  sqrt(s_i^2 + f), so the filtered Gaussian keeps its 3D integral;
* 2D mip filter: Sigma' = J W Sigma_f W^T J^T + 0.1 I replaces the 0.3
  dilation, and the opacity is scaled by sqrt(det(Sigma'-0.1 I) / det Sigma'),
  so the splat keeps its 2D integral;
* the blending opacity o' = sigmoid(logit) times both factors replaces o in
  the cull, the footprint and Eq. 1.

Guard bands flag the decisions that float32 and float64 may legitimately take
differently, so tests can exclude exactly those cases.
"""
from __future__ import annotations

import numpy as np

from . import sh as _sh

F64 = np.float64
NEAR_DEFAULT = 0.2
DILATION = 0.3
MIP_2D_VARIANCE = 0.1   # the 2D mip filter: a one-pixel box approximated by a Gaussian
FILTER_3D_SCALE = 0.2   # Mip-Splatting's 3D filter variance in units of (pixel footprint)^2
ALPHA_MIN = 1.0 / 255.0
EXT_REL = 1.0e-3
EXT_ABS = 1.0e-2
# guard band (pixels) for the box edges: relative to the coordinate magnitude
RECT_GUARD_REL = 4.0e-6
RECT_GUARD_ABS = 1.0e-5
RGB_GUARD = 1.0e-5
OPACITY_GUARD_REL = 1.0e-5


def depth_f32(means: np.ndarray, R: np.ndarray, t: np.ndarray) -> np.ndarray:
    """The float32 depth of each mean, rounded step by step as the key defines it."""
    m = np.asarray(means, np.float32)
    R32 = np.asarray(R, np.float32)
    t32 = np.asarray(t, np.float32)
    p0 = m[:, 0] * R32[2, 0]
    p1 = m[:, 1] * R32[2, 1]
    p2 = m[:, 2] * R32[2, 2]
    s = (p0 + p1).astype(np.float32)
    s = (s + p2).astype(np.float32)
    return (s + t32[2]).astype(np.float32)


def quat_to_rot(q: np.ndarray) -> np.ndarray:
    """Rotation matrix of unit quaternions q = (w, x, y, z), [N,3,3]."""
    w, x, y, z = q[:, 0], q[:, 1], q[:, 2], q[:, 3]
    R = np.empty((q.shape[0], 3, 3), F64)
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - w * z)
    R[:, 0, 2] = 2 * (x * z + w * y)
    R[:, 1, 0] = 2 * (x * y + w * z)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - w * x)
    R[:, 2, 0] = 2 * (x * z - w * y)
    R[:, 2, 1] = 2 * (y * z + w * x)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _near_edge(v: np.ndarray, fn, guard: np.ndarray) -> np.ndarray:
    """True where fn(v) would change inside [v - guard, v + guard]."""
    return fn(v - guard) != fn(v + guard)


def project(scene: dict, cam, tile: int = 16, sh_degree: int = 3, mip2d: bool = False,
            filter3d=None) -> dict:
    """Project every Gaussian of ``scene`` into ``cam``; all outputs FP64 unless noted.
    ``mip2d``: the 2D mip filter instead of the 0.3 dilation; ``filter3d``:
    per-Gaussian 3D filter variances [N] (None: no 3D filter).

    Returns a dict with
      xc [N,3], depth_f32 [N] (float32), mean2d [N,2], cov2d [N,3] (S00,S01,S11),
      conic [N,3] (a,b,c), opacity [N], rgb_raw [N,3], rgb [N,3], dirs [N,3],
      dist [N], Rq [N,3,3], scales [N,3], qn [N,4], Sigma [N,3,3], J [N,2,3],
      Tm [N,2,3], live [N] (passes z/det/opacity culls: the blend candidates),
      rect [N,4] int64 (tx0, ty0, tx1, ty1 inclusive), tiles_touched [N] int64,
      px_box [N,4] int64 (pixel box, inclusive, clamped), flag_rect, flag_rgb [N,3],
      flag_opacity; opacity is the blending opacity o', opacity_raw the sigmoid,
      coef3 / coef2 the 3D / 2D filter factors (1 when off), C2raw [N,3] the
      projected covariance before the 2D low-pass, Sigma the filtered Sigma_f.
    """
    means = np.asarray(scene["means"], F64)
    ls = np.asarray(scene["log_scales"], F64)
    q = np.asarray(scene["quats"], F64)
    logit = np.asarray(scene["opacity_logits"], F64)
    shc = np.asarray(scene["sh"], F64)
    n = means.shape[0]
    W, H = int(cam.width), int(cam.height)
    Rc = np.asarray(cam.R, F64)
    tc = np.asarray(cam.t, F64)
    fx, fy, cx, cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    near = float(getattr(cam, "near", NEAR_DEFAULT))

    xc = means @ Rc.T + tc
    z32 = depth_f32(scene["means"], cam.R, cam.t)
    x, y, z = xc[:, 0], xc[:, 1], xc[:, 2]
    front = z32 > np.float32(near)
    zs = np.where(front, z, 1.0)  # avoid division by ~0 on culled rows

    s = np.exp(ls)
    qn = q / np.linalg.norm(q, axis=1, keepdims=True)
    Rq = quat_to_rot(qn)
    M = Rq * s[:, None, :]
    Sigma = M @ np.transpose(M, (0, 2, 1))
    f3 = np.zeros(n) if filter3d is None else np.asarray(filter3d, F64)
    if filter3d is not None:
        Sigma = Sigma + f3[:, None, None] * np.eye(3)
        coef3 = np.prod(s, axis=1) / np.sqrt(np.prod(s * s + f3[:, None], axis=1))
    else:
        coef3 = np.ones(n)

    J = np.zeros((n, 2, 3), F64)
    J[:, 0, 0] = fx / zs
    J[:, 0, 2] = -fx * x / (zs * zs)
    J[:, 1, 1] = fy / zs
    J[:, 1, 2] = -fy * y / (zs * zs)
    Tm = J @ Rc
    C2 = Tm @ Sigma @ np.transpose(Tm, (0, 2, 1))
    low = MIP_2D_VARIANCE if mip2d else DILATION
    c00 = C2[:, 0, 0] + low
    c01 = C2[:, 0, 1]
    c11 = C2[:, 1, 1] + low
    det = c00 * c11 - c01 * c01
    good_det = det > 0
    dets = np.where(good_det, det, 1.0)
    if mip2d:
        det_raw = C2[:, 0, 0] * C2[:, 1, 1] - C2[:, 0, 1] * C2[:, 0, 1]
        coef2 = np.sqrt(np.maximum(det_raw, 0.0) / dets)
    else:
        coef2 = np.ones(n)
    conic = np.stack([c11 / dets, -c01 / dets, c00 / dets], axis=1)
    mean2d = np.stack([fx * x / zs + cx, fy * y / zs + cy], axis=1)

    campos = -Rc.T @ tc
    v = means - campos
    dist = np.linalg.norm(v, axis=1)
    dirs = v / np.maximum(dist, 1e-300)[:, None]
    K = _sh.n_coeffs(sh_degree)
    Y = _sh.basis(dirs, sh_degree)                       # [N,K]
    rgb_raw = np.einsum("nk,nkc->nc", Y, shc[:, :K, :]) + 0.5
    rgb = np.maximum(rgb_raw, 0.0)

    opacity_raw = 1.0 / (1.0 + np.exp(-logit))
    opacity = opacity_raw
    if filter3d is not None:
        opacity = opacity * coef3
    if mip2d:
        opacity = opacity * coef2
    opaque = opacity >= ALPHA_MIN
    live = front & good_det & opaque

    # conservative footprint box (pixel centres), then tiles
    k2 = 2.0 * np.log(np.maximum(255.0 * opacity, 1.0))
    ext_x = np.sqrt(k2 * c00) * (1.0 + EXT_REL) + EXT_ABS
    ext_y = np.sqrt(k2 * c11) * (1.0 + EXT_REL) + EXT_ABS
    lo_x = mean2d[:, 0] - ext_x - 0.5
    hi_x = mean2d[:, 0] + ext_x - 0.5
    lo_y = mean2d[:, 1] - ext_y - 0.5
    hi_y = mean2d[:, 1] + ext_y - 0.5

    def box(lo, hi, size):
        a = np.clip(np.ceil(np.clip(lo, -2.0, size + 2.0)), 0, size - 1)
        b = np.clip(np.floor(np.clip(hi, -2.0, size + 2.0)), 0, size - 1)
        empty = (np.ceil(np.clip(lo, -2.0, size + 2.0)) > size - 1) | \
                (np.floor(np.clip(hi, -2.0, size + 2.0)) < 0) | (a > b)
        return a.astype(np.int64), b.astype(np.int64), empty

    px0, px1, ex = box(lo_x, hi_x, W)
    py0, py1, ey = box(lo_y, hi_y, H)
    has_box = live & ~ex & ~ey
    rect = np.stack([px0 // tile, py0 // tile, px1 // tile, py1 // tile], axis=1)
    rect[~has_box] = 0
    tiles_touched = np.where(has_box, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)

    # guard bands: would the tile rectangle (or emptiness) change within the guard?
    def tile_of_lo(v, size):
        c = np.ceil(np.clip(v, -2.0, size + 2.0))
        return np.where(c > size - 1, -1, np.clip(c, 0, size - 1) // tile)

    def tile_of_hi(v, size):
        f = np.floor(np.clip(v, -2.0, size + 2.0))
        return np.where(f < 0, -1, np.clip(f, 0, size - 1) // tile)

    gx = RECT_GUARD_REL * (np.abs(mean2d[:, 0]) + ext_x) + RECT_GUARD_ABS
    gy = RECT_GUARD_REL * (np.abs(mean2d[:, 1]) + ext_y) + RECT_GUARD_ABS
    flag_rect = live & (_near_edge(lo_x, lambda v: tile_of_lo(v, W), gx) |
                        _near_edge(hi_x, lambda v: tile_of_hi(v, W), gx) |
                        _near_edge(lo_y, lambda v: tile_of_lo(v, H), gy) |
                        _near_edge(hi_y, lambda v: tile_of_hi(v, H), gy))
    flag_rgb = np.abs(rgb_raw) < RGB_GUARD
    flag_opacity = np.abs(opacity - ALPHA_MIN) < OPACITY_GUARD_REL * ALPHA_MIN

    return dict(xc=xc, depth_f32=z32, mean2d=mean2d, cov2d=np.stack([c00, c01, c11], 1),
                conic=conic, opacity=opacity, opacity_raw=opacity_raw, coef3=coef3, coef2=coef2,
                C2raw=np.stack([C2[:, 0, 0], C2[:, 0, 1], C2[:, 1, 1]], 1), f3=f3,
                mip2d=bool(mip2d), has_filter3d=filter3d is not None,
                rgb_raw=rgb_raw, rgb=rgb, dirs=dirs, dist=dist,
                Y=Y, Rq=Rq, scales=s, qn=qn, qnorm=np.linalg.norm(q, axis=1), Sigma=Sigma,
                J=J, Tm=Tm, Rc=Rc, campos=campos, live=live, rect=rect,
                tiles_touched=tiles_touched.astype(np.int64),
                px_box=np.stack([px0, py0, px1, py1], 1), flag_rect=flag_rect,
                flag_rgb=flag_rgb, flag_opacity=flag_opacity, sh_degree=sh_degree,
                width=W, height=H, tile=tile, fx=fx, fy=fy)


def filter3d_variance(means, cams, scale: float = FILTER_3D_SCALE):
    """Mip-Splatting's 3D smoothing filter: per Gaussian, the variance
    scale / nu^2 with nu the highest sampling rate fx / z over the cameras
    whose image rectangle [0, W] x [0, H] contains the projected centre in
    front of the near plane.  A Gaussian that no camera sees takes the largest
    variance among the seen ones (0 when none is seen).

    Also returns flag [N]: the centre sits within a float32 guard band of an
    image edge or the near plane in some camera, where a float32 evaluation
    may see it differently."""
    m = np.asarray(means, F64)
    n = m.shape[0]
    nu = np.zeros(n)
    flag = np.zeros(n, bool)
    for cam in cams:
        R, t = np.asarray(cam.R, F64), np.asarray(cam.t, F64)
        xc = m @ R.T + t
        z = xc[:, 2]
        near = float(getattr(cam, "near", NEAR_DEFAULT))
        zs = np.where(z > 0, z, 1.0)
        u = float(cam.fx) * xc[:, 0] / zs + float(cam.cx)
        v = float(cam.fy) * xc[:, 1] / zs + float(cam.cy)
        W, H = float(cam.width), float(cam.height)
        seen = (z > near) & (u >= 0) & (u <= W) & (v >= 0) & (v <= H)
        nu = np.where(seen, np.maximum(nu, float(cam.fx) / zs), nu)
        g = 1e-4 * (np.abs(u) + np.abs(v) + W + H)
        flag |= (z > 0) & ((np.abs(z - near) < 1e-5 * np.abs(z) + 1e-6) |
                           (np.minimum(np.abs(u), np.abs(u - W)) < g) |
                           (np.minimum(np.abs(v), np.abs(v - H)) < g))
    seen = nu > 0
    var = np.where(seen, scale / np.where(seen, nu, 1.0) ** 2, 0.0)
    if seen.any():
        var[~seen] = var[seen].max()
    return var, flag
