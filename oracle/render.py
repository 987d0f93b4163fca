"""Per-pixel brute-force blend (Sec. 3, Eq. 1) and its analytic backward, FP64.

Forward, for every pixel centre u = (px+0.5, py+0.5), over ALL live Gaussians
(no tiles: the footprint boxes are conservative, so binning is only an
acceleration and must not change a pixel), taken in ascending (z_f32, index)
order:

  D = u - mean2d;  power = -(a Dx^2 + c Dy^2)/2 - b Dx Dy
  skip when power > 0;  alpha = min(0.99, o exp(power));  skip when alpha < 1/255
  T' = T (1 - alpha);  if T' < 1e-4 stop *without* blending this Gaussian
  C += alpha T rgb;  T = T'

Output C + T bg, final T, and the ordered list of blended Gaussians.  This is
Eq. 1 with w_i = o_i G2D_i(u) plus the rasterizer's cutoff, clamp and
early-exit conventions (the paper is silent on those; they are readings).

Backward: with g = dL/dC, S_i the colour accumulated behind i (including
T_final bg), dC/dc_i = alpha_i T_i and dC/dalpha_i = T_i c_i - S_i/(1-alpha_i);
the 0.99 clamp has zero derivative where it is active.  Then through
alpha = o G and G = exp(power) to (mean2d, conic, opacity, rgb) and, in
``chain_to_3d``, through the projection of ``project.py`` to the parameters.
With Mip-Splatting's filters the blending opacity is sigmoid(logit) c3 c2, so
its gradient also reaches the log-scales through the 3D factor c3 and the
projected covariance through the 2D factor c2.

Test infrastructure only: imported by tests/ (and bench.py's CPU baseline),
never by the product path.
"""
from __future__ import annotations

import numpy as np

from . import project as _proj
from . import sh as _sh

F64 = np.float64
ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_MIN = 1.0e-4
# guard bands for float32-vs-float64 decisions (relative)
ALPHA_GUARD = 1.0e-4
T_GUARD = 1.0e-4
CLAMP_GUARD = 1.0e-5


def _order(P: dict) -> np.ndarray:
    """Indices of live Gaussians in ascending (z_f32, index) order."""
    live = np.nonzero(P["live"])[0]
    z = P["depth_f32"][live]
    return live[np.lexsort((live, z))]


def _pixel_block(P, order, pix, W):
    px = (pix % W).astype(F64) + 0.5
    py = (pix // W).astype(F64) + 0.5
    mx = P["mean2d"][order, 0]
    my = P["mean2d"][order, 1]
    a, b, c = P["conic"][order, 0], P["conic"][order, 1], P["conic"][order, 2]
    dx = px[:, None] - mx[None, :]
    dy = py[:, None] - my[None, :]
    power = -0.5 * (a[None, :] * dx * dx + c[None, :] * dy * dy) - b[None, :] * dx * dy
    G = np.exp(np.minimum(power, 0.0))
    o = P["opacity"][order][None, :]
    raw = o * G
    alpha = np.minimum(ALPHA_MAX, raw)
    valid = (power <= 0.0) & (alpha >= ALPHA_MIN)
    aeff = np.where(valid, alpha, 0.0)
    Tincl = np.cumprod(1.0 - aeff, axis=1)
    below = Tincl < T_MIN
    n = aeff.shape[1]
    stop = np.where(below.any(axis=1), below.argmax(axis=1), n)
    cols = np.arange(n)[None, :]
    keep = valid & (cols < stop[:, None])
    Tbefore = np.concatenate([np.ones((aeff.shape[0], 1)), Tincl[:, :-1]], axis=1)
    return dict(dx=dx, dy=dy, power=power, G=G, raw=raw, alpha=alpha, valid=valid,
                keep=keep, Tbefore=Tbefore, Tincl=Tincl, stop=stop, cols=cols)


def _guard_flags(B: dict) -> np.ndarray:
    """Pixels of a block with a discrete decision, up to and including the stop
    column, inside the float32 guard band (alpha vs 1/255, T' vs 1e-4, the
    0.99 clamp, power at 0)."""
    upto = B["cols"] <= B["stop"][:, None]
    near_cut = np.abs(B["alpha"] / ALPHA_MIN - 1.0) < ALPHA_GUARD
    near_T = np.abs(B["Tincl"] / T_MIN - 1.0) < T_GUARD
    near_clamp = B["valid"] & (np.abs(B["raw"] / ALPHA_MAX - 1.0) < CLAMP_GUARD)
    near_pow = B["valid"] & (B["power"] > -1e-12)
    return ((near_cut | near_T | near_clamp | near_pow) & upto).any(axis=1)


def render_fwd(P: dict, bg=(0.0, 0.0, 0.0), pixels=None, chunk: int = 256,
               want_lists: bool = False) -> dict:
    """Blend every requested pixel (default: all, row-major).

    Returns image [3,npix] (or [3,H,W] for all pixels), final_T, n_contrib,
    last_id (Gaussian index of the last blended Gaussian, -1 when none),
    flag (guard-band pixels), and optionally the per-pixel blended id lists.
    """
    W, H = P["width"], P["height"]
    all_px = pixels is None
    pix = np.arange(W * H) if all_px else np.asarray(pixels, np.int64)
    order = _order(P)
    rgb = P["rgb"][order]
    bg = np.asarray(bg, F64)
    npx = pix.shape[0]
    img = np.zeros((3, npx))
    fT = np.ones(npx)
    ncon = np.zeros(npx, np.int64)
    last = np.full(npx, -1, np.int64)
    flag = np.zeros(npx, bool)
    lists = [] if want_lists else None
    for s in range(0, npx, chunk):
        blk = pix[s:s + chunk]
        B = _pixel_block(P, order, blk, W)
        w = np.where(B["keep"], B["alpha"] * B["Tbefore"], 0.0)
        img[:, s:s + len(blk)] = (w @ rgb).T
        Tf = np.prod(np.where(B["keep"], 1.0 - B["alpha"], 1.0), axis=1)
        fT[s:s + len(blk)] = Tf
        img[:, s:s + len(blk)] += Tf[None, :] * bg[:, None]
        ncon[s:s + len(blk)] = B["keep"].sum(axis=1)
        has = B["keep"].any(axis=1)
        lastcol = B["keep"].shape[1] - 1 - np.argmax(B["keep"][:, ::-1], axis=1)
        last[s:s + len(blk)] = np.where(has, order[lastcol] if len(order) else -1, -1)
        flag[s:s + len(blk)] = _guard_flags(B)
        if want_lists:
            for r in range(len(blk)):
                lists.append(order[B["keep"][r]])
    out = dict(image=img, final_T=fT, n_contrib=ncon, last_id=last, flag=flag, pixels=pix,
               order=order)
    if want_lists:
        out["lists"] = lists
    if all_px:
        out["image"] = img.reshape(3, H, W)
        out["final_T"] = fT.reshape(H, W)
        out["n_contrib"] = ncon.reshape(H, W)
        out["last_id"] = last.reshape(H, W)
        out["flag"] = flag.reshape(H, W)
    return out


def _bwd_block(P: dict, cand: np.ndarray, blk: np.ndarray, g: np.ndarray, bg: np.ndarray):
    """Backward of the pixels ``blk`` (dL/dC rows ``g`` [p,3]) over the Gaussians
    ``cand`` taken in that order: per-candidate sums of the 2D gradients and of
    the absolute values of their terms (the error scale)."""
    W = P["width"]
    rgb = P["rgb"][cand]
    o = P["opacity"][cand]
    a, b, c = P["conic"][cand, 0], P["conic"][cand, 1], P["conic"][cand, 2]
    B = _pixel_block(P, cand, blk, W)
    keep = B["keep"]
    alpha = np.where(keep, B["alpha"], 0.0)
    T = B["Tbefore"]
    w = alpha * T                                         # [p,n]
    Tf = np.prod(np.where(keep, 1.0 - alpha, 1.0), axis=1)
    # colour behind each Gaussian: sum over later blended ones + T_final * bg
    contrib_c = w[:, :, None] * rgb[None, :, :]           # [p,n,3]
    rev = np.cumsum(contrib_c[:, ::-1, :], axis=1)[:, ::-1, :]
    behind = rev - contrib_c + (Tf[:, None] * 1.0)[:, :, None] * bg[None, None, :]
    dC_dalpha = T[:, :, None] * rgb[None, :, :] - behind / (1.0 - alpha)[:, :, None]
    dL_dalpha = np.where(keep, np.einsum("pnc,pc->pn", dC_dalpha, g), 0.0)
    unclamped = keep & (B["raw"] <= ALPHA_MAX)
    G = B["G"]
    dL_dpow = np.where(unclamped, dL_dalpha * o[None, :] * G, 0.0)
    dx, dy = B["dx"], B["dy"]
    terms = [dL_dpow * (a[None, :] * dx + b[None, :] * dy),
             dL_dpow * (b[None, :] * dx + c[None, :] * dy),
             dL_dpow * (-0.5 * dx * dx), dL_dpow * (-dx * dy), dL_dpow * (-0.5 * dy * dy),
             np.where(unclamped, dL_dalpha * G, 0.0),
             w * g[:, 0:1], w * g[:, 1:2], w * g[:, 2:3]]
    return dict(d_mean=np.stack([terms[0].sum(axis=0), terms[1].sum(axis=0)], 1),
                d_con=np.stack([terms[2].sum(axis=0), terms[3].sum(axis=0),
                                terms[4].sum(axis=0)], 1),
                d_op=terms[5].sum(axis=0), d_rgb=np.einsum("pn,pc->nc", w, g),
                abs2d=np.stack([np.abs(t).sum(axis=0) for t in terms], 1),
                contrib=keep.any(axis=0))


def _bwd_out(n: int) -> dict:
    return dict(d_mean2d=np.zeros((n, 2)), d_conic=np.zeros((n, 3)), d_opacity=np.zeros(n),
                d_rgb=np.zeros((n, 3)), contrib=np.zeros(n, bool), abs2d=np.zeros((n, 9)))


def _bwd_add(out: dict, cand: np.ndarray, r: dict):
    """Add one block's per-candidate sums (``cand`` holds no index twice)."""
    out["d_mean2d"][cand] += r["d_mean"]
    out["d_conic"][cand] += r["d_con"]
    out["d_opacity"][cand] += r["d_op"]
    out["d_rgb"][cand] += r["d_rgb"]
    out["abs2d"][cand] += r["abs2d"]
    out["contrib"][cand] |= r["contrib"]


def render_bwd_2d(P: dict, dL_dC: np.ndarray, bg=(0.0, 0.0, 0.0), pixels=None,
                  chunk: int = 256) -> dict:
    """Gradients of L w.r.t. the per-Gaussian 2D quantities.

    ``dL_dC`` is [3,H,W] (all pixels) or [3,npix] matching ``pixels``.
    Returns d_mean2d [N,2], d_conic [N,3] (a,b,c as stored), d_opacity [N],
    d_rgb [N,3], and contrib [N] (True for Gaussians blended in some pixel).
    """
    W, H = P["width"], P["height"]
    n = P["mean2d"].shape[0]
    pix = np.arange(W * H) if pixels is None else np.asarray(pixels, np.int64)
    g_all = np.asarray(dL_dC, F64).reshape(3, -1)
    order = _order(P)
    bg = np.asarray(bg, F64)
    out = _bwd_out(n)
    for s in range(0, pix.shape[0], chunk):
        blk = pix[s:s + chunk]
        _bwd_add(out, order, _bwd_block(P, order, blk, g_all[:, s:s + len(blk)].T, bg))
    return out


# ---------------------------------------------------------------- binned form
def tile_candidates(P: dict):
    """For each tile of the view (row-major), the live Gaussians whose
    conservative footprint box covers it, in ascending (z_f32, index) order.
    Every other Gaussian has alpha < 1/255 at each of the tile's pixel
    centres, so it is skipped there: blending only these candidates gives the
    same pixels as the brute force over all Gaussians."""
    T, W, H = P["tile"], P["width"], P["height"]
    gw, gh = -(-W // T), -(-H // T)
    order = _order(P)
    order = order[P["tiles_touched"][order] > 0]
    r = P["rect"][order]
    out = []
    for ty in range(gh):
        row = order[(r[:, 1] <= ty) & (r[:, 3] >= ty)]
        rr = P["rect"][row]
        for tx in range(gw):
            out.append(row[(rr[:, 0] <= tx) & (rr[:, 2] >= tx)])
    return out


def tile_pixels(P: dict, t: int) -> np.ndarray:
    """Row-major pixel indices of tile t (ragged at the right and bottom edges)."""
    T, W, H = P["tile"], P["width"], P["height"]
    gw = -(-W // T)
    ty, tx = divmod(t, gw)
    ys = np.arange(ty * T, min(H, (ty + 1) * T))
    xs = np.arange(tx * T, min(W, (tx + 1) * T))
    return (ys[:, None] * W + xs[None, :]).ravel()


def render_fwd_binned(P: dict, bg=(0.0, 0.0, 0.0), tiles=None, cands=None) -> dict:
    """``render_fwd`` over all pixels of the given tiles (default: every tile),
    each pixel blending only its tile's candidates.  Returns image [3,npix],
    final_T, n_contrib, last_id and the guard-band flag for the pixels
    ``pixels`` (tile after tile, row-major inside each)."""
    cands = tile_candidates(P) if cands is None else cands
    tiles = range(len(cands)) if tiles is None else tiles
    bg = np.asarray(bg, F64)
    pix, img, fT, ncon, last, flag = [], [], [], [], [], []
    for t in tiles:
        blk = tile_pixels(P, t)
        cand = cands[t]
        pix.append(blk)
        if len(cand) == 0:   # nothing reaches the tile: the background
            img.append(np.repeat(bg[:, None], len(blk), axis=1))
            fT.append(np.ones(len(blk)))
            ncon.append(np.zeros(len(blk), np.int64))
            last.append(np.full(len(blk), -1, np.int64))
            flag.append(np.zeros(len(blk), bool))
            continue
        B = _pixel_block(P, cand, blk, P["width"])
        w = np.where(B["keep"], B["alpha"] * B["Tbefore"], 0.0)
        Tf = np.prod(np.where(B["keep"], 1.0 - B["alpha"], 1.0), axis=1)
        img.append((w @ P["rgb"][cand]).T + Tf[None, :] * bg[:, None])
        fT.append(Tf)
        ncon.append(B["keep"].sum(axis=1))
        has = B["keep"].any(axis=1)
        lastcol = B["keep"].shape[1] - 1 - np.argmax(B["keep"][:, ::-1], axis=1)
        last.append(np.where(has, cand[lastcol] if len(cand) else -1, -1))
        flag.append(_guard_flags(B))
    cat = lambda xs, ax=0: np.concatenate(xs, axis=ax) if xs else np.zeros(0)
    return dict(pixels=cat(pix).astype(np.int64), image=cat(img, 1).reshape(3, -1),
                final_T=cat(fT), n_contrib=cat(ncon).astype(np.int64),
                last_id=cat(last).astype(np.int64), flag=cat(flag).astype(bool))


def render_bwd_2d_binned(P: dict, dL_dC: np.ndarray, bg=(0.0, 0.0, 0.0), tiles=None,
                         cands=None) -> dict:
    """``render_bwd_2d`` with every pixel of the given tiles (default: all)
    blending only its tile's candidates; ``dL_dC`` is [3,H,W]."""
    cands = tile_candidates(P) if cands is None else cands
    tiles = range(len(cands)) if tiles is None else tiles
    g_all = np.asarray(dL_dC, F64).reshape(3, -1)
    bg = np.asarray(bg, F64)
    out = _bwd_out(P["mean2d"].shape[0])
    for t in tiles:
        blk = tile_pixels(P, t)
        if len(cands[t]):
            _bwd_add(out, cands[t], _bwd_block(P, cands[t], blk, g_all[:, blk].T, bg))
    return out


def _dR_dq(qn: np.ndarray) -> np.ndarray:
    """d R(q)_{ij} / d q_k for unit-quaternion components (w,x,y,z): [N,3,3,4]."""
    w, x, y, z = qn[:, 0], qn[:, 1], qn[:, 2], qn[:, 3]
    n = qn.shape[0]
    D = np.zeros((n, 3, 3, 4))
    # R00 = 1 - 2(y^2 + z^2)
    D[:, 0, 0, 2] = -4 * y; D[:, 0, 0, 3] = -4 * z
    # R01 = 2(xy - wz)
    D[:, 0, 1, 0] = -2 * z; D[:, 0, 1, 1] = 2 * y; D[:, 0, 1, 2] = 2 * x; D[:, 0, 1, 3] = -2 * w
    # R02 = 2(xz + wy)
    D[:, 0, 2, 0] = 2 * y; D[:, 0, 2, 1] = 2 * z; D[:, 0, 2, 2] = 2 * w; D[:, 0, 2, 3] = 2 * x
    # R10 = 2(xy + wz)
    D[:, 1, 0, 0] = 2 * z; D[:, 1, 0, 1] = 2 * y; D[:, 1, 0, 2] = 2 * x; D[:, 1, 0, 3] = 2 * w
    # R11 = 1 - 2(x^2 + z^2)
    D[:, 1, 1, 1] = -4 * x; D[:, 1, 1, 3] = -4 * z
    # R12 = 2(yz - wx)
    D[:, 1, 2, 0] = -2 * x; D[:, 1, 2, 1] = -2 * w; D[:, 1, 2, 2] = 2 * z; D[:, 1, 2, 3] = 2 * y
    # R20 = 2(xz - wy)
    D[:, 2, 0, 0] = -2 * y; D[:, 2, 0, 1] = 2 * z; D[:, 2, 0, 2] = -2 * w; D[:, 2, 0, 3] = 2 * x
    # R21 = 2(yz + wx)
    D[:, 2, 1, 0] = 2 * x; D[:, 2, 1, 1] = 2 * w; D[:, 2, 1, 2] = 2 * z; D[:, 2, 1, 3] = 2 * y
    # R22 = 1 - 2(x^2 + y^2)
    D[:, 2, 2, 1] = -4 * x; D[:, 2, 2, 2] = -4 * y
    return D


def _dcoef2(P: dict, absolute: bool = False) -> np.ndarray:
    """Symmetric 2x2 gradient of the 2D mip filter's factor c2 = sqrt(D1/D2)
    w.r.t. the projected covariance (a, b; b, c) before the low-pass h:
    d/da = c2/2 (c/D1 - (c+h)/D2), d/dc likewise, d/db = c2 b (1/D2 - 1/D1),
    split half and half over the two off-diagonal entries.  ``absolute``: the
    same with every term taken in magnitude (for the error scale)."""
    h = _proj.MIP_2D_VARIANCE
    a, b, c = P["C2raw"][:, 0], P["C2raw"][:, 1], P["C2raw"][:, 2]
    live = P["live"]
    D1 = np.where(live, a * c - b * b, 1.0)
    D2 = np.where(live, (a + h) * (c + h) - b * b, 1.0)
    c2 = P["coef2"]
    if absolute:
        A = np.abs
        da = 0.5 * c2 * (A(c) / D1 + A(c + h) / D2)
        dc = 0.5 * c2 * (A(a) / D1 + A(a + h) / D2)
        db = c2 * A(b) * (1.0 / D2 + 1.0 / D1)
    else:
        da = 0.5 * c2 * (c / D1 - (c + h) / D2)
        dc = 0.5 * c2 * (a / D1 - (a + h) / D2)
        db = c2 * b * (1.0 / D2 - 1.0 / D1)
    return np.stack([np.stack([da, 0.5 * db], -1), np.stack([0.5 * db, dc], -1)], -2)


def chain_to_3d(scene: dict, P: dict, g2: dict) -> dict:
    """Chain the 2D gradients of ``render_bwd_2d`` back to the parameters.

    Returns d_means [N,3], d_log_scales [N,3], d_quats [N,4],
    d_opacity_logits [N], d_sh [N,16,3]; rows of culled Gaussians are zero.
    """
    n = P["mean2d"].shape[0]
    live = P["live"]
    x, y, z = P["xc"][:, 0], P["xc"][:, 1], np.where(live, P["xc"][:, 2], 1.0)
    fx, fy = P["fx"], P["fy"]
    gm = g2["d_mean2d"]
    ga, gb, gc = g2["d_conic"][:, 0], g2["d_conic"][:, 1], g2["d_conic"][:, 2]
    # conic -> Sigma': dL/dSigma' = -Q G_Q Q with G_Q the symmetric gradient of Q
    a, b, c = P["conic"][:, 0], P["conic"][:, 1], P["conic"][:, 2]
    Q = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    GQ = np.stack([np.stack([ga, 0.5 * gb], -1), np.stack([0.5 * gb, gc], -1)], -2)
    GS2 = -Q @ GQ @ Q                                       # [N,2,2] symmetric
    go = g2["d_opacity"]                                    # w.r.t. the blending opacity
    o_raw, c3, c2 = P["opacity_raw"], P["coef3"], P["coef2"]
    if P["mip2d"]:
        # c2 = sqrt(D1 / D2), D1 = det(C2raw), D2 = det(C2raw + h I): its gradient
        # w.r.t. the symmetric C2raw (= w.r.t. Sigma', which differs by a constant)
        GS2 = GS2 + (go * o_raw * c3)[:, None, None] * _dcoef2(P)
    Tm, Sigma, Rc = P["Tm"], P["Sigma"], P["Rc"]
    GSigma = np.transpose(Tm, (0, 2, 1)) @ GS2 @ Tm         # [N,3,3]
    GTm = 2.0 * GS2 @ Tm @ Sigma                            # [N,2,3]
    GJ = GTm @ Rc.T                                         # [N,2,3]
    gx = gm[:, 0] * fx / z + GJ[:, 0, 2] * (-fx / (z * z))
    gy = gm[:, 1] * fy / z + GJ[:, 1, 2] * (-fy / (z * z))
    gz = (gm[:, 0] * (-fx * x / (z * z)) + gm[:, 1] * (-fy * y / (z * z))
          + GJ[:, 0, 0] * (-fx / (z * z)) + GJ[:, 0, 2] * (2.0 * fx * x / (z ** 3))
          + GJ[:, 1, 1] * (-fy / (z * z)) + GJ[:, 1, 2] * (2.0 * fy * y / (z ** 3)))
    gxc = np.stack([gx, gy, gz], 1)
    d_means = gxc @ Rc                                      # R^T g, row form
    # Sigma = M M^T, M = Rq diag(s)
    s, Rq = P["scales"], P["Rq"]
    M = Rq * s[:, None, :]
    GM = 2.0 * GSigma @ M
    gs = np.einsum("nik,nik->nk", GM, Rq)
    d_ls = gs * s
    if P["has_filter3d"]:
        # c3 = prod_i s_i / sqrt(s_i^2 + f): d c3 / d log s_i = c3 f / (s_i^2 + f)
        f3 = P["f3"][:, None]
        d_ls = d_ls + (go * o_raw * c2 * c3)[:, None] * f3 / (s * s + f3)
    GR = GM * s[:, None, :]
    gqn = np.einsum("nij,nijk->nk", GR, _dR_dq(P["qn"]))
    qn = P["qn"]
    d_q = (gqn - qn * np.sum(qn * gqn, axis=1, keepdims=True)) / P["qnorm"][:, None]
    d_logit = go * c3 * c2 * o_raw * (1.0 - o_raw)
    # colour: rgb = max(0, sum_k sh_k Y_k(d) + 0.5); clamped channels pass nothing
    deg = P["sh_degree"]
    K = _sh.n_coeffs(deg)
    grgb = np.where(P["rgb_raw"] < 0.0, 0.0, g2["d_rgb"])     # [N,3]
    d_sh = np.zeros((n, 16, 3))
    d_sh[:, :K, :] = P["Y"][:, :, None] * grgb[:, None, :]
    dY = _sh.basis_grad(P["dirs"], deg)                     # [N,K,3]
    shc = np.asarray(scene["sh"], F64)[:, :K, :]
    gdir = np.einsum("nc,nkc,nkj->nj", grgb, shc, dY)
    d = P["dirs"]
    proj_d = gdir - d * np.sum(d * gdir, axis=1, keepdims=True)
    d_means = d_means + proj_d / P["dist"][:, None]
    out = dict(d_means=d_means, d_log_scales=d_ls, d_quats=d_q, d_opacity_logits=d_logit,
               d_sh=d_sh)
    for k in out:
        out[k][~live] = 0.0
    return out


def chain_abs_bound(scene: dict, P: dict, abs2d: np.ndarray) -> dict:
    """Running error scale of every parameter gradient.

    ``chain_to_3d`` evaluated on absolute values: every input, matrix entry
    and intermediate replaced by its magnitude and every difference by a sum,
    fed with the per-Gaussian sums over pixels of the absolute 2D terms
    (``abs2d``).  The result bounds the sum of the magnitudes of all products
    that a floating-point evaluation adds up into each gradient element, so a
    float32 result that cancels from large terms has an error proportional to
    it (the usual forward error bound |fl(s) - s| <= gamma * sum |terms|).
    """
    n = P["mean2d"].shape[0]
    A = np.abs
    x, y = A(P["xc"][:, 0]), A(P["xc"][:, 1])
    z = np.where(P["live"], P["xc"][:, 2], 1.0)
    fx, fy = P["fx"], P["fy"]
    gm = abs2d[:, 0:2]
    ga, gb, gc = abs2d[:, 2], abs2d[:, 3], abs2d[:, 4]
    a, b, c = A(P["conic"][:, 0]), A(P["conic"][:, 1]), A(P["conic"][:, 2])
    Q = np.stack([np.stack([a, b], -1), np.stack([b, c], -1)], -2)
    GQ = np.stack([np.stack([ga, 0.5 * gb], -1), np.stack([0.5 * gb, gc], -1)], -2)
    GS2 = Q @ GQ @ Q
    go = abs2d[:, 5]
    o_raw, c3, c2 = P["opacity_raw"], P["coef3"], P["coef2"]
    if P["mip2d"]:
        GS2 = GS2 + (go * o_raw * c3)[:, None, None] * _dcoef2(P, absolute=True)
    Tm, Sigma, Rc = A(P["Tm"]), A(P["Sigma"]), A(P["Rc"])
    GSigma = np.transpose(Tm, (0, 2, 1)) @ GS2 @ Tm
    GJ = (2.0 * GS2 @ Tm @ Sigma) @ Rc.T
    gx = gm[:, 0] * fx / z + GJ[:, 0, 2] * fx / (z * z)
    gy = gm[:, 1] * fy / z + GJ[:, 1, 2] * fy / (z * z)
    gz = (gm[:, 0] * fx * x / (z * z) + gm[:, 1] * fy * y / (z * z)
          + GJ[:, 0, 0] * fx / (z * z) + GJ[:, 0, 2] * 2.0 * fx * x / z ** 3
          + GJ[:, 1, 1] * fy / (z * z) + GJ[:, 1, 2] * 2.0 * fy * y / z ** 3)
    d_means = np.stack([gx, gy, gz], 1) @ Rc
    s, Rq = P["scales"], A(P["Rq"])
    M = Rq * s[:, None, :]
    GM = 2.0 * GSigma @ M
    d_ls = np.einsum("nik,nik->nk", GM, Rq) * s
    if P["has_filter3d"]:
        f3 = P["f3"][:, None]
        d_ls = d_ls + (go * o_raw * c2 * c3)[:, None] * f3 / (s * s + f3)
    GR = GM * s[:, None, :]
    qn = A(P["qn"])
    gqn = np.einsum("nij,nijk->nk", GR, A(_dR_dq(P["qn"])))
    d_q = (gqn + qn * np.sum(qn * gqn, axis=1, keepdims=True)) / P["qnorm"][:, None]
    d_logit = go * c3 * c2 * o_raw * (1.0 - o_raw)
    deg = P["sh_degree"]
    K = _sh.n_coeffs(deg)
    grgb = abs2d[:, 6:9]
    d_sh = np.zeros((n, 16, 3))
    d_sh[:, :K, :] = A(P["Y"])[:, :, None] * grgb[:, None, :]
    dY = A(_sh.basis_grad(P["dirs"], deg))
    shc = A(np.asarray(scene["sh"], F64)[:, :K, :])
    gdir = np.einsum("nc,nkc,nkj->nj", grgb, shc, dY)
    d = A(P["dirs"])
    d_means = d_means + (gdir + d * np.sum(d * gdir, axis=1, keepdims=True)) / P["dist"][:, None]
    out = dict(d_means=d_means, d_log_scales=d_ls, d_quats=d_q, d_opacity_logits=d_logit,
               d_sh=d_sh)
    for k in out:
        out[k][~P["live"]] = 0.0
    return out


def render_bwd(scene: dict, P: dict, dL_dC: np.ndarray, bg=(0.0, 0.0, 0.0), pixels=None,
               chunk: int = 256, with_bound: bool = False) -> dict:
    """Full backward: 2D gradients then the chain to the parameters.

    With ``with_bound`` also returns ``bound``: the per-element term scale of
    ``chain_abs_bound`` for every parameter gradient.
    """
    g2 = render_bwd_2d(P, dL_dC, bg=bg, pixels=pixels, chunk=chunk)
    out = chain_to_3d(scene, P, g2)
    out["g2d"] = g2
    if with_bound:
        out["bound"] = chain_abs_bound(scene, P, g2["abs2d"])
    return out


def loss_weighted(scene: dict, cam, w: np.ndarray, tile: int = 16, sh_degree: int = 3,
                  bg=(0.0, 0.0, 0.0), mip2d: bool = False, filter3d=None) -> float:
    """L = sum(w * C) over all pixels: the O(1) scalar used for finite differences."""
    P = _proj.project(scene, cam, tile=tile, sh_degree=sh_degree, mip2d=mip2d,
                      filter3d=filter3d)
    C = render_fwd(P, bg=bg)["image"]
    return float(np.sum(np.asarray(w, F64) * C))
