"""FP64 oracle of the frequency-guided resolution schedule (Sec. 4.2, Eq. 2
and the supplementary's Eq. 6-7) and of the anti-aliased ground-truth
downsampling (supplementary, "Ground Truth Downsampling").

Test infrastructure only: imported by tests/ and bench.py's CPU baseline,
never by the product path.  numpy's FFT serves as the DFT (a library step);
everything else is written out from the definitions.

Readings (the paper leaves these open):
* An image's frequency norm ||F(i,j)||_2 is taken over the colour channels:
  sqrt(sum_c |DFT(I_c)(i,j)|^2), with the unnormalised forward DFT.
* The spectrum of a view downsampled by r (anti-aliased, Sec. 4.1) is the
  central (H/r) x (W/r) crop of the full spectrum scaled by 1/r^2: the ideal
  low-pass downsample.  So X(F_r) is a crop sum of the full-resolution mean
  magnitude map M; the crop keeps the frequencies with |k_y| <= H/(2r) and
  |k_x| <= W/(2r).  Two normalisations: "sum" takes Eq. 2 literally with the
  unnormalised DFT, X(F_r) = (1/r^2) sum_crop M; "mean" normalises each
  view's DFT by its own pixel count (h w), X(F_r) = sum_crop M / (H W).  Under
  "sum", a 1/f amplitude spectrum gives X(F_r) ~ r^-3, so X(F_{r_m}) = X(F)/a
  puts r_m near a^(1/3) (1.6 for a = 4) and floor(r) never leaves 1; under
  "mean", X(F_r) ~ 1/r and r_m is near a.  X(F_r) is non-increasing in r
  either way.
* r_m is the largest r with X(F_r) >= X(F)/a, and likewise r_i for the knot
  values X_i: "solve" means the boundary of the superlevel set, found by
  bisection on [1, r_max].
* The knots' values X_i are the targets themselves: X(F_{r_i}) = X_i by the
  construction of r_i, so Eq. 7 gives s_{r_i} = S ln(X_i / X_m) / ln(X_F / X_m),
  with s_{r_m} = 0 and s = S at r_0 = 1.
* The number of knots m is a parameter (default 4).
* Between knots, 1/r^2 is linear in the iteration (the "inverse square"
  interpolation); the render uses the integer factor floor(r).
"""
from __future__ import annotations

import numpy as np


# ------------------------------------------------------------------ Eq. 2
def magnitude_map(images) -> np.ndarray:
    """M(i,j) = (1/N) sum_n ||F^n(i,j)||_2 over views [N, C, H, W] (or one
    [C, H, W]); F^n is the unnormalised 2D DFT, the norm runs over channels.
    Returned with the zero frequency at the centre (index H//2, W//2)."""
    x = np.asarray(images, dtype=np.float64)
    if x.ndim == 3:
        x = x[None]
    F = np.fft.fft2(x, axes=(-2, -1))
    mag = np.sqrt((np.abs(F) ** 2).sum(axis=1))   # norm over channels
    return np.fft.fftshift(mag.mean(axis=0), axes=(-2, -1))


def significance(images) -> float:
    """X(F) of Eq. 2 at the images' own resolution."""
    return float(magnitude_map(images).sum())


def crop_significance(M: np.ndarray, r: float, norm: str = "sum") -> float:
    """X(F_r) under the crop reading: the sum of M over the frequencies with
    |k_y| <= H/(2r) and |k_x| <= W/(2r), times 1/r^2 ("sum") or 1/(H W)
    ("mean")."""
    H, W = M.shape
    ky = np.arange(H) - H // 2
    kx = np.arange(W) - W // 2
    sel_y = np.abs(ky) <= H / (2.0 * r)
    sel_x = np.abs(kx) <= W / (2.0 * r)
    total = float(M[np.ix_(sel_y, sel_x)].sum())
    return total / (r * r) if norm == "sum" else total / (H * W)


def solve_r(M: np.ndarray, target: float, r_max: float, iters: int = 60,
            norm: str = "sum") -> float:
    """Largest r in [1, r_max] with X(F_r) >= target (bisection; X is
    non-increasing in r).  r_max when even X(F_{r_max}) >= target."""
    if crop_significance(M, r_max, norm) >= target:
        return float(r_max)
    lo, hi = 1.0, float(r_max)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if crop_significance(M, mid, norm) >= target:
            lo = mid
        else:
            hi = mid
    return lo


# ------------------------------------------------------------ Eq. 6 and 7
def schedule_knots(M: np.ndarray, S: int, a: float = 4.0, m: int = 4, r_max: float | None = None,
                   norm: str = "sum"):
    """Knots (r_i, s_{r_i}) for i = 0..m, with r_0 = 1 at s = S and r_m at s = 0.

    X_F = X(F); r_m solves X(F_{r_m}) = X_F / a; the values X_1..X_{m-1} are
    spaced linearly between X_F and X_m and solved for r_i; Eq. 7 places them
    at s_{r_i} = S ln(X_i / X_m) / ln(X_F / X_m)."""
    H, W = M.shape
    if r_max is None:
        r_max = float(min(H, W))
    XF = crop_significance(M, 1.0, norm)
    Xm = XF / a
    X = [XF - (XF - Xm) * i / m for i in range(m + 1)]
    r = [1.0] + [solve_r(M, X[i], r_max, norm=norm) for i in range(1, m + 1)]
    s = [S * np.log(X[i] / Xm) / np.log(XF / Xm) for i in range(m + 1)]
    return np.array(r), np.array(s), np.array(X)


def resolution_at(k: float, r_knots, s_knots) -> float:
    """r(k): 1/r^2 linear in k between consecutive knots (s decreasing in i);
    1 from s_0 = S on."""
    r = np.asarray(r_knots, np.float64)
    s = np.asarray(s_knots, np.float64)
    if k >= s[0]:
        return 1.0
    for i in range(1, len(r)):
        if k >= s[i]:
            t = (k - s[i]) / (s[i - 1] - s[i])
            inv2 = 1.0 / r[i] ** 2 + t * (1.0 / r[i - 1] ** 2 - 1.0 / r[i] ** 2)
            return float(1.0 / np.sqrt(inv2))
    return float(r[-1])


def render_factor(k: float, r_knots, s_knots) -> int:
    """The integer downsampling factor rendered at iteration k: floor(r(k))."""
    return int(np.floor(resolution_at(k, r_knots, s_knots)))


# ------------------------------------------------- ground-truth downsampling
def aa_weights(n_in: int, n_out: int) -> np.ndarray:
    """Rows of the separable anti-aliased linear resampling from n_in to n_out
    samples: output i is centred at input coordinate (i + 0.5) n_in / n_out
    (pixel centres at j + 0.5); a triangle of half-width max(1, n_in / n_out)
    input pixels weighs the inputs, normalised to sum 1."""
    s = n_in / n_out
    half = max(s, 1.0)
    Wm = np.zeros((n_out, n_in))
    j = np.arange(n_in)
    for i in range(n_out):
        t = ((j + 0.5) - (i + 0.5) * s) / half
        w = np.maximum(0.0, 1.0 - np.abs(t))
        Wm[i] = w / w.sum()
    return Wm


def downsample_aa(img, h: int, w: int) -> np.ndarray:
    """[C, H, W] -> [C, h, w] anti-aliased resize: Wy @ I_c @ Wx^T per channel."""
    x = np.asarray(img, dtype=np.float64)
    Wy, Wx = aa_weights(x.shape[1], h), aa_weights(x.shape[2], w)
    return np.stack([Wy @ x[c] @ Wx.T for c in range(x.shape[0])])


# --------------------------------------------- the position learning rate
def position_lr(k: int, factors, lr_init: float, lr_final: float) -> float:
    """Learning rate of the Gaussian means at iteration k (supplementary,
    "Learning Rate"): held at its initial value during the low-resolution
    stage and allowed to decay only from i* = argmin_i {floor(r^(i)) = 1}.

    ``factors`` is the integer factor floor(r^(i)) rendered at each of the S
    iterations i = 0..S-1.  Reading (the paper names the switch point, not
    the decay): from i* on, the rate decays as in the 3DGS backbone, the
    exponential (log-linear) interpolation from lr_init to lr_final, here
    spread over the remaining iterations, so that it reaches lr_final at
    i = S.  Without a full-resolution iteration the rate never decays."""
    f = np.asarray(factors)
    S = f.shape[0]
    full = [i for i in range(S) if int(f[i]) == 1]
    if not full or k <= full[0]:
        return float(lr_init)
    i_star = full[0]
    t = (k - i_star) / (S - i_star)
    return float(np.exp((1.0 - t) * np.log(lr_init) + t * np.log(lr_final)))
