"""Pins of the resolution-schedule oracle (Sec. 4.2, Eq. 2, Eq. 6-7) and of
its anti-aliased downsampling, against closed forms, an exactly sampled
band-limited signal and torch's CPU resize (a library routine)."""
import math

import numpy as np
import pytest
import torch

from oracle import schedule as O


def test_constant_image_has_only_the_dc_term():
    H, W = 24, 40
    c = np.array([0.2, 0.5, 0.7])
    img = np.broadcast_to(c[:, None, None], (3, H, W))
    M = O.magnitude_map(img)
    assert M[H // 2, W // 2] == pytest.approx(H * W * np.linalg.norm(c), rel=1e-12)
    assert O.significance(img) == pytest.approx(H * W * np.linalg.norm(c), rel=1e-12)


def test_single_cosine_two_peaks():
    H, W, u, v = 32, 48, 5, 3
    y, x = np.mgrid[0:H, 0:W]
    img = np.zeros((3, H, W))
    img[1] = np.cos(2 * np.pi * (u * x / W + v * y / H))
    M = O.magnitude_map(img)
    assert M[H // 2 + v, W // 2 + u] == pytest.approx(H * W / 2, rel=1e-12)
    assert M[H // 2 - v, W // 2 - u] == pytest.approx(H * W / 2, rel=1e-12)
    assert O.significance(img) == pytest.approx(H * W, rel=1e-12)


def test_views_are_averaged():
    rng = np.random.default_rng(0)
    a, b = rng.uniform(size=(3, 16, 20)), rng.uniform(size=(3, 16, 20))
    assert O.significance(np.stack([a, b])) == pytest.approx(
        0.5 * (O.significance(a) + O.significance(b)), rel=1e-12)


@pytest.mark.parametrize("r", [2, 4])
@pytest.mark.parametrize("norm", ["sum", "mean"])
def test_crop_equals_ideal_downsample_of_band_limited_image(r, norm):
    """A sum of cosines below the coarse grid's Nyquist limit, sampled on the
    full and on the r-times coarser pixel grid (same continuous image): the
    coarse image's X equals the full spectrum's crop scaled by 1/r^2 (or, with
    each DFT normalised by its pixel count, by 1/(H W))."""
    H, W = 64, 96
    rng = np.random.default_rng(1)
    waves = [(rng.integers(0, W // (2 * r) - 1), rng.integers(0, H // (2 * r) - 1),
              rng.uniform(0.2, 1.0), rng.uniform(0, 2 * np.pi), rng.integers(0, 3))
             for _ in range(6)]

    def sample(h, w):
        y, x = np.mgrid[0:h, 0:w]
        img = np.zeros((3, h, w))
        for (u, v, amp, ph, ch) in waves:   # frequencies in cycles per image
            img[ch] += amp * np.cos(2 * np.pi * (u * (x + 0.5) / w + v * (y + 0.5) / h) + ph)
        return img + 0.3

    M = O.magnitude_map(sample(H, W))
    coarse = O.significance(sample(H // r, W // r))
    if norm == "mean":   # each view's DFT normalised by its own pixel count
        coarse /= (H // r) * (W // r)
    assert O.crop_significance(M, float(r), norm) == pytest.approx(coarse, rel=1e-10)


def test_crop_at_one_is_the_full_sum_and_nonincreasing():
    rng = np.random.default_rng(2)
    M = O.magnitude_map(rng.uniform(size=(2, 3, 45, 60)))
    assert O.crop_significance(M, 1.0) == pytest.approx(M.sum(), rel=1e-12)
    rs = np.linspace(1.0, 20.0, 400)
    xs = np.array([O.crop_significance(M, r) for r in rs])
    assert np.all(np.diff(xs) <= 1e-9 * xs[0])


@pytest.mark.parametrize("norm", ["sum", "mean"])
def test_knots_follow_eq7(norm):
    rng = np.random.default_rng(3)
    img = rng.uniform(size=(3, 64, 96))
    M = O.magnitude_map(img)
    S, a, m = 6000, 4.0, 4
    r, s, X = O.schedule_knots(M, S, a=a, m=m, norm=norm)
    assert r[0] == 1.0 and s[0] == pytest.approx(S) and s[-1] == pytest.approx(0.0, abs=1e-9)
    assert np.all(np.diff(r) >= 0) and np.all(np.diff(s) < 0)
    # Eq. 7 with linearly spaced X_i depends only on a and m
    for i in range(m + 1):
        assert s[i] == pytest.approx(S * math.log(a * (1 - i / m * (1 - 1 / a))) / math.log(a),
                                     rel=1e-12, abs=1e-9)
    # r_i is the boundary of {r : X(F_r) >= X_i}
    for i in range(1, m + 1):
        assert O.crop_significance(M, r[i], norm) >= X[i]
        assert O.crop_significance(M, r[i] * (1 + 1e-6), norm) < X[i]


def test_resolution_curve():
    r = np.array([1.0, 1.5, 2.5, 4.0])
    s = np.array([900.0, 500.0, 200.0, 0.0])
    assert O.resolution_at(0, r, s) == pytest.approx(4.0)
    for i in range(4):
        assert O.resolution_at(s[i], r, s) == pytest.approx(r[i])
    assert O.resolution_at(1e6, r, s) == 1.0
    mid = O.resolution_at(350.0, r, s)     # halfway between knots 2 and 1 in 1/r^2
    assert 1 / mid ** 2 == pytest.approx(0.5 * (1 / 2.5 ** 2 + 1 / 1.5 ** 2))
    ks = np.arange(0, 1000)
    rr = np.array([O.resolution_at(k, r, s) for k in ks])
    assert np.all(np.diff(rr) <= 1e-12)
    assert O.render_factor(0, r, s) == 4 and O.render_factor(950, r, s) == 1


@pytest.mark.parametrize("H,W,h,w", [(96, 128, 48, 64), (133, 200, 33, 50), (97, 131, 31, 17),
                                     (64, 64, 64, 64), (40, 30, 80, 45)])
def test_downsample_matches_torch_antialias(H, W, h, w):
    x = np.random.default_rng(4).uniform(size=(3, H, W))
    ref = torch.nn.functional.interpolate(torch.from_numpy(x)[None], size=(h, w), mode="bilinear",
                                          antialias=True, align_corners=False)[0].numpy()
    assert np.abs(O.downsample_aa(x, h, w) - ref).max() < 1e-12


def test_downsample_keeps_constants():
    x = np.full((3, 50, 70), 0.25)
    assert np.abs(O.downsample_aa(x, 7, 9) - 0.25).max() < 1e-15


def test_one_over_f_spectrum_places_r_m():
    """Amplitude 1/|f| (natural-image statistics), no DC: X(F_r) ~ r^-3 under
    "sum" and ~ r^-1 under "mean", so r_m is near a^(1/3) and a."""
    H = W = 512
    ky = np.arange(H) - H // 2
    kx = np.arange(W) - W // 2
    f = np.hypot(*np.meshgrid(ky, kx, indexing="ij"))
    M = np.where(f > 0, 1.0 / np.maximum(f, 1e-12), 0.0)
    r_sum = O.schedule_knots(M, 100, a=4.0, m=1, norm="sum")[0][1]
    r_mean = O.schedule_knots(M, 100, a=4.0, m=1, norm="mean")[0][1]
    assert r_sum == pytest.approx(4.0 ** (1 / 3), rel=0.05)
    assert r_mean == pytest.approx(4.0, rel=0.05)


# ---- the position learning rate (supplementary, "Learning Rate")
LR0, LR1 = 1.6e-4, 1.6e-6


def test_position_lr_is_held_until_the_first_full_resolution_iteration():
    # a schedule of 4 -> 2 -> 1 with the first full-resolution iteration at 60
    factors = [4] * 25 + [3] * 10 + [2] * 25 + [1] * 40
    S = len(factors)
    i_star = next(i for i, f in enumerate(factors) if f == 1)   # brute-force argmin
    assert i_star == 60
    for k in range(i_star + 1):
        assert O.position_lr(k, factors, LR0, LR1) == LR0
    assert O.position_lr(i_star + 1, factors, LR0, LR1) < LR0
    # decays monotonically and reaches the final value at the end
    lrs = [O.position_lr(k, factors, LR0, LR1) for k in range(i_star, S + 1)]
    assert all(b < a for a, b in zip(lrs, lrs[1:]))
    assert lrs[-1] == pytest.approx(LR1, rel=1e-12)


def test_position_lr_decay_is_log_linear():
    # the backbone's decay is exponential: log(lr) is linear in the iteration,
    # so the midpoint of the decaying stretch sits at the geometric mean
    factors = [2] * 20 + [1] * 80
    mid = 20 + 40
    assert O.position_lr(mid, factors, LR0, LR1) == pytest.approx(math.sqrt(LR0 * LR1), rel=1e-12)
    logs = np.log([O.position_lr(k, factors, LR0, LR1) for k in range(20, 101)])
    assert np.abs(np.diff(logs, 2)).max() < 1e-12
    # a linear decay would put the midpoint at the arithmetic mean instead
    assert abs(O.position_lr(mid, factors, LR0, LR1) - 0.5 * (LR0 + LR1)) > 1e-5


def test_position_lr_special_cases():
    # every iteration at full resolution: the backbone's decay from iteration 0,
    # lr0 (lr1 / lr0)^(k / S)
    S = 50
    for k in (0, 1, 17, 49, 50):
        want = LR0 * (LR1 / LR0) ** (k / S)
        assert O.position_lr(k, [1] * S, LR0, LR1) == pytest.approx(want, rel=1e-12)
    # never at full resolution: the rate is never allowed to decay
    assert all(O.position_lr(k, [2] * S, LR0, LR1) == LR0 for k in range(S + 1))
