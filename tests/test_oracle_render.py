"""Pins for the oracle's blend (Sec. 3, Eq. 1) and its backward (CPU only).

Closed forms: one isotropic Gaussian on the optical axis (value and
gradients), two coincident Gaussians, a stack of alpha = 0.5 Gaussians (the
T < 1e-4 exit blends exactly 13), the 1/255 cutoff ring.  Invariants: the
blend weights sum to 1 - T_final; shuffling the input order changes nothing.
Backward: central finite differences of the FP64 forward on tiny scenes.
"""
import math

import numpy as np
import pytest

from oracle import project, render
from paper_2503_18402_amd import scenes

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def _stack(n, d=3.0, s=0.05, logit=0.0, dc=1.0, W=33, H=33, f=40.0, cx=None):
    sc = dict(means=np.zeros((n, 3), np.float32),
              log_scales=np.full((n, 3), math.log(s), np.float32),
              quats=np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1)),
              opacity_logits=np.full(n, logit, np.float32),
              sh=np.zeros((n, 16, 3), np.float32))
    sc["sh"][:, 0, :] = dc
    cam = scenes.look_at((0, 0, -d), (0, 0, 0), W, H, f)
    if cx is not None:
        cam.cx = cam.cy = cx
    return sc, cam


def test_single_isotropic_value():
    d, s, f, dc = 3.0, 0.05, 40.0, 0.8
    sc, cam = _stack(1, d, s, logit=0.3, dc=dc, W=32, H=32, f=f)
    P = project.project(sc, cam)
    out = render.render_fwd(P)
    s32 = math.exp(float(np.float32(math.log(s))))
    var = (f * s32 / d) ** 2 + 0.3
    o = 1 / (1 + math.exp(-float(np.float32(0.3))))
    c = max(0.0, Y00 * float(np.float32(dc)) + 0.5)
    py, px = np.mgrid[0:32, 0:32]
    r2 = (px + 0.5 - 16) ** 2 + (py + 0.5 - 16) ** 2
    a = np.minimum(0.99, o * np.exp(-r2 / (2 * var)))
    a = np.where(a >= 1 / 255, a, 0.0)
    for ch in range(3):
        assert np.abs(out["image"][ch] - a * c).max() < 1e-14
    assert np.abs(out["final_T"] - (1 - a)).max() < 1e-14


def test_two_coincident():
    sc, cam = _stack(2, logit=0.5, cx=16.5, W=33, H=33)
    sc["sh"][1, 0, :] = [0.2, -0.3, 0.9]
    P = project.project(sc, cam)
    out = render.render_fwd(P)
    a = P["opacity"][0]  # both have G = 1 at the centre pixel, below the 0.99 clamp
    c1, c2 = P["rgb"][0], P["rgb"][1]
    expect = a * c1 + (1 - a) * a * c2
    assert np.abs(out["image"][:, 16, 16] - expect).max() < 1e-14
    assert out["n_contrib"][16, 16] == 2
    assert out["last_id"][16, 16] == 1


def test_half_alpha_stack_blends_13():
    # G = 1 at the centre pixel and o = 0.5: after k blends T = 2^-k; the 14th would
    # take T to 6.1e-5 < 1e-4 and is not blended (exclude-then-stop).
    sc, cam = _stack(24, logit=0.0, dc=1.0, cx=16.5)
    P = project.project(sc, cam)
    out = render.render_fwd(P, pixels=[16 * 33 + 16], want_lists=True)
    assert out["n_contrib"][0] == 13
    assert list(out["lists"][0]) == list(range(13))
    c = Y00 * 1.0 + 0.5
    assert abs(out["image"][0, 0] - c * (1 - 2.0 ** -13)) < 1e-15
    assert abs(out["final_T"][0] - 2.0 ** -13) < 1e-18


def test_cutoff_ring():
    d, s, f = 3.0, 0.2, 40.0
    sc, cam = _stack(1, d, s, logit=0.0, W=64, H=64, f=f)
    P = project.project(sc, cam)
    out = render.render_fwd(P)
    var = P["cov2d"][0, 0]
    py, px = np.mgrid[0:64, 0:64]
    r2 = (px + 0.5 - 32) ** 2 + (py + 0.5 - 32) ** 2
    bound = 2 * var * math.log(127.5)
    blended = out["n_contrib"] > 0
    assert np.all(blended[r2 < 0.999 * bound])
    assert not np.any(blended[r2 > 1.001 * bound])
    assert blended.sum() > 20


def test_weights_sum_and_white():
    sc, cam = scenes.small_scene()
    sc = scenes.subset(sc, slice(0, 600))
    sc["sh"][:] = 0.0
    sc["sh"][:, 0, :] = 0.5 / Y00          # every colour the same c (= 1 up to float32)
    P = project.project(sc, cam)
    c = P["rgb"][0, 0]
    assert np.all(P["rgb"] == c) and abs(c - 1.0) < 1e-6
    out = render.render_fwd(P)
    # sum_i alpha_i T_i = 1 - T_final, so C = c (1 - T_final)
    err = np.abs(out["image"] - c * (1.0 - out["final_T"])[None]).max()
    assert err < 1e-12
    assert (out["n_contrib"] > 0).mean() > 0.3


def test_background():
    sc, cam = scenes.small_scene()
    sc = scenes.subset(sc, slice(0, 300))
    P = project.project(sc, cam)
    a = render.render_fwd(P)
    bg = (0.2, 0.5, 0.9)
    b = render.render_fwd(P, bg=bg)
    for ch in range(3):
        assert np.abs(b["image"][ch] - a["image"][ch] - bg[ch] * a["final_T"]).max() < 1e-14


def test_permutation_invariance():
    sc, cam = scenes.small_scene()
    # keep Gaussians whose float32 depths are distinct, so the order is fully determined
    # (equal depths would be ordered by index, which a shuffle changes)
    z = project.project(sc, cam)["depth_f32"]
    _, first, counts = np.unique(z, return_index=True, return_counts=True)
    uniq = np.sort(first[counts == 1])[:800]
    sc = scenes.subset(sc, uniq)
    P = project.project(sc, cam)
    assert len(np.unique(P["depth_f32"])) == 800
    out = render.render_fwd(P)
    perm = np.random.default_rng(1).permutation(800)
    P2 = project.project(scenes.subset(sc, perm), cam)
    out2 = render.render_fwd(P2)
    assert np.array_equal(out["image"], out2["image"])
    assert np.array_equal(out["final_T"], out2["final_T"])
    ids = np.where(out2["last_id"] >= 0, perm[np.maximum(out2["last_id"], 0)], -1)
    assert np.array_equal(ids, out["last_id"])


def _single_grad_setup():
    d, s, f = 3.0, 0.05, 40.0
    sc, cam = _stack(1, d, s, logit=-0.4, dc=0.7, W=32, H=32, f=f)
    return sc, cam, d, f


def test_single_isotropic_gradients_closed_form():
    sc, cam, d, f = _single_grad_setup()
    # upstream: red channel of one pixel on the +x axis of the centre (dx = 2.5, dy = 0)
    px, py = 18, 15
    g = np.zeros((3, 32, 32))
    g[0, py, px] = 1.0
    dx = px + 0.5 - 16.0
    cam.cy = 15.5
    P = project.project(sc, cam)
    dy = py + 0.5 - 15.5
    assert dy == 0.0
    B = render.render_bwd(sc, P, g)
    s = float(P["scales"][0, 0])
    var = P["cov2d"][0, 0]
    o = P["opacity"][0]
    G = math.exp(-dx * dx / (2 * var))
    c = P["rgb"][0, 0]
    C = o * G * c
    assert abs(B["d_means"][0, 0] - C * dx * (f / d) / var) < 1e-12
    assert abs(B["d_log_scales"][0, 0] - C * dx * dx * (f * s / d) ** 2 / var ** 2) < 1e-12
    assert abs(B["d_log_scales"][0, 2]) < 1e-14
    assert abs(B["d_opacity_logits"][0] - c * G * o * (1 - o)) < 1e-12
    assert abs(B["d_sh"][0, 0, 0] - o * G * Y00) < 1e-12
    assert np.abs(B["d_sh"][0, 0, 1:]).max() == 0.0


def _fd_check(sc, cam, seed, tol=1e-6, bg=(0.0, 0.0, 0.0)):
    w = np.random.default_rng(seed).uniform(-1, 1, size=(3, cam.height, cam.width))
    P = project.project(sc, cam)
    F = render.render_fwd(P, bg=bg)
    assert not F["flag"].any()
    B = render.render_bwd(sc, P, w, bg=bg)
    sc64 = {k: v.astype(np.float64) for k, v in sc.items()}
    names = [("means", "d_means"), ("log_scales", "d_log_scales"), ("quats", "d_quats"),
             ("opacity_logits", "d_opacity_logits"), ("sh", "d_sh")]
    worst = 0.0
    for pn, gn in names:
        flat = sc64[pn].reshape(-1)
        gflat = B[gn].reshape(-1)
        for j in range(flat.shape[0]):
            h = 1e-6 * max(1.0, abs(flat[j]))
            old = flat[j]
            flat[j] = old + h
            lp = render.loss_weighted(sc64, cam, w, bg=bg)
            flat[j] = old - h
            lm = render.loss_weighted(sc64, cam, w, bg=bg)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            err = abs(fd - gflat[j])
            assert err <= tol * max(1.0, abs(fd)), (pn, j, fd, gflat[j])
            worst = max(worst, err)
    return worst


def test_fd_single_anisotropic():
    sc = scenes.make_scene(1, seed=11, mean_range=0.2, ls_mu=-2.5, ls_sigma=0.4, rest_sigma=0.2)
    cam = scenes.look_at((0.4, -0.3, -2.5), (0, 0, 0), 20, 16, 24.0)
    _fd_check(sc, cam, seed=1)


def test_fd_few_gaussians_overlapping():
    sc = scenes.make_scene(4, seed=12, mean_range=0.25, ls_mu=-2.3, ls_sigma=0.3, rest_sigma=0.2)
    sc["opacity_logits"][:] = [-0.5, 0.2, -1.0, 0.4]
    cam = scenes.look_at((0.2, 0.1, -2.5), (0, 0, 0), 24, 24, 30.0)
    _fd_check(sc, cam, seed=2, bg=(0.3, 0.1, 0.6))


@pytest.mark.slow
def test_fd_eight_gaussians():
    sc = scenes.make_scene(8, seed=13, mean_range=0.3, ls_mu=-2.4, ls_sigma=0.3, rest_sigma=0.2)
    cam = scenes.look_at((-0.3, 0.2, -2.6), (0, 0, 0), 32, 32, 36.0)
    _fd_check(sc, cam, seed=3)


def test_clamped_alpha_has_zero_gradient():
    # o*G > 0.99 at the centre pixel: that pixel passes nothing to opacity / shape
    sc, cam = _stack(1, logit=6.0, cx=16.5)
    P = project.project(sc, cam)
    g = np.zeros((3, 33, 33))
    g[:, 16, 16] = 1.0
    B = render.render_bwd(sc, P, g)
    assert B["g2d"]["d_opacity"][0] == 0.0
    assert np.all(B["g2d"]["d_conic"][0] == 0.0)
    assert B["g2d"]["d_rgb"][0, 0] == pytest.approx(0.99)


def test_error_scale_bounds_every_gradient():
    # the absolute-value chain dominates the gradient it accompanies, element by element
    sc = scenes.make_scene(6, seed=14, mean_range=0.3, ls_mu=-2.4, ls_sigma=0.3, rest_sigma=0.2)
    cam = scenes.look_at((0.2, -0.1, -2.6), (0, 0, 0), 32, 28, 36.0)
    P = project.project(sc, cam)
    w = np.random.default_rng(6).uniform(-1, 1, size=(3, 28, 32))
    B = render.render_bwd(sc, P, w, with_bound=True)
    for k in ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_sh"):
        assert np.all(B["bound"][k] >= np.abs(B[k]) * (1 - 1e-12))
    # one Gaussian seen by one pixel: the 2D term magnitudes are the 2D gradients themselves
    g = np.zeros((3, 28, 32))
    g[0, 14, 16] = 1.0
    B1 = render.render_bwd(sc, P, g)
    assert np.allclose(B1["g2d"]["abs2d"][:, 6], np.abs(B1["g2d"]["d_rgb"][:, 0]))


@pytest.mark.parametrize("tile", [16, 8])
def test_binned_form_equals_brute_force(tile):
    """The binned oracle (each tile blends only the Gaussians whose conservative
    footprint box covers it) gives the brute force's pixels and 2D gradients on
    the 4096-Gaussian scene: every skipped Gaussian has alpha < 1/255 at the
    tile's pixels, so only zero terms drop out of the sums."""
    sc, cam = scenes.small_scene()
    P = project.project(sc, cam, tile=tile)
    Fb = render.render_fwd_binned(P)
    F = render.render_fwd(P)
    pix = Fb["pixels"]
    assert np.array_equal(np.sort(pix), np.arange(cam.width * cam.height))
    assert np.abs(Fb["image"] - F["image"].reshape(3, -1)[:, pix]).max() < 1e-12
    assert np.abs(Fb["final_T"] - F["final_T"].reshape(-1)[pix]).max() < 1e-12
    assert np.array_equal(Fb["last_id"], F["last_id"].reshape(-1)[pix])
    assert np.array_equal(Fb["n_contrib"], F["n_contrib"].reshape(-1)[pix])
    # a skipped Gaussian could only add flags (alpha just below the cutoff)
    assert not (Fb["flag"] & ~F["flag"].reshape(-1)[pix]).any()
    assert Fb["flag"].sum() == F["flag"].sum()
    w = scenes.random_upstream(cam, seed=3)
    Gb = render.render_bwd_2d_binned(P, w)
    G = render.render_bwd_2d(P, w)
    assert np.array_equal(Gb["contrib"], G["contrib"])
    scale = G["abs2d"].max(axis=1, keepdims=True) + 1e-300
    for k in ("d_mean2d", "d_conic", "d_opacity", "d_rgb"):
        d = np.abs(Gb[k] - G[k]).reshape(len(scale), -1)
        assert (d <= 1e-12 * scale).all(), k
