"""Pins of the oracle's Mip-Splatting filters (the 3D smoothing filter and the
2D mip filter of the Mip-Splatting backbone the paper equips, Sec. 5 and the
supplementary): a single isotropic Gaussian on the optical axis against its
closed form, finite differences of the FP64 forward for every gradient, the
error scale against every gradient, and the 3D filter's variance on
hand-placed points and cameras."""
import numpy as np
import pytest

from oracle import project, render
from paper_2503_18402_amd import scenes


def _iso_scene(s, logit, rgb):
    sh = np.zeros((1, 16, 3))
    sh[0, 0] = (np.asarray(rgb) - 0.5) / 0.28209479177387814
    return dict(means=np.zeros((1, 3)), log_scales=np.full((1, 3), np.log(s)),
                quats=np.array([[1.0, 0.0, 0.0, 0.0]]), opacity_logits=np.array([logit]), sh=sh)


@pytest.mark.parametrize("f3,mip", [(0.0004, True), (0.0004, False), (None, True)])
def test_isotropic_gaussian_on_the_axis(f3, mip):
    """Centre at the origin, camera at distance d on the axis: Sigma_f = (s^2+f)
    I, the projected covariance is (F/d)^2 (s^2+f) I, and every pixel is
    o c3 c2 exp(-r^2 / (2 var)) times the colour, with c3 = (s^2/(s^2+f))^1.5,
    c2 = raw/(raw+0.1) and var = raw + 0.1 (or raw + 0.3 without the 2D filter)."""
    s, d, F, W, H, logit, rgb = 0.05, 2.0, 60.0, 24, 20, 0.3, (0.7, 0.2, 0.4)
    sc = _iso_scene(s, logit, rgb)
    cam = scenes.look_at((0.0, 0.0, -d), (0.0, 0.0, 0.0), W, H, F)
    filt = None if f3 is None else np.array([f3])
    P = project.project(sc, cam, mip2d=mip, filter3d=filt)
    img = render.render_fwd(P)["image"]
    f = 0.0 if f3 is None else f3
    raw = (F / d) ** 2 * (s * s + f)
    c3 = (s * s / (s * s + f)) ** 1.5
    c2 = raw / (raw + 0.1) if mip else 1.0
    var = raw + (0.1 if mip else 0.3)
    o = 1.0 / (1.0 + np.exp(-logit)) * c3 * c2
    y, x = np.mgrid[0:H, 0:W]
    r2 = (x + 0.5 - W / 2) ** 2 + (y + 0.5 - H / 2) ** 2
    a = np.minimum(0.99, o * np.exp(-r2 / (2 * var)))
    a = np.where(a >= 1 / 255, a, 0.0)
    for ch in range(3):
        assert np.abs(img[ch] - a * rgb[ch]).max() < 1e-12
    assert P["coef3"][0] == pytest.approx(c3, rel=1e-12)
    assert P["coef2"][0] == pytest.approx(c2, rel=1e-12)


def _fd(sc, cam, w, mip, filt, tol=1e-6):
    P = project.project(sc, cam, mip2d=mip, filter3d=filt)
    assert not render.render_fwd(P)["flag"].any()
    B = render.render_bwd(sc, P, w, with_bound=True)
    for k in ("d_means", "d_log_scales", "d_quats", "d_opacity_logits", "d_sh"):
        assert np.all(B["bound"][k] >= np.abs(B[k]) * (1 - 1e-12)), k
    sc64 = {k: v.astype(np.float64) for k, v in sc.items()}
    for pn in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        flat = sc64[pn].reshape(-1)
        g = B["d_" + pn].reshape(-1)
        for j in range(flat.shape[0]):
            h = 1e-6 * max(1.0, abs(flat[j]))
            old = flat[j]
            flat[j] = old + h
            lp = render.loss_weighted(sc64, cam, w, mip2d=mip, filter3d=filt)
            flat[j] = old - h
            lm = render.loss_weighted(sc64, cam, w, mip2d=mip, filter3d=filt)
            flat[j] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[j]) <= tol * max(1.0, abs(fd)), (pn, j, fd, g[j])


@pytest.mark.parametrize("mip,use3d", [(True, True), (True, False), (False, True)])
def test_filter_gradients_match_finite_differences(mip, use3d):
    sc = scenes.make_scene(4, seed=81, mean_range=0.25, ls_mu=-2.6, ls_sigma=0.5, rest_sigma=0.2)
    sc["opacity_logits"][:] = [-0.3, 0.4, -1.1, 0.8]
    cam = scenes.look_at((0.3, -0.2, -2.5), (0, 0, 0), 24, 20, 26.0)
    # variances comparable to the smallest squared scales, so the filter matters
    filt = np.array([2e-3, 5e-3, 1e-3, 8e-3]) if use3d else None
    w = np.random.default_rng(82).uniform(-1, 1, size=(3, 20, 24))
    _fd(sc, cam, w, mip, filt)


def test_filter3d_variance_on_placed_points():
    """Camera A at distance 2 (fx 100), camera B at distance 4 (fx 300), both
    64x64 looking at the origin along +z.  The origin is seen by both: nu =
    max(100/2, 300/4) = 75.  (0.5, 0, 0) projects to u = 57 in A and 69.5 in B
    (outside): nu = 50.  A point behind both cameras takes the largest variance
    of the seen ones."""
    A = scenes.look_at((0, 0, -2.0), (0, 0, 0), 64, 64, 100.0)
    B = scenes.look_at((0, 0, -4.0), (0, 0, 0), 64, 64, 300.0)
    pts = np.array([[0.0, 0.0, 0.0], [0.5, 0.0, 0.0], [0.0, 0.0, -10.0], [0.0, 0.25, 0.0]])
    var, flag = project.filter3d_variance(pts, [A, B], scale=0.2)
    assert not flag.any()
    # (0, 0.25, 0): v = 100*0.25/2 + 32 = 44.5 in A, 300*0.25/4 + 32 = 50.75 in B: seen by both
    expect = np.array([0.2 / 75 ** 2, 0.2 / 50 ** 2, 0.2 / 50 ** 2, 0.2 / 75 ** 2])
    assert np.allclose(var, expect, rtol=1e-6)
    var0, _ = project.filter3d_variance(pts[2:3], [A, B])
    assert var0[0] == 0.0


def test_filter3d_variance_flags_edge_points():
    A = scenes.look_at((0, 0, -2.0), (0, 0, 0), 64, 64, 100.0)
    x_edge = (64 - 32) * 2.0 / 100.0          # projects exactly onto u = W
    _, flag = project.filter3d_variance(np.array([[x_edge, 0.0, 0.0], [0.1, 0.1, 0.0]]), [A])
    assert flag.tolist() == [True, False]
