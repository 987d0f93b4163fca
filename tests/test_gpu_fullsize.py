"""GPU parity at the paper-scale workload (1M Gaussians, 1600x1064 and its
downscaled levels), in the launch configuration bench.py times (16x16 tiles,
LDS batch 128), on outputs the FP64 oracle can compute one by one:

* image, final T and last contributor at sampled pixels (random ones plus the
  ragged last tile row and column);
* every parameter gradient for an upstream that is non-zero only at sampled
  pixels, so the oracle's per-pixel brute force covers all contributions;
* the batched 16-view form against the plain per-view form and against the
  oracle at sampled pixels of its largest view.  A plain launch of a
  low-resolution view (fewer than 2048 tiles) splits its long lists across
  waves, while the batch (tens of thousands of tiles) walks every list in one
  wave: those views agree within twice the oracle's image tolerance (each side
  is within it), the full-resolution views, on the same path, bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import project, render
from paper_2503_18402_amd import raster, scenes
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

TILE, BATCH = 16, 128


@pytest.fixture(scope="module")
def scene1m():
    sc, _ = scenes.paper_scale_scene(level=1)
    return sc


def _sample_pixels(cam, n_rand, seed):
    rng = np.random.default_rng(seed)
    W, H = cam.width, cam.height
    pix = list(rng.choice(W * H, n_rand, replace=False))
    # ragged edges: last row and last column, corners
    pix += [(H - 1) * W + x for x in rng.choice(W, 4, replace=False)]
    pix += [y * W + (W - 1) for y in rng.choice(H, 4, replace=False)]
    pix += [0, W - 1, (H - 1) * W, H * W - 1]
    return np.unique(np.array(pix, np.int64))


@pytest.mark.parametrize("level", [1, 8])
def test_forward_sampled_pixels(scene1m, level):
    _, cam = scenes.paper_scale_scene(level=level, n=1)
    params = raster.to_device(scene1m, "cuda")
    frame = raster.render(params, [cam], tile=TILE, lds_batch=BATCH)
    torch.cuda.synchronize()
    P = project.project(scene1m, cam, tile=TILE)
    pix = _sample_pixels(cam, 40, seed=level)
    F = render.render_fwd(P, pixels=pix, chunk=4)
    img = frame.image.view(3, -1).cpu().numpy()[:, pix]
    fT = frame.final_T.cpu().numpy()[pix]
    ok = ~F["flag"]
    assert ok.sum() >= len(pix) - 2
    assert np.abs(img - F["image"])[:, ok].max() < 1e-5
    assert np.abs(fT - F["final_T"])[ok].max() < 1e-5
    # last contributor as a Gaussian id
    last = frame.last_contrib.cpu().numpy().astype(np.int64)[pix]
    vals = frame.vals.cpu().numpy().astype(np.int64)
    ranges = frame.ranges.cpu().numpy().astype(np.int64).reshape(-1, 2)
    gw = -(-cam.width // TILE)
    t = (pix // cam.width) // TILE * gw + (pix % cam.width) // TILE
    gid = np.where(last > 0, vals[np.clip(ranges[t, 0] + last - 1, 0, None)], -1)
    assert np.array_equal(gid[ok], F["last_id"][ok])


def test_backward_sparse_upstream(scene1m):
    _, cam = scenes.paper_scale_scene(level=1, n=1)
    pix = _sample_pixels(cam, 20, seed=11)
    rng = np.random.default_rng(12)
    w = np.zeros((3, cam.height * cam.width), np.float32)
    w[:, pix] = rng.uniform(-1, 1, size=(3, len(pix)))
    params = raster.to_device(scene1m, "cuda")
    frame = raster.render(params, [cam], tile=TILE, lds_batch=BATCH)
    g = U.grads_np(raster.render_backward(params, frame, torch.from_numpy(w.reshape(-1)).cuda()))
    P = project.project(scene1m, cam, tile=TILE)
    F = render.render_fwd(P, pixels=pix, chunk=4)
    B = render.render_bwd(scene1m, P, w[:, pix], pixels=pix, chunk=4, with_bound=True)
    skip = P["flag_rgb"].any(1)
    flagged = pix[F["flag"]]
    if flagged.size:
        order = render._order(P)
        Bk = render._pixel_block(P, order, flagged, cam.width)
        skip[order[(Bk["alpha"] >= 0.9 / 255.0).any(axis=0)]] = True
    touched = B["g2d"]["contrib"]
    assert touched.sum() > 100
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        U.check_grads(g[name], B["d_" + name], B["bound"]["d_" + name], mask=~skip)
    # Gaussians no sampled pixel sees get exactly zero
    for name in ("means", "sh"):
        assert not g[name][~touched & ~skip].any()


def test_batched_mixed_views_equal_plain_and_oracle(scene1m):
    cams = scenes.mixed_resolution_views()
    params = raster.to_device(scene1m, "cuda")
    fb = raster.render(params, cams, tile=TILE, lds_batch=BATCH)
    imgs = fb.images()
    for k in (0, 5, 10, 15):
        fp = raster.render(params, [cams[k]], tile=TILE, lds_batch=BATCH)
        tiles = -(-cams[k].width // TILE) * -(-cams[k].height // TILE)
        if tiles >= 2048:
            assert torch.equal(imgs[k].reshape(-1), fp.image), k
        else:
            assert (imgs[k].reshape(-1) - fp.image).abs().max().item() < 2e-5, k
    cam = cams[15]
    P = project.project(scene1m, cam, tile=TILE)
    pix = _sample_pixels(cam, 16, seed=21)
    F = render.render_fwd(P, pixels=pix, chunk=4)
    img = imgs[15].reshape(3, -1).cpu().numpy()[:, pix]
    ok = ~F["flag"]
    assert np.abs(img - F["image"])[:, ok].max() < 1e-5


def test_gradcheck_smooth_subcase():
    """torch.autograd.gradcheck of RasterizeFn on 64 Gaussians at 32x32, with
    footprints larger than the image, low opacities and no saturation: no
    pixel sits near the 1/255 cutoff, the T exit or the 0.99 clamp, so the
    blend is smooth and finite differences are meaningful."""
    sc = scenes.make_scene(64, seed=31, mean_range=0.3, ls_mu=0.5, ls_sigma=0.2, rest_sigma=0.1)
    sc["opacity_logits"][:] = np.random.default_rng(32).uniform(-3.0, -2.0, 64)
    cam = scenes.look_at((0.1, -0.1, -3.0), (0, 0, 0), 32, 32, 30.0)
    P = project.project(sc, cam)
    F = render.render_fwd(P)
    assert not F["flag"].any() and F["final_T"].min() > 1e-3
    inp = [torch.from_numpy(sc[k]).cuda().requires_grad_(True) for k in raster.PARAM_NAMES]
    settings = {"cams": [cam], "tile": 8, "lds_batch": 128}
    fn = lambda *a: raster.RasterizeFn.apply(*a, settings)
    assert torch.autograd.gradcheck(fn, tuple(inp), eps=1e-3, atol=2e-3, rtol=2e-2,
                                    fast_mode=True, check_undefined_grad=False,
                                    nondet_tol=1e-6)
    # and the same sub-case against the FP64 oracle gradient
    w = np.random.default_rng(33).uniform(-1, 1, size=(3, 32, 32))
    out = fn(*inp)
    (out * torch.from_numpy(w.astype(np.float32)).cuda().reshape(-1)).sum().backward()
    B = render.render_bwd(sc, P, w, with_bound=True)
    for k, name in zip(inp, raster.PARAM_NAMES):
        U.check_grads(k.grad.cpu().numpy(), B["d_" + name], B["bound"]["d_" + name], max_frac=0.0)


def test_large_scene_batched_sampled_pixels():
    """The 4M-Gaussian workload: all 16 views (8 at 1920x1080, 8 at 960x540) in
    one batched launch, in the bench's launch configuration; sampled pixels of
    one view of each resolution (plus the ragged edges) against the oracle."""
    sc, cams = scenes.large_scene_views()
    params = raster.to_device(sc, "cuda")
    fb = raster.render(params, cams, tile=TILE, lds_batch=BATCH)
    imgs = fb.images()
    torch.cuda.synchronize()
    del params
    for k in (0, 12):
        cam = cams[k]
        P = project.project(sc, cam, tile=TILE)
        pix = _sample_pixels(cam, 8, seed=30 + k)
        F = render.render_fwd(P, pixels=pix, chunk=4)
        img = imgs[k].reshape(3, -1).cpu().numpy()[:, pix]
        ok = ~F["flag"]
        assert ok.sum() >= len(pix) - 2
        assert np.abs(img - F["image"])[:, ok].max() < 1e-5, k
