"""GPU parity at the paper-scale workload (1M Gaussians, 1600x1064 and its
downscaled levels), in the launch configuration bench.py times (16x16 tiles,
LDS batch 128), on outputs the FP64 oracle can compute one by one:

* image, final T and last contributor at sampled pixels (random ones plus the
  ragged last tile row and column);
* every parameter gradient for an upstream that is non-zero only at sampled
  pixels, so the oracle's per-pixel brute force covers all contributions;
* sorted keys, values and tile ranges against the oracle's binning, bit for
  bit, at full resolution and at the 1/8 level, at 16- and 8-pixel tiles;
* every gradient at the 1/8 level, whose long lists run list-parallel;
* the batched 16-view form against the plain per-view form and against the
  oracle at sampled pixels of its largest view, and its gradients against the
  oracle's sum over views.  A plain launch of a
  low-resolution view (fewer than 2048 tiles) splits its long lists across
  waves, while the batch (tens of thousands of tiles) walks every list in one
  wave: those views agree within twice the oracle's image tolerance (each side
  is within it), the full-resolution views, on the same path, bit for bit.
"""
import numpy as np
import pytest
import torch

from oracle import binning, project, render, spatial
from paper_2503_18402_amd import gsmi, raster, scenes
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
    P = project.project(scene1m, cam, tile=TILE)
    F = render.render_fwd(P, pixels=pix, chunk=4)
    w[:, pix] = U.zero_flagged(w[:, pix], F)
    params = raster.to_device(scene1m, "cuda")
    frame = raster.render(params, [cam], tile=TILE, lds_batch=BATCH)
    g = U.grads_np(raster.render_backward(params, frame, torch.from_numpy(w.reshape(-1)).cuda()))
    B = render.render_bwd(scene1m, P, w[:, pix], pixels=pix, chunk=4, with_bound=True)
    skip = U.gaussian_flags(P)
    touched = B["g2d"]["contrib"]
    assert touched.sum() > 100
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        U.check_grads(g[name], B["d_" + name], B["bound"]["d_" + name], mask=~skip, name=name)
    # Gaussians no sampled pixel sees get exactly zero
    for name in ("means", "sh"):
        assert not g[name][~touched & ~skip].any()


@pytest.mark.parametrize("level,tile,order", [(1, 16, "index"), (1, 8, "index"),
                                              (8, 16, "index"), (8, 8, "index"),
                                              (1, 16, "spatial"), (1, 8, "spatial")])
def test_keys_and_ranges_match_oracle(scene1m, level, tile, order):
    """The sorted (tile | depth) keys, their Gaussian ids and the tile ranges of
    the 1M-Gaussian view against the oracle's binning over its own FP64
    footprint boxes (stable sort of the keys emitted in index order).  A
    Gaussian whose box edge sits within the float32 guard band of a tile
    boundary (about 1 in 1000) may cover one tile more or less on the device:
    its pairs are removed on both sides, and tiles holding such a pair are left
    out of the range-length comparison.  Device ranges must delimit exactly
    the runs of their tile in the device's keys, [0, 0) when empty.  The
    "spatial" cases store the scene in the oracle's Morton order first: the
    binning's blocks then count most of their pairs in LDS over the tile
    rectangle of their footprints."""
    _, cam = scenes.paper_scale_scene(level=level, n=1)
    if order == "spatial":
        scene1m = scenes.subset(scene1m, spatial.morton_order(scene1m["means"]))
    P = project.project(scene1m, cam, tile=tile)
    gw, gh = -(-cam.width // tile), -(-cam.height // tile)
    k, v, r = binning.bin_sort(P["rect"], P["tiles_touched"], P["depth_f32"], gw, gh)
    flag = P["flag_rect"]
    del P
    params = raster.to_device(scene1m, "cuda")
    frame = raster.render(params, [cam], tile=tile, lds_batch=BATCH, want_keys=True)
    npairs = int(frame.n_pairs_dev.item())
    gk = frame.keys[:npairs].cpu().numpy().view(np.uint64)
    gv = frame.vals[:npairs].cpu().numpy().view(np.uint32)
    gr = frame.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
    del frame, params
    assert flag.mean() < 2e-3
    keep_g, keep_o = ~flag[gv], ~flag[v]
    assert keep_o.sum() > 0.99 * len(v)
    assert np.array_equal(gk[keep_g], k[keep_o])
    assert np.array_equal(gv[keep_g], v[keep_o])
    t_g = (gk >> np.uint64(32)).astype(np.int64)
    tiles = np.arange(gw * gh)
    lo, hi = np.searchsorted(t_g, tiles, "left"), np.searchsorted(t_g, tiles, "right")
    assert np.array_equal(gr, np.where((hi > lo)[:, None], np.stack([lo, hi], 1), 0))
    t_o = (k >> np.uint64(32)).astype(np.int64)
    dirty = np.zeros(gw * gh, bool)
    dirty[t_o[~keep_o]] = True
    dirty[t_g[~keep_g]] = True
    r = r.astype(np.int64)
    assert np.array_equal((gr[:, 1] - gr[:, 0])[~dirty], (r[:, 1] - r[:, 0])[~dirty])
    if not flag.any():
        assert np.array_equal(gr, r)


@pytest.mark.parametrize("tile", [16, 8])
def test_backward_low_resolution_list_parallel(scene1m, tile):
    """The 1/8 level of the 1M-Gaussian view (200x133: 117 or 425 tiles, lists
    of thousands of entries) runs the list-parallel backward, whose chunks are
    walked by separate waves from the chunk-boundary transmittance and colour
    behind.  Upstream non-zero at sampled pixels (random ones plus the ragged
    edges); every parameter gradient against the FP64 oracle."""
    _, cam = scenes.paper_scale_scene(level=8, n=1)
    pix = _sample_pixels(cam, 24, seed=13 + tile)
    P = project.project(scene1m, cam, tile=tile)
    F = render.render_fwd(P, pixels=pix, chunk=4)
    w = np.zeros((3, cam.height * cam.width), np.float32)
    w[:, pix] = np.random.default_rng(14).uniform(-1, 1, size=(3, len(pix)))
    w[:, pix] = U.zero_flagged(w[:, pix], F)
    B = render.render_bwd(scene1m, P, w[:, pix], pixels=pix, chunk=4, with_bound=True)
    skip = U.gaussian_flags(P)
    del P
    params = raster.to_device(scene1m, "cuda")
    frame = raster.render(params, [cam], tile=tile, lds_batch=BATCH)
    gsmi.gs_profile_enable(True)
    try:
        g = raster.render_backward(params, frame, torch.from_numpy(w.reshape(-1)).cuda())
        launched = gsmi.gs_profile_collect()
    finally:
        gsmi.gs_profile_enable(False)
    g = U.grads_np(g)
    assert "k_blend_bwd_long" in launched
    assert B["g2d"]["contrib"].sum() > 1000
    for name in raster.PARAM_NAMES:
        U.check_grads(g[name], B["d_" + name], B["bound"]["d_" + name], mask=~skip, name=name)


def test_batched_mixed_views_gradients_match_oracle(scene1m):
    """The 16-view batch (4 views each at 200x133, 400x266, 800x532 and
    1600x1064) in one launch per kernel: upstream non-zero at sampled pixels
    of two views per resolution, every parameter gradient against the sum over
    views of the oracle's per-view gradients."""
    cams = scenes.mixed_resolution_views()
    rng = np.random.default_rng(61)
    ups, ref, bnd = [], None, None
    skip = np.zeros(scene1m["means"].shape[0], bool)
    for k, c in enumerate(cams):
        w = np.zeros((3, c.height * c.width), np.float32)
        if k % 2 == 0:
            pix = _sample_pixels(c, 4, seed=62 + k)
            P = project.project(scene1m, c, tile=TILE)
            F = render.render_fwd(P, pixels=pix, chunk=4)
            w[:, pix] = rng.uniform(-1, 1, size=(3, len(pix)))
            w[:, pix] = U.zero_flagged(w[:, pix], F)
            B = render.render_bwd(scene1m, P, w[:, pix], pixels=pix, chunk=4, with_bound=True)
            skip |= U.gaussian_flags(P)
            del P
            ref = {n: B["d_" + n] for n in raster.PARAM_NAMES} if ref is None else \
                {n: ref[n] + B["d_" + n] for n in raster.PARAM_NAMES}
            bnd = {n: B["bound"]["d_" + n] for n in raster.PARAM_NAMES} if bnd is None else \
                {n: bnd[n] + B["bound"]["d_" + n] for n in raster.PARAM_NAMES}
        ups.append(w.reshape(-1))
    params = raster.to_device(scene1m, "cuda")
    frame = raster.render(params, cams, tile=TILE, lds_batch=BATCH)
    g = U.grads_np(raster.render_backward(params, frame,
                                          torch.from_numpy(np.concatenate(ups)).cuda()))
    for name in raster.PARAM_NAMES:
        U.check_grads(g[name], ref[name], bnd[name], mask=~skip, name=name)


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
    """torch.autograd.gradcheck (full Jacobian, eps 1e-3, atol 1e-3, rtol 1e-2)
    of RasterizeFn on 64 Gaussians at 32x32, with footprints larger than the
    image, low opacities and no saturation: every alpha stays well above
    1/255, T above 1e-4 and o G below 0.99, and the depths sit on a grid of
    0.0094 spacing, so no perturbation of 1e-3 reorders the blend.  The blend
    is then smooth and finite differences are meaningful."""
    sc = scenes.make_scene(64, seed=31, mean_range=0.3, ls_mu=0.5, ls_sigma=0.2, rest_sigma=0.1)
    sc["opacity_logits"][:] = np.random.default_rng(32).uniform(-3.0, -2.0, 64)
    cam = scenes.look_at((0.1, -0.1, -3.0), (0, 0, 0), 32, 32, 30.0)
    R, t = cam.R.astype(np.float64), cam.t.astype(np.float64)
    depth = 2.7 + 0.6 * (np.random.default_rng(34).permutation(64) + 0.5) / 64
    m = sc["means"].astype(np.float64)
    m[:, 2] = (depth - t[2] - R[2, 0] * m[:, 0] - R[2, 1] * m[:, 1]) / R[2, 2]
    sc["means"][:] = m.astype(np.float32)
    P = project.project(sc, cam)
    F = render.render_fwd(P)
    assert not F["flag"].any() and F["final_T"].min() > 1e-3
    assert np.diff(np.sort(P["xc"][:, 2])).min() > 5e-3
    Bk = render._pixel_block(P, render._order(P), np.arange(32 * 32), 32)
    assert Bk["alpha"].min() > 1.5 / 255.0 and Bk["raw"].max() < 0.2
    inp = [torch.from_numpy(sc[k]).cuda().requires_grad_(True) for k in raster.PARAM_NAMES]
    settings = {"cams": [cam], "tile": 8, "lds_batch": 128}
    fn = lambda *a: raster.RasterizeFn.apply(*a, settings)
    assert torch.autograd.gradcheck(fn, tuple(inp), eps=1e-3, atol=1e-3, rtol=1e-2,
                                    fast_mode=False, check_undefined_grad=False,
                                    nondet_tol=1e-6)
    # and the same sub-case against the FP64 oracle gradient
    w = np.random.default_rng(33).uniform(-1, 1, size=(3, 32, 32))
    out = fn(*inp)
    (out * torch.from_numpy(w.astype(np.float32)).cuda().reshape(-1)).sum().backward()
    B = render.render_bwd(sc, P, w, with_bound=True)
    for k, name in zip(inp, raster.PARAM_NAMES):
        U.check_grads(k.grad.cpu().numpy(), B["d_" + name], B["bound"]["d_" + name], name=name)


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
