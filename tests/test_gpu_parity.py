"""GPU parity: every call of the C ABI against the FP64 oracle (the 4096-Gaussian scene and
small edge scenes).  Tolerances: keys / values / ranges bit-exact; images and
final T within 1e-5 absolute; gradients |g - g_ref| <= 1e-3 |g_ref| + 1e-6
with an O(1) upstream (L = sum w * C, w ~ U[-1,1]).  Pixels the oracle flags
as within a float32 guard band of a discrete decision leave the image check
and get a zero upstream on both sides (so they add nothing to any gradient);
Gaussians with a per-Gaussian guard-band decision (a colour channel at the
clamp, the opacity at the cull) leave the gradient check."""
import numpy as np
import pytest
import torch

from oracle import adam as o_adam
from oracle import binning, loss as o_loss, project, render
from paper_2503_18402_amd import gsmi, raster, scenes
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5


@pytest.fixture(scope="module")
def small():
    sc, cam = scenes.small_scene()
    P = project.project(sc, cam, tile=16)
    F = render.render_fwd(P, want_lists=True)
    w = U.zero_flagged(scenes.random_upstream(cam), F)
    B = render.render_bwd(sc, P, w, with_bound=True)
    return dict(sc=sc, cam=cam, w=w, P=P, F=F, B=B)


def test_preprocess_matches_oracle(small):
    sc, cam, P = small["sc"], small["cam"], small["P"]
    _, frame, _ = U.run(sc, [cam], upstream=None)
    d = U.decode_proj(frame)
    live = P["tiles_touched"] > 0
    assert np.array_equal(d["depth"].view(np.uint32), P["depth_f32"].view(np.uint32))
    ok = ~P["flag_rect"]
    assert np.array_equal(d["tt"][ok], P["tiles_touched"][ok])
    assert np.array_equal(d["px_box"][live & ok], P["px_box"][live & ok])
    assert np.abs(d["mean2d"][live] - P["mean2d"][live]).max() < 2e-4
    rel = np.abs(d["conic"][live] - P["conic"][live]) / (np.abs(P["conic"][live]).max(1, keepdims=True))
    assert rel.max() < 1e-4
    assert np.abs(d["opacity"][live] - P["opacity"][live]).max() < 1e-6
    assert np.abs(d["rgb"][live] - P["rgb"][live]).max() < 1e-5
    clamp = (P["rgb_raw"] < 0) & ~P["flag_rgb"]
    for c in range(3):
        assert np.array_equal(((d["flags"] >> c) & 1).astype(bool)[live], clamp[live, c])


def test_bin_sort_properties(small):
    """Device keys are sorted, stable (equal keys keep ascending index), carry each
    pair's own depth bits, give every Gaussian exactly its tile count, and the
    ranges cover exactly the runs of each tile."""
    sc, cam = small["sc"], small["cam"]
    for tile in (8, 16, 32):
        _, frame, _ = U.run(sc, [cam], tile=tile)
        d = U.decode_proj(frame)
        npairs = int(frame.n_pairs_dev.item())
        assert npairs == int(d["tt"].sum())
        keys = frame.keys[:npairs].cpu().numpy().view(np.uint64)
        vals = frame.vals[:npairs].cpu().numpy().view(np.uint32).astype(np.int64)
        order = np.lexsort((vals, keys))
        assert np.array_equal(order, np.arange(npairs))          # sorted by (key, index)
        assert np.array_equal((keys & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                              d["depth"][vals].view(np.uint32))
        assert np.array_equal(np.bincount(vals, minlength=frame.n), d["tt"])
        tiles = (keys >> np.uint64(32)).astype(np.int64)
        rects = U.gpu_rect(d, tile)
        assert np.all((tiles % -(-cam.width // tile) >= rects[vals, 0]) &
                      (tiles % -(-cam.width // tile) <= rects[vals, 2]))
        r = frame.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2).astype(np.int64)
        for t in range(r.shape[0]):
            sel = np.nonzero(tiles == t)[0]
            if sel.size:
                assert r[t, 0] == sel[0] and r[t, 1] == sel[-1] + 1
            else:
                assert r[t, 0] == 0 and r[t, 1] == 0


@pytest.mark.parametrize("n,longest", [(1500, 512), (3000, 2048), (12000, 8192), (40000, 16384)])
def test_bin_sort_long_lists(n, longest):
    """Tile lists longer than the one-wave register sort (512 keys), than the
    256-thread LDS sort (2048 keys) and than one LDS chunk (8192 keys, sorted
    through global memory; two chunks and more): still the exact (tile, depth, index) order of the
    oracle's binning.  A quarter of the Gaussians share their mean, hence their
    depth, with another one, so ties are broken by index."""
    sc = scenes.make_scene(n, seed=41, mean_range=0.2, ls_mu=-3.0, ls_sigma=0.2)
    sc["means"][n // 2:n // 2 + n // 4] = sc["means"][:n // 4]
    cam = scenes.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 32, 32, 40.0)
    P = project.project(sc, cam, tile=16)
    k, v, r = binning.bin_sort(P["rect"], P["tiles_touched"], P["depth_f32"], 2, 2)
    assert np.diff(r, axis=1).max() > longest
    _, frame, _ = U.run(sc, [cam], tile=16)
    npairs = int(frame.n_pairs_dev.item())
    gk = frame.keys[:npairs].cpu().numpy().view(np.uint64)
    gv = frame.vals[:npairs].cpu().numpy().view(np.uint32)
    if not P["flag_rect"].any():
        assert np.array_equal(gk, k) and np.array_equal(gv, v)
        assert np.array_equal(frame.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), r)
    else:
        assert np.array_equal(gv[~P["flag_rect"][gv]], v[~P["flag_rect"][v]])


@pytest.mark.parametrize("n,tile", [(1500, 16), (3000, 8)])
def test_backward_long_lists(n, tile):
    """Tile lists of 700-1400 entries with low opacities, so pixels blend deep
    into them: the backward runs list-parallel (chunks walked by separate
    waves from the chunk-boundary transmittance and colour behind).  Every
    gradient against the FP64 oracle at the conditioned tolerance."""
    sc = scenes.make_scene(n, seed=43, mean_range=0.2, ls_mu=-3.0, ls_sigma=0.2)
    sc["opacity_logits"][:] = np.random.default_rng(44).uniform(-4.6, -3.5, n)
    cam = scenes.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 32, 32, 40.0)
    P = project.project(sc, cam, tile=tile)
    F = render.render_fwd(P)
    w = np.random.default_rng(45).uniform(-1, 1, size=(3, 32, 32)).astype(np.float32)
    w = U.zero_flagged(w, F)
    B = render.render_bwd(sc, P, w, with_bound=True)
    _, frame, g = U.run(sc, [cam], tile=tile, upstream=[w])
    assert np.diff(frame.ranges.cpu().numpy().reshape(-1, 2), axis=1).max() > 512
    skip = U.gaussian_flags(P)
    img = frame.image.view(3, 32, 32).cpu().numpy()
    assert np.abs(img - F["image"])[:, ~F["flag"].reshape(32, 32)].max() < IMG_TOL
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        U.check_grads(g[name], B["d_" + name], B["bound"]["d_" + name], mask=~skip, name=name)


def test_bin_sort_end_to_end_matches_oracle(small):
    sc, cam, P = small["sc"], small["cam"], small["P"]
    _, frame, _ = U.run(sc, [cam], tile=16)
    gw, gh = -(-cam.width // 16), -(-cam.height // 16)
    k, v, r = binning.bin_sort(P["rect"], P["tiles_touched"], P["depth_f32"], gw, gh)
    npairs = int(frame.n_pairs_dev.item())
    if not P["flag_rect"].any():
        assert npairs == k.shape[0]
        assert np.array_equal(frame.keys[:npairs].cpu().numpy().view(np.uint64), k)
        assert np.array_equal(frame.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), r)
    else:  # compare with the flagged Gaussians' pairs removed on both sides
        gk = frame.keys[:npairs].cpu().numpy().view(np.uint64)
        gv = frame.vals[:npairs].cpu().numpy().view(np.uint32)
        keep_o = ~P["flag_rect"][v]
        keep_g = ~P["flag_rect"][gv]
        assert np.array_equal(gk[keep_g], k[keep_o])


def test_render_fwd_matches_oracle(small):
    sc, cam, F = small["sc"], small["cam"], small["F"]
    _, frame, _ = U.run(sc, [cam], tile=16)
    img = frame.image.view(3, cam.height, cam.width).cpu().numpy()
    fT = frame.final_T.view(cam.height, cam.width).cpu().numpy()
    ok = ~F["flag"]
    assert ok.mean() > 0.99
    assert np.abs(img - F["image"])[:, ok].max() < IMG_TOL
    assert np.abs(fT - F["final_T"])[ok].max() < IMG_TOL
    # last contributor compared as a Gaussian id
    last = frame.last_contrib.view(cam.height, cam.width).cpu().numpy().astype(np.int64)
    vals = frame.vals.cpu().numpy().astype(np.int64)
    ranges = frame.ranges.cpu().numpy().astype(np.int64).reshape(-1, 2)
    gw = -(-cam.width // 16)
    ys, xs = np.mgrid[0:cam.height, 0:cam.width]
    t = (ys // 16) * gw + xs // 16
    gid = np.where(last > 0, vals[np.clip(ranges[t, 0] + last - 1, 0, None)], -1)
    assert np.array_equal(gid[ok], F["last_id"][ok])


def test_image_independent_of_tile_and_batch(small):
    """Binning is result-neutral: the LDS batch size changes no bit; the tile size
    changes only the float32 rounding of the mean moved into each tile's frame."""
    sc, cam = small["sc"], small["cam"]
    ref = None
    for tile in (8, 16, 32):
        per_tile = None
        for batch in (128, 256, 512):
            _, frame, _ = U.run(sc, [cam], tile=tile, lds_batch=batch, want_keys=False)
            img = frame.image.cpu().numpy()
            if per_tile is None:
                per_tile = img
            assert np.array_equal(img, per_tile), (tile, batch)
        if ref is None:
            ref = per_tile
        assert np.abs(per_tile - ref).max() < 2e-6, tile


def test_render_bwd_matches_oracle(small):
    sc, cam, w, P, F, B = (small[k] for k in ("sc", "cam", "w", "P", "F", "B"))
    _, frame, g = U.run(sc, [cam], upstream=[w])
    mask = ~U.gaussian_flags(P)
    assert mask.mean() > 0.999
    for name in ("means", "log_scales", "quats", "opacity_logits", "sh"):
        U.check_grads(g[name], B["d_" + name], B["bound"]["d_" + name], mask=mask, name=name)


@pytest.mark.parametrize("tile,batch", [(8, 128), (32, 512)])
def test_render_bwd_other_tiles(small, tile, batch):
    sc, cam, w, P, F, B = (small[k] for k in ("sc", "cam", "w", "P", "F", "B"))
    _, _, g = U.run(sc, [cam], tile=tile, lds_batch=batch, upstream=[w])
    mask = ~U.gaussian_flags(P)
    for name in raster.PARAM_NAMES:
        U.check_grads(g[name], B["d_" + name], B["bound"]["d_" + name], mask=mask, name=name,
                      max_frac=U.MEANS_CANCELLATION_FRAC if name == "means" else 0.0)


def test_background_and_degree(small):
    sc = scenes.subset(small["sc"], slice(0, 1500))
    cam = small["cam"]
    bg = (0.25, 0.5, 0.75)
    for deg in (0, 1, 2):
        P = project.project(sc, cam, sh_degree=deg)
        F = render.render_fwd(P, bg=bg)
        w = U.zero_flagged(scenes.random_upstream(cam, seed=9), F)
        Bo = render.render_bwd(sc, P, w, bg=bg, with_bound=True)
        _, frame, g = U.run(sc, [cam], bg=bg, sh_degree=deg, upstream=[w])
        img = frame.image.view(3, cam.height, cam.width).cpu().numpy()
        ok = ~F["flag"]
        assert np.abs(img - F["image"])[:, ok].max() < IMG_TOL
        mask = ~U.gaussian_flags(P)
        for name in raster.PARAM_NAMES:
            U.check_grads(g[name], Bo["d_" + name], Bo["bound"]["d_" + name], mask=mask,
                          name=name)
        K = (deg + 1) ** 2
        assert np.all(g["sh"][:, K:, :] == 0.0)


def test_batched_views_equal_plain():
    sc, _ = scenes.small_scene()
    base = scenes.orbit_cameras(4, 3.0, 128, 96, 120.0)
    cams = [base[0], scenes.downscale(base[1], 2), base[2], scenes.downscale(base[3], 4)]
    ups = [scenes.random_upstream(c, seed=20 + k) for k, c in enumerate(cams)]
    _, fb, gb = U.run(sc, cams, upstream=ups, want_keys=False)
    gsum = None
    scale = None
    off = 0
    for k, c in enumerate(cams):
        _, fp, gp = U.run(sc, [c], upstream=[ups[k]], want_keys=False)
        npx = 3 * c.width * c.height
        assert np.array_equal(fb.image[off:off + npx].cpu().numpy(), fp.image.cpu().numpy())
        off += npx
        gsum = gp if gsum is None else {n: gsum[n] + gp[n] for n in gsum}
        P = project.project(sc, c)
        bnd = render.chain_abs_bound(sc, P, render.render_bwd_2d(P, ups[k])["abs2d"])
        scale = bnd if scale is None else {n: scale[n] + bnd[n] for n in scale}
    # same per-view kernels; only the float32 order of the sum over views differs
    for name in gsum:
        err = np.abs(gb[name] - gsum[name])
        assert np.all(err <= 1e-6 * scale["d_" + name] + 1e-9), (name, float(
            np.max(err / (scale["d_" + name] + 1e-30))))


def test_one_view_and_several_view_preprocess_records_equal():
    """The one-view preprocess (each lane loads its own SH row) and the
    several-view form (rows staged once through LDS for all views) write the
    same records: every word of a Gaussian with a footprint, and the tile
    count, box and depth of every Gaussian (a Gaussian without a footprint has
    no colour the later calls read)."""
    sc, _ = scenes.small_scene()
    base = scenes.orbit_cameras(4, 3.0, 128, 96, 120.0)
    cams = [base[0], scenes.downscale(base[1], 2), base[2], scenes.downscale(base[3], 4)]
    _, fb, _ = U.run(sc, cams, upstream=None, want_keys=False)
    for k, c in enumerate(cams):
        _, fp, _ = U.run(sc, [c], upstream=None, want_keys=False)
        b, p = U.decode_proj(fb, view=k), U.decode_proj(fp)
        assert np.array_equal(b["tt"], p["tt"]), k
        assert np.array_equal(b["px_box"], p["px_box"]), k
        assert np.array_equal(b["depth"].view(np.uint32), p["depth"].view(np.uint32)), k
        live = p["tt"] > 0
        assert live.sum() > 100, k
        for name in ("mean2d", "conic", "opacity", "rgb"):
            assert np.array_equal(b[name][live], p[name][live]), (k, name)
        assert np.array_equal(b["flags"][live], p["flags"][live]), k


def test_multiview_grads_match_oracle_sum():
    sc, _ = scenes.small_scene()
    sc = scenes.subset(sc, slice(0, 2000))
    cams = scenes.orbit_cameras(3, 3.0, 64, 48, 60.0)
    ups, ref = [], None
    skip = np.zeros(2000, bool)
    for k, c in enumerate(cams):
        P = project.project(sc, c)
        F = render.render_fwd(P)
        u = U.zero_flagged(scenes.random_upstream(c, seed=40 + k), F)
        ups.append(u)
        Bo = render.render_bwd(sc, P, u, with_bound=True)
        skip |= U.gaussian_flags(P)
        cur = {"d_" + n: Bo["d_" + n] for n in raster.PARAM_NAMES}
        cur.update({"b_d_" + n: Bo["bound"]["d_" + n] for n in raster.PARAM_NAMES})
        ref = cur if ref is None else {k: ref[k] + cur[k] for k in ref}
    _, _, g = U.run(sc, cams, upstream=ups, want_keys=False)
    for name in raster.PARAM_NAMES:
        U.check_grads(g[name], ref["d_" + name], ref["b_d_" + name], mask=~skip, name=name,
                      max_frac=U.MEANS_CANCELLATION_FRAC if name == "means" else 0.0)


def test_backward_balanced_order_dense_upstream():
    """A 1024x512 view at 32-pixel tiles: 512 tiles and no list-parallel split,
    so the backward deals its tiles to blocks in the balanced order (ranked by
    list length, two rounds of 256, the second reversed).  A dense O(1)
    upstream over every pixel, every gradient of all 3000 Gaussians against the
    binned oracle (each tile blends its footprint candidates; equal to the
    brute force): a tile the order dropped or took twice would leave its pair
    slots at zero or double them."""
    sc = scenes.make_scene(3000, seed=51, mean_range=1.0, ls_mu=-3.0, ls_sigma=0.4)
    cam = scenes.look_at((0.2, -0.1, -3.0), (0.0, 0.0, 0.0), 1024, 512, 700.0)
    P = project.project(sc, cam, tile=32)
    cands = render.tile_candidates(P)
    assert len(cands) == 512 and max(len(c) for c in cands) > 2 * min(len(c) for c in cands)
    Fb = render.render_fwd_binned(P, cands=cands)
    flag = np.zeros(cam.width * cam.height, bool)
    flag[Fb["pixels"]] = Fb["flag"]
    w = U.zero_flagged(scenes.random_upstream(cam, seed=52), dict(flag=flag))
    g2 = render.render_bwd_2d_binned(P, w, cands=cands)
    ref = render.chain_to_3d(sc, P, g2)
    bnd = render.chain_abs_bound(sc, P, g2["abs2d"])
    _, frame, g = U.run(sc, [cam], tile=32, lds_batch=256, upstream=[w], want_keys=False)
    img = frame.image.view(3, -1).cpu().numpy()[:, Fb["pixels"]]
    assert np.abs(img - Fb["image"])[:, ~Fb["flag"]].max() < IMG_TOL
    mask = ~U.gaussian_flags(P)
    assert g2["contrib"].sum() > 2500
    for name in raster.PARAM_NAMES:
        U.check_grads(g[name], ref["d_" + name], bnd["d_" + name], mask=mask, name=name,
                      max_frac=U.MEANS_CANCELLATION_FRAC if name == "means" else 0.0)


def test_l1_loss_grad_matches_oracle():
    rng = np.random.default_rng(0)
    img = rng.uniform(size=(3, 37, 29)).astype(np.float32)
    tgt = rng.uniform(size=(3, 37, 29)).astype(np.float32)
    tgt[0, 0, :5] = img[0, 0, :5]
    gi, gt = torch.from_numpy(img).cuda(), torch.from_numpy(tgt).cuda()
    dL = torch.empty_like(gi)
    ls = torch.zeros(1, device="cuda")
    gsmi.gs_l1_loss_grad(gi, gt, 1.0 / img.size, dL, ls)
    val, g = o_loss.l1(img, tgt)
    assert np.array_equal(dL.cpu().numpy(), g.astype(np.float32))
    assert abs(float(ls.item()) - val) < 1e-6


def test_adam_matches_oracle():
    rng = np.random.default_rng(1)
    sizes = [1003, 16, 7, 4096]
    lrs = [1e-2, 5e-3, 1e-3, 2.5e-3]
    host = [dict(p=rng.normal(size=s), m=np.zeros(s), v=np.zeros(s)) for s in sizes]
    dev = [{k: torch.from_numpy(h[k].astype(np.float32)).cuda() for k in h} for h in host]
    for step in range(1, 6):
        grads = [rng.normal(size=s) for s in sizes]
        gdev = [torch.from_numpy(g.astype(np.float32)).cuda() for g in grads]
        gsmi.gs_adam_step([(d["p"], gg, d["m"], d["v"], lr) for d, gg, lr in zip(dev, gdev, lrs)],
                          step, 0.9, 0.999, 1e-15)
        for h, g, lr in zip(host, grads, lrs):
            g32 = g.astype(np.float32).astype(np.float64)
            h["p"], h["m"], h["v"] = o_adam.adam_step(h["p"], g32, h["m"], h["v"], step, lr)
    for h, d in zip(host, dev):
        assert np.abs(d["p"].cpu().numpy() - h["p"]).max() < 1e-5
        assert np.abs(d["m"].cpu().numpy() - h["m"]).max() < 1e-6


# ------------------------------------------------------------------- edges

def test_empty_scene():
    sc = scenes.subset(scenes.small_scene()[0], slice(0, 0))
    cam = scenes.small_scene()[1]
    _, frame, g = U.run(sc, [cam], upstream=[scenes.random_upstream(cam)])
    assert int(frame.n_pairs_dev.item()) == 0
    assert np.all(frame.image.cpu().numpy() == 0.0)
    assert np.all(frame.final_T.cpu().numpy() == 1.0)
    assert not frame.ranges.cpu().numpy().any()


def test_all_culled_and_behind_camera():
    sc = scenes.make_scene(300, seed=3)
    sc["means"][:, 2] = -5.0          # all behind the camera at z = -3
    cam = scenes.small_scene()[1]
    _, frame, g = U.run(sc, [cam], upstream=[scenes.random_upstream(cam)])
    assert int(frame.n_pairs_dev.item()) == 0
    assert np.all(frame.image.cpu().numpy() == 0.0)
    for v in g.values():
        assert not v.any()


def test_single_gaussian_covering_every_tile():
    sc = scenes.make_scene(1, seed=4, ls_mu=-0.3, ls_sigma=0.2)
    sc["means"][:] = 0.0
    sc["opacity_logits"][:] = 3.0
    cam = scenes.look_at((0, 0, -3), (0, 0, 0), 70, 45, 60.0)   # ragged 16x16 tiles
    P = project.project(sc, cam)
    assert P["tiles_touched"][0] == 5 * 3
    F = render.render_fwd(P)
    w = U.zero_flagged(scenes.random_upstream(cam, seed=5), F)
    Bo = render.render_bwd(sc, P, w, with_bound=True)
    _, frame, g = U.run(sc, [cam], upstream=[w])
    img = frame.image.view(3, 45, 70).cpu().numpy()
    ok = ~F["flag"]
    assert np.abs(img - F["image"])[:, ok].max() < IMG_TOL
    for name in ("means", "log_scales", "opacity_logits", "quats", "sh"):
        U.check_grads(g[name], Bo["d_" + name], Bo["bound"]["d_" + name], name=name)


def test_saturating_stack_exit():
    # 24 coincident Gaussians with alpha = 0.5 at the centre pixel: 13 are blended
    n = 24
    sc = dict(means=np.zeros((n, 3), np.float32), log_scales=np.full((n, 3), -3.0, np.float32),
              quats=np.tile(np.array([[1, 0, 0, 0]], np.float32), (n, 1)),
              opacity_logits=np.zeros(n, np.float32), sh=np.zeros((n, 16, 3), np.float32))
    sc["sh"][:, 0, :] = 1.0
    cam = scenes.look_at((0, 0, -3), (0, 0, 0), 33, 33, 40.0)
    cam.cx = cam.cy = 16.5
    _, frame, _ = U.run(sc, [cam])
    last = frame.last_contrib.view(33, 33).cpu().numpy()
    fT = frame.final_T.view(33, 33).cpu().numpy()
    assert last[16, 16] == 13
    assert abs(fT[16, 16] - 2.0 ** -13) < 1e-9


def test_capacity_overflow_reported_and_regrown(small):
    sc, cam = small["sc"], small["cam"]
    params = raster.to_device(sc, "cuda")
    frame = raster.render(params, [cam], capacity=100, check_capacity=False)
    torch.cuda.synchronize()
    assert int(frame.n_pairs_dev.item()) > 100
    assert not frame.ranges.cpu().numpy().any()      # ranges invalid -> left empty
    frame2 = raster.render(params, [cam], capacity=100, check_capacity=True)
    assert frame2.capacity >= int(frame2.n_pairs_dev.item())
    ref = raster.render(params, [cam])
    assert torch.equal(frame2.image, ref.image)


def test_autograd_function_matches_oracle(small):
    sc, cam, w, P, F, B = (small[k] for k in ("sc", "cam", "w", "P", "F", "B"))
    prm = {k: v.requires_grad_(True) for k, v in raster.to_device(sc, "cuda").items()}
    img = raster.RasterizeFn.apply(prm["means"], prm["log_scales"], prm["quats"],
                                   prm["opacity_logits"], prm["sh"], {"cams": [cam]})
    loss = (img * torch.from_numpy(w).cuda().reshape(-1)).sum()
    loss.backward()
    mask = ~U.gaussian_flags(P)
    for name in raster.PARAM_NAMES:
        U.check_grads(prm[name].grad.cpu().numpy(), B["d_" + name], B["bound"]["d_" + name],
                      mask=mask, name=name)


def test_overwrite_equals_accumulate_into_zero(small):
    sc, cam, w = small["sc"], small["cam"], small["w"]
    params = raster.to_device(sc, "cuda")
    frame = raster.render(params, [cam])
    dL = torch.from_numpy(w).cuda().reshape(-1)
    acc = raster.render_backward(params, frame, dL)
    junk = {k: torch.full_like(v, 7.0) for k, v in acc.items()}
    m2 = torch.full((params["means"].shape[0],), 3.0, device="cuda")
    over = raster.render_backward(params, frame, dL, grads=junk, mean2d_abs=m2, accumulate=False)
    for k in acc:
        assert torch.equal(acc[k], over[k]), k
    m2b = torch.zeros_like(m2)
    raster.render_backward(params, frame, dL, mean2d_abs=m2b)
    assert torch.equal(m2, m2b)
    # accumulating twice doubles
    twice = raster.render_backward(params, frame, dL, grads={k: v.clone() for k, v in acc.items()})
    for k in acc:
        assert torch.allclose(twice[k], 2 * acc[k], rtol=1e-6, atol=0), k


@pytest.mark.parametrize("tile", [8, 16])
def test_empty_tiles_have_zero_ranges(tile):
    """A sparse scene leaves most tiles empty: their ranges are [0, 0), and every
    range equals the oracle's (R7), for both binning forms."""
    sc = scenes.subset(scenes.small_scene()[0], slice(0, 60))
    cam = scenes.small_scene()[1]
    P = project.project(sc, cam, tile=tile)
    assert not P["flag_rect"].any()
    gw, gh = -(-cam.width // tile), -(-cam.height // tile)
    _, _, r = binning.bin_sort(P["rect"], P["tiles_touched"], P["depth_f32"], gw, gh)
    assert (r[:, 0] == r[:, 1]).sum() >= 5      # several empty tiles
    _, frame, _ = U.run(sc, [cam], tile=tile)
    assert np.array_equal(frame.ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), r)
    n = 60
    ws = torch.empty(gsmi.gs_bin_sort_radix_workspace_bytes(1, n, frame.capacity),
                     dtype=torch.uint8, device="cuda")
    vals = torch.empty(frame.capacity, dtype=torch.int32, device="cuda")
    ranges = torch.empty_like(frame.ranges)
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    gsmi.gs_bin_sort_radix(frame.cams_c, frame.cfg, n, frame.proj, frame.capacity, ws, None, vals,
                           ranges, npairs)
    torch.cuda.synchronize()
    assert np.array_equal(ranges.cpu().numpy().view(np.uint32).reshape(-1, 2), r)
