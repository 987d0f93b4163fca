"""Edge cases of the device path against the FP64 oracle: views smaller than a
tile and ragged in both directions (down to 1x1) batched with an ordinary
view, at 8- and 16-pixel tiles; the largest batch (GS_MAX_VIEWS views) against
the plain per-view calls; and densification that prunes every Gaussian or is
given none."""
import numpy as np
import pytest
import torch

from oracle import densify as OD
from oracle import project, render
from paper_2503_18402_amd import densify, gsmi, raster, scenes
from tests import gpu_util as U

pytestmark = pytest.mark.gpu

IMG_TOL = 1e-5


@pytest.mark.parametrize("tile", [8, 16])
def test_tiny_and_ragged_views_match_oracle(tile):
    sc, _ = scenes.small_scene()
    sc = scenes.subset(sc, slice(0, 1500))
    sizes = [(1, 1), (7, 3), (17, 9), (128, 96)]
    cams = [scenes.look_at((0.3 * k, -0.2, -3.0), (0, 0, 0), w, h, 120.0 * w / 128.0)
            for k, (w, h) in enumerate(sizes)]
    Ps = [project.project(sc, c, tile=tile) for c in cams]
    Fs = [render.render_fwd(P) for P in Ps]
    ups = [U.zero_flagged(scenes.random_upstream(c, seed=70 + k), F)
           for k, (c, F) in enumerate(zip(cams, Fs))]
    _, frame, g = U.run(sc, cams, tile=tile, upstream=ups, want_keys=False)
    ref, bnd, skip, off = None, None, np.zeros(1500, bool), 0
    for c, u, P, F in zip(cams, ups, Ps, Fs):
        B = render.render_bwd(sc, P, u, with_bound=True)
        npx = 3 * c.width * c.height
        img = frame.image[off:off + npx].view(3, c.height, c.width).cpu().numpy()
        ok = ~F["flag"].reshape(c.height, c.width)
        assert np.abs(img - F["image"].reshape(3, c.height, c.width))[:, ok].max(initial=0) < IMG_TOL
        off += npx
        skip |= U.gaussian_flags(P)
        ref = {k: B["d_" + k] for k in raster.PARAM_NAMES} if ref is None else \
            {k: ref[k] + B["d_" + k] for k in raster.PARAM_NAMES}
        bnd = {k: B["bound"]["d_" + k] for k in raster.PARAM_NAMES} if bnd is None else \
            {k: bnd[k] + B["bound"]["d_" + k] for k in raster.PARAM_NAMES}
    for name in raster.PARAM_NAMES:
        U.check_grads(g[name], ref[name], bnd[name], mask=~skip, name=name,
                      max_frac=U.MEANS_CANCELLATION_FRAC if name == "means" else 0.0)


def test_largest_batch_equals_plain_views():
    sc, _ = scenes.small_scene()
    sc = scenes.subset(sc, slice(0, 2000))
    cams = scenes.orbit_cameras(gsmi.GS_MAX_VIEWS, 3.0, 64, 48, 60.0)
    ups = [scenes.random_upstream(c, seed=100 + k) for k, c in enumerate(cams)]
    _, fb, gb = U.run(sc, cams, upstream=ups, want_keys=False)
    gsum, off = None, 0
    for k, c in enumerate(cams):
        _, fp, gp = U.run(sc, [c], upstream=[ups[k]], want_keys=False)
        npx = 3 * c.width * c.height
        # both launches have few tiles, so every list takes the same path
        assert torch.equal(fb.image[off:off + npx], fp.image), k
        off += npx
        gsum = gp if gsum is None else {n: gsum[n] + gp[n] for n in gsum}
    for name in gsum:   # the same per-view kernels; only the float32 order over views differs
        scale = np.abs(gsum[name]).max() + 1e-12
        assert np.abs(gb[name] - gsum[name]).max() <= 1e-5 * scale, name
    with pytest.raises(RuntimeError):
        U.run(sc, scenes.orbit_cameras(gsmi.GS_MAX_VIEWS + 1, 3.0, 64, 48, 60.0))


def _dev(d):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in d.items()}


@pytest.mark.parametrize("n", [0, 700])
def test_densify_everything_pruned_or_nothing_given(n):
    rng = np.random.default_rng(7)
    p = dict(means=rng.uniform(-1, 1, (n, 3)), log_scales=rng.normal(-3, 0.5, (n, 3)),
             quats=rng.normal(size=(n, 4)), opacity_logits=rng.normal(-6.0, 0.3, n),
             sh=rng.normal(0, 0.1, (n, 16, 3)))
    p = {k: v.astype(np.float32) for k, v in p.items()}
    accum = rng.uniform(0, 1, n).astype(np.float32)
    count = np.ones(n, np.float32)
    z = rng.normal(size=(n, 2, 3)).astype(np.float32)
    mom = {k: np.zeros_like(v) for k, v in p.items()}
    # min opacity 0.05: every sigmoid(-6 +- 1) is below it
    _, _, info_o = OD.densify({k: v.astype(np.float64) for k, v in p.items()}, {},
                              accum, count, z.astype(np.float64), 0.1, 0.05, 0.01, 10)
    assert info_o["n_new"] == 0
    newp, newm, newv, info = densify.densify_step(
        _dev(p), _dev(mom), _dev(mom), torch.from_numpy(accum).cuda(),
        torch.from_numpy(count).cuda(), torch.from_numpy(z).cuda(), 0.1, 0.05, 0.01,
        lambda kept, cand: 10)
    torch.cuda.synchronize()
    assert info["n_new"] == 0 and info["n_pruned"] == n
    for name in raster.PARAM_NAMES:
        assert newp[name].shape[0] == 0 and newm[name].shape[0] == 0
