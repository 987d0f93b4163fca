"""The resolution schedule's device parts against the FP64 oracle: the
frequency map of Eq. 2 (natural DFT order, mean over views of the
channel-norm of the unnormalised DFT), the anti-aliased ground-truth
downsampling, and the knots computed end to end from the device map."""
import numpy as np
import pytest
import torch

from oracle import schedule as O
from paper_2503_18402_amd import gsmi, raster, scenes

pytestmark = pytest.mark.gpu


def _freq_map(imgs_np):
    n, _, H, W = imgs_np.shape
    x = torch.from_numpy(np.ascontiguousarray(imgs_np, np.float32)).cuda()
    mag = torch.empty(H, W, dtype=torch.float64, device="cuda")
    ws = torch.empty(gsmi.gs_frequency_map_workspace_bytes(H, W), dtype=torch.uint8,
                     device="cuda")
    gsmi.gs_frequency_map(x, H, W, mag, ws)
    torch.cuda.synchronize()
    return mag.cpu().numpy()


@pytest.mark.parametrize("shape", [(3, 3, 96, 128), (2, 3, 133, 200), (1, 3, 45, 61),
                                   (1, 3, 7, 1), (1, 3, 1064, 1600)])
def test_frequency_map_matches_oracle(shape):
    imgs = np.random.default_rng(sum(shape)).uniform(size=shape).astype(np.float32)
    got = _freq_map(imgs)
    ref = np.fft.ifftshift(O.magnitude_map(imgs.astype(np.float64)))
    assert np.abs(got - ref).max() <= 1e-10 * ref.max()


@pytest.mark.parametrize("H,W,h,w", [(1064, 1600, 133, 200), (800, 1200, 266, 400),
                                     (97, 131, 31, 17), (40, 30, 80, 45), (64, 64, 64, 64),
                                     (1080, 1920, 540, 960)])
def test_downsample_matches_oracle(H, W, h, w):
    x = np.random.default_rng(H + w).uniform(size=(2, 3, H, W)).astype(np.float32)
    src = torch.from_numpy(x).cuda()
    dst = torch.empty(2 * 3 * h * w, device="cuda")
    gsmi.gs_downsample_aa(src, 6, H, W, h, w, dst)
    torch.cuda.synchronize()
    got = dst.view(2, 3, h, w).cpu().numpy()
    ref = np.stack([O.downsample_aa(x[k].astype(np.float64), h, w) for k in range(2)])
    assert np.abs(got - ref).max() < 2e-6


@pytest.mark.parametrize("norm", ["sum", "mean"])
def test_knots_from_rendered_views(norm):
    """Render views of a scene, build the map on the device, solve the knots on
    the host, and compare with the oracle's knots from its own map."""
    sc = scenes.make_scene(20000, seed=61, mean_range=1.0, ls_mu=-3.5, ls_sigma=0.6)
    cams = scenes.orbit_cameras(4, 3.0, 200, 150, 180.0)
    params = raster.to_device(sc, "cuda")
    imgs = torch.stack([raster.render(params, [c]).image.view(3, 150, 200) for c in cams])
    torch.cuda.synchronize()
    imgs_np = imgs.cpu().numpy()
    got = _freq_map(imgs_np)
    r_c, s_c = gsmi.gs_resolution_schedule(got, 6000, a=4.0, m=4, norm=norm)
    r_o, s_o, _ = O.schedule_knots(O.magnitude_map(imgs_np.astype(np.float64)), 6000, a=4.0, m=4,
                                   norm=norm)
    assert np.allclose(r_c, r_o, rtol=1e-9) and np.allclose(s_c, s_o, rtol=1e-12, atol=1e-9)
    assert r_c[-1] > 1.2
