"""The LSD radix-sort binning (gs_bin_sort_radix) against the bucket-and-tile-
sort binning (gs_bin_sort) and the oracle: the stable sort of the (tile |
depth) keys is unique, so keys, values, ranges and the pair count must agree
bit for bit, here on the 4096-Gaussian view, a multi-resolution batch, tile
lists longer than every per-tile sort tier, the 1M-Gaussian view, an empty
scene and a capacity overflow."""
import numpy as np
import pytest
import torch

from oracle import binning, project
from paper_2503_18402_amd import gsmi, raster, scenes

pytestmark = pytest.mark.gpu


def _both(sc, cams, tile=16, cap=None):
    params = raster.to_device(sc, "cuda")
    fr = raster.render(params, cams, tile=tile, want_keys=True, capacity=cap)
    cap = fr.capacity
    n = params["means"].shape[0]
    ws = torch.empty(max(gsmi.gs_bin_sort_radix_workspace_bytes(len(cams), n, cap), 16),
                     dtype=torch.uint8, device="cuda")
    keys = torch.empty(max(cap, 1), dtype=torch.int64, device="cuda")
    vals = torch.empty(max(cap, 1), dtype=torch.int32, device="cuda")
    ranges = torch.empty_like(fr.ranges)
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    gsmi.gs_bin_sort_radix(fr.cams_c, fr.cfg, n, fr.proj, cap, ws, keys, vals, ranges, npairs)
    torch.cuda.synchronize()
    return fr, keys, vals, ranges, npairs


def _same(fr, keys, vals, ranges, npairs):
    np_ = int(fr.n_pairs_dev.item())
    assert int(npairs.item()) == np_
    assert torch.equal(keys[:np_], fr.keys[:np_])
    assert torch.equal(vals[:np_], fr.vals[:np_])
    assert torch.equal(ranges, fr.ranges)
    return np_


def test_radix_equals_bucket_and_oracle_small_scene():
    sc, cam = scenes.small_scene()
    fr, keys, vals, ranges, npairs = _both(sc, [cam])
    np_ = _same(fr, keys, vals, ranges, npairs)
    P = project.project(sc, cam, tile=16)
    if not P["flag_rect"].any():
        k, v, r = binning.bin_sort(P["rect"], P["tiles_touched"], P["depth_f32"], 8, 6)
        assert np.array_equal(keys[:np_].cpu().numpy().view(np.uint64), k)
        assert np.array_equal(vals[:np_].cpu().numpy().view(np.uint32), v)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_radix_equals_bucket_multiview(tile):
    sc, _ = scenes.small_scene()
    base = scenes.orbit_cameras(4, 3.0, 160, 120, 150.0)
    cams = [scenes.downscale(base[0], 4), scenes.downscale(base[1], 2), base[2], base[3]]
    _same(*_both(sc, cams, tile=tile))


def test_radix_equals_bucket_long_lists():
    sc = scenes.make_scene(40000, seed=43, mean_range=0.2, ls_mu=-3.0, ls_sigma=0.2)
    cam = scenes.look_at((0.0, 0.0, -3.0), (0.0, 0.0, 0.0), 32, 32, 40.0)
    fr, *rest = _both(sc, [cam])
    assert np.diff(fr.ranges.cpu().numpy().reshape(-1, 2), axis=1).max() > 16384
    _same(fr, *rest)


def test_radix_equals_bucket_paper_scale():
    sc, cam = scenes.paper_scale_scene(level=1)
    _same(*_both(sc, [cam]))


def test_radix_empty_and_overflow():
    sc, cam = scenes.small_scene()
    _same(*_both(scenes.subset(sc, slice(0, 0)), [cam]))
    params = raster.to_device(sc, "cuda")
    fr = raster.render(params, [cam])
    need = int(fr.n_pairs_dev.item())
    cap = need // 2
    ws = torch.empty(gsmi.gs_bin_sort_radix_workspace_bytes(1, 4096, cap), dtype=torch.uint8,
                     device="cuda")
    vals = torch.empty(cap, dtype=torch.int32, device="cuda")
    ranges = torch.empty_like(fr.ranges)
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    gsmi.gs_bin_sort_radix(fr.cams_c, fr.cfg, 4096, fr.proj, cap, ws, None, vals, ranges, npairs)
    torch.cuda.synchronize()
    assert int(npairs.item()) == need   # reported, so the caller can grow and call again
