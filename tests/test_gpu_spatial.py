"""The spatial storage order (gs_spatial_order, gs_gather_rows) against the
oracle's definition (oracle/spatial.py): the permutation bit for bit, the
row gather, and the rasterizer's independence of the order: the same image
and the same gradients, moved with their Gaussians."""
import numpy as np
import pytest
import torch

from oracle import project, spatial
from paper_2503_18402_amd import gsmi, raster, scenes
from tests import gpu_util as U

pytestmark = pytest.mark.gpu


def _perm(means_np):
    m = torch.from_numpy(np.ascontiguousarray(means_np, np.float32)).cuda()
    n = m.shape[0]
    perm = torch.full((max(n, 1),), -1, dtype=torch.int32, device="cuda")
    ws = torch.empty(max(gsmi.gs_spatial_order_workspace_bytes(n), 16), dtype=torch.uint8,
                     device="cuda")
    gsmi.gs_spatial_order(n, m, ws, perm)
    torch.cuda.synchronize()
    return perm[:n].cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("n,spread", [(1, 1.0), (4097, 1.0), (1_000_000, 4.0)])
def test_order_matches_oracle(n, spread):
    m = np.random.default_rng(80 + n % 7).uniform(-spread, spread, size=(n, 3)).astype(np.float32)
    if n > 100:
        m[n // 2:n // 2 + n // 10] = m[:n // 10]          # equal means: ties by index
    assert np.array_equal(_perm(m), spatial.morton_order(m))


def test_order_degenerate_inputs():
    assert _perm(np.zeros((0, 3), np.float32)).shape == (0,)
    assert list(_perm(np.ones((9, 3), np.float32))) == list(range(9))
    m = np.stack([np.arange(300, dtype=np.float32)[::-1], np.zeros(300, np.float32),
                  np.full(300, 2.5, np.float32)], 1)
    assert np.array_equal(_perm(m), spatial.morton_order(m))


def test_gather_rows_moves_every_group():
    sc, _ = scenes.small_scene()
    p = raster.to_device(sc, "cuda")
    m = {k: torch.randn_like(v) for k, v in p.items()}
    v = {k: torch.rand_like(t) for k, t in p.items()}
    perm, p2, m2, v2 = raster.spatial_order(p, m, v)
    idx = perm.long()
    assert np.array_equal(perm.cpu().numpy(), spatial.morton_order(sc["means"]))
    for src, dst in ((p, p2), (m, m2), (v, v2)):
        for k in raster.PARAM_NAMES:
            assert torch.equal(dst[k], src[k][idx]), k


def test_render_and_gradients_independent_of_order():
    """Every depth of this scene is distinct, so no tie-break changes: the image
    is bit-identical and each Gaussian's gradients move with it bit for bit."""
    sc, cam = scenes.small_scene()
    # three pairs of this scene share a float32 depth: move one of each apart
    z = project.depth_f32(sc["means"], cam.R, cam.t)
    _, first = np.unique(z, return_index=True)
    dup = np.setdiff1d(np.arange(len(z)), first)
    sc["means"][dup, 2] += np.float32(1e-3)
    assert len(np.unique(project.depth_f32(sc["means"], cam.R, cam.t))) == len(z)
    w = torch.from_numpy(scenes.random_upstream(cam)).cuda().reshape(-1)
    p = raster.to_device(sc, "cuda")
    perm, q = raster.spatial_order(p)
    idx = perm.long()
    assert not torch.equal(idx, torch.arange(len(idx), device="cuda"))
    fa = raster.render(p, [cam])
    fb = raster.render(q, [cam])
    assert torch.equal(fa.image, fb.image) and torch.equal(fa.final_T, fb.final_T)
    ga = raster.render_backward(p, fa, w)
    gb = raster.render_backward(q, fb, w)
    for k in raster.PARAM_NAMES:
        assert torch.equal(gb[k], ga[k][idx]), k
