"""The forward blend with the L1 loss gradient written beside the image
(gs_render_fwd_l1) against the two calls it replaces (gs_render_fwd, then
gs_l1_loss_grad) on the same binned lists: image, final_T, last_contrib and
dL/dimage agree bit for bit, and every element is written (the outputs start
as NaN / all ones).  The loss value is a sum of per-workgroup float atomics in
both, so it agrees to float rounding.  Cases: the per-tile kernel alone (tile
32, and a view of more than 2048 tiles with a ragged edge), the list-parallel
kernel of a low-resolution view, a batch of views at different resolutions,
and a white background.  A quarter of the target equals the image exactly, so
sign(0) = 0 is exercised.  The separate calls are checked against the FP64
oracle in test_gpu_parity.py."""
import pytest
import torch

from paper_2503_18402_amd import gsmi, raster, scenes

pytestmark = pytest.mark.gpu


def _cams(case):
    if case == "wide":   # 1000x712 at tile 16: 63x45 tiles, ragged on both edges
        return [scenes.look_at((0, 0, -3), (0, 0, 0), 1000, 712, 900.0)], 16
    if case == "tile32":
        return [scenes.look_at((0, 0, -3), (0, 0, 0), 200, 136, 180.0)], 32
    if case == "long":   # 48 tiles of long lists: the list-parallel kernel
        return [scenes.look_at((0, 0, -3), (0, 0, 0), 128, 96, 120.0)], 16
    base = scenes.orbit_cameras(4, 3.0, 160, 120, 150.0)
    return [scenes.downscale(base[0], 4), scenes.downscale(base[1], 2), base[2], base[3]], 8


@pytest.mark.parametrize("case,bg", [("wide", (0.0, 0.0, 0.0)), ("tile32", (0.0, 0.0, 0.0)),
                                     ("long", (1.0, 1.0, 1.0)), ("batch", (0.2, 0.5, 0.9))])
def test_forward_l1_equals_separate_calls(case, bg):
    cams, tile = _cams(case)
    sc = scenes.make_scene(20001, seed=71, mean_range=1.0, ls_mu=-3.5, ls_sigma=0.3)
    tgt0 = torch.zeros(sum(3 * c.width * c.height for c in cams), device="cuda")
    pipe = raster.Pipeline(raster.to_device(sc), cams, tgt0, tile=tile, lds_batch=128, bg=bg)
    pipe.forward()
    torch.cuda.synchronize()
    assert not pipe.overflowed()
    # target: the image itself on a quarter of the elements, shifted up or down elsewhere
    tgt = pipe.image.clone()
    tgt[0::4] += 0.05
    tgt[1::4] -= 0.05
    tgt[2::4] += 1e-7
    scale = 1.0 / pipe.image.numel()
    dl_a = torch.full_like(pipe.image, float("nan"))
    loss_a = torch.zeros(1, device="cuda")
    gsmi.gs_l1_loss_grad(pipe.image, tgt, scale, dl_a, loss_a)

    img_b = torch.full_like(pipe.image, float("nan"))
    ft_b = torch.full_like(pipe.final_T, float("nan"))
    last_b = torch.full_like(pipe.last, -1)
    dl_b = torch.full_like(pipe.image, float("nan"))
    loss_b = torch.zeros(1, device="cuda")
    gsmi.gs_render_fwd_l1(pipe.cams_c, pipe.cfg, pipe.n, pipe.proj, pipe.ranges, pipe.vals,
                          img_b, ft_b, last_b, tgt, scale, dl_b, loss_b)
    # without a loss pointer: the same gradient
    dl_c = torch.full_like(pipe.image, float("nan"))
    gsmi.gs_render_fwd_l1(pipe.cams_c, pipe.cfg, pipe.n, pipe.proj, pipe.ranges, pipe.vals,
                          img_b, ft_b, last_b, tgt, scale, dl_c, None)
    torch.cuda.synchronize()
    assert torch.equal(img_b, pipe.image)
    assert torch.equal(ft_b, pipe.final_T)
    assert torch.equal(last_b, pipe.last)
    assert torch.equal(dl_b, dl_a)
    assert torch.equal(dl_c, dl_a)
    assert (dl_a == 0).float().mean().item() >= 0.25
    assert (dl_a > 0).any() and (dl_a < 0).any()
    # recursive float summation of positive terms: relative error at most (terms - 1) u,
    # u = 2^-24, over the longest chain (a thread's pixels, the wave and block
    # reductions, then one atomic per workgroup: at most one per tile, or 1024 for
    # gs_l1_loss_grad)
    ref = float((pipe.image.double() - tgt.double()).abs().sum() * scale)
    chain = max(gsmi.gs_total_tiles(pipe.cams_c, pipe.cfg), 1024) + 64
    assert abs(loss_b.item() - ref) <= chain * 2.0 ** -24 * ref
    assert abs(loss_a.item() - ref) <= chain * 2.0 ** -24 * ref


def test_pipeline_step_uses_the_fused_forward():
    """Pipeline.step() (fused forward + L1) leaves the same dL and loss as the
    separate forward and gs_l1_loss_grad."""
    cams, tile = _cams("batch")
    sc = scenes.make_scene(5003, seed=72, mean_range=1.0, ls_mu=-3.5, ls_sigma=0.3)
    tgt = torch.cat([torch.from_numpy(scenes.uniform_target(c, seed=73 + k)).reshape(-1)
                     for k, c in enumerate(cams)]).cuda()
    pa = raster.Pipeline(raster.to_device(sc), cams, tgt, tile=tile, lds_batch=128)
    pb = raster.Pipeline(raster.to_device(sc), cams, tgt, tile=tile, lds_batch=128,
                         capacity=pa.capacity)
    pa.forward()
    pa.backward_adam()          # separate L1 call
    pb.forward(l1=True)
    pb.backward_adam(l1_done=True)
    torch.cuda.synchronize()
    assert torch.equal(pa.dL, pb.dL)
    chain = max(gsmi.gs_total_tiles(pa.cams_c, pa.cfg), 1024) + 64
    assert abs(pa.loss.item() - pb.loss.item()) <= 2 * chain * 2.0 ** -24 * abs(pa.loss.item())
    for name in raster.PARAM_NAMES:
        assert torch.equal(pa.params[name], pb.params[name]), name
