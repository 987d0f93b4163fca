"""Rasterizer front end over the C ABI: buffer management and autograd.

``render`` runs preprocess -> bin_sort -> render_fwd for one or several views
(several views go into ONE launch per kernel: the batched form) and returns a
``Frame`` holding every device buffer the backward needs.  ``render_backward``
runs gs_render_bwd on that frame.  ``RasterizeFn`` wraps both as a
``torch.autograd.Function``.  Nothing here computes: it allocates, calls the
library, and checks the one device-side overflow count.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import gsmi

PARAM_NAMES = ("means", "log_scales", "quats", "opacity_logits", "sh")


@dataclass
class Frame:
    cams_c: object
    cfg: object
    n: int
    sh_degree: int
    proj: torch.Tensor
    vals: torch.Tensor
    keys: torch.Tensor | None
    ranges: torch.Tensor
    n_pairs_dev: torch.Tensor
    capacity: int
    image: torch.Tensor          # [sum 3*H*W] concatenated per view
    final_T: torch.Tensor
    last_contrib: torch.Tensor
    sizes: list = field(default_factory=list)   # (W, H) per view
    filter3d: object = None      # the 3D filter variances the cfg points at (kept alive)

    def images(self):
        """Per-view [3,H,W] views into the concatenated image."""
        out, off = [], 0
        for (W, H) in self.sizes:
            out.append(self.image[off:off + 3 * W * H].view(3, H, W))
            off += 3 * W * H
        return out

    def pixel_views(self, t):
        out, off = [], 0
        for (W, H) in self.sizes:
            out.append(t[off:off + W * H].view(H, W))
            off += W * H
        return out


def _aligned(t: torch.Tensor) -> torch.Tensor:
    t = t.contiguous()
    if t.data_ptr() % 16:
        t = t.clone()
    return t


def default_capacity(n: int, n_views: int) -> int:
    return max(1024, 8 * n * n_views)


def render(params: dict, cams, tile: int = 16, lds_batch: int = 256, bg=(0.0, 0.0, 0.0),
           sh_degree: int = 3, capacity: int | None = None, want_keys: bool = False,
           check_capacity: bool = True, stream=None, mip2d: bool = False,
           filter3d: torch.Tensor | None = None) -> Frame:
    """Forward pass for the cameras ``cams`` (one launch per kernel for all views).

    With ``check_capacity`` the pair count is read back once (one 8-byte copy)
    and the sort is re-run with a larger buffer if it overflowed.  ``mip2d``
    and ``filter3d`` select Mip-Splatting's filters (see gs_raster_cfg); the
    frame keeps ``filter3d`` alive for the backward.
    """
    dev = params["means"].device
    n = params["means"].shape[0]
    cams_c = gsmi.make_cameras(cams)
    cfg = gsmi.make_cfg(tile, lds_batch, bg, mip2d=mip2d, filter3d=filter3d)
    nv = len(cams)
    quats = _aligned(params["quats"])
    proj = torch.empty(max(gsmi.gs_proj_bytes(nv, n), 16), dtype=torch.uint8, device=dev)
    gsmi.gs_preprocess(cams_c, cfg, n, params["means"], params["log_scales"], quats,
                       params["opacity_logits"], params["sh"], sh_degree, proj, stream)
    cap = default_capacity(n, nv) if capacity is None else int(capacity)
    total_tiles = gsmi.gs_total_tiles(cams_c, cfg)
    ranges = torch.empty(2 * max(total_tiles, 1), dtype=torch.int32, device=dev)
    n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
    while True:
        ws = torch.empty(max(gsmi.gs_bin_sort_workspace_bytes(nv, n, cap), 16), dtype=torch.uint8,
                         device=dev)
        vals = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        keys = torch.empty(max(cap, 1), dtype=torch.int64, device=dev) if want_keys else None
        gsmi.gs_bin_sort(cams_c, cfg, n, proj, cap, ws, keys, vals, ranges, n_pairs, stream)
        if not check_capacity:
            break
        np_ = int(n_pairs.item())
        if np_ <= cap:
            break
        cap = int(np_ * 1.25) + 1024
    del ws
    npx = sum(int(c.width) * int(c.height) for c in cams)
    image = torch.empty(3 * npx, dtype=torch.float32, device=dev)
    final_T = torch.empty(npx, dtype=torch.float32, device=dev)
    last = torch.empty(npx, dtype=torch.int32, device=dev)
    gsmi.gs_render_fwd(cams_c, cfg, n, proj, ranges, vals, image, final_T, last, stream)
    fr = Frame(cams_c=cams_c, cfg=cfg, n=n, sh_degree=sh_degree, proj=proj, vals=vals,
               keys=keys, ranges=ranges, n_pairs_dev=n_pairs, capacity=cap, image=image,
               final_T=final_T, last_contrib=last,
               sizes=[(int(c.width), int(c.height)) for c in cams], filter3d=filter3d)
    return fr


def zero_grads(params: dict) -> dict:
    return {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}


def render_backward(params: dict, frame: Frame, dL_dimage: torch.Tensor, grads: dict | None = None,
                    mean2d_abs: torch.Tensor | None = None, stream=None,
                    accumulate: bool = True) -> dict:
    """Parameter gradients of L given dL/dimage (concatenated layout), added to
    ``grads`` (``accumulate``) or written over them."""
    if grads is None:
        grads = zero_grads(params)
    n = frame.n
    dev = params["means"].device
    ws = torch.empty(max(gsmi.gs_render_bwd_workspace_bytes(len(frame.sizes), n, frame.capacity),
                         16), dtype=torch.uint8, device=dev)
    gsmi.gs_render_bwd(frame.cams_c, frame.cfg, n, params["means"], params["log_scales"],
                       _aligned(params["quats"]), params["opacity_logits"], params["sh"],
                       frame.sh_degree, frame.proj, frame.ranges, frame.vals, frame.final_T,
                       frame.last_contrib, dL_dimage.contiguous(), grads["means"],
                       grads["log_scales"], grads["quats"], grads["opacity_logits"], grads["sh"],
                       mean2d_abs, frame.capacity, ws, stream, accumulate=accumulate)
    return grads


class RasterizeFn(torch.autograd.Function):
    """image = RasterizeFn.apply(means, log_scales, quats, opacity_logits, sh, settings)

    ``settings`` is a dict with ``cams`` and optionally tile, lds_batch, bg,
    sh_degree, mip2d, filter3d.  The forward keeps only the frame buffers (projected records,
    sorted pair values, ranges, final T and last contributor per pixel); the
    backward recomputes each pixel's blend state from them.

    Optional settings for a training loop: ``capacity`` (pair capacity) with
    ``check_capacity`` False skips the forward's read-back of the pair count
    (the caller checks the frame's ``n_pairs_dev`` later); ``mean2d_abs`` (a
    device [n] tensor) receives the backward's |dL/dmean2D| statistic (added
    to it); the forward stores its frame in ``settings["frame"]``.
    """

    @staticmethod
    def forward(ctx, means, log_scales, quats, opacity_logits, sh, settings):
        params = dict(means=means.detach().contiguous(), log_scales=log_scales.detach().contiguous(),
                      quats=quats.detach().contiguous(),
                      opacity_logits=opacity_logits.detach().contiguous(),
                      sh=sh.detach().contiguous())
        frame = render(params, settings["cams"], tile=settings.get("tile", 16),
                       lds_batch=settings.get("lds_batch", 256),
                       bg=settings.get("bg", (0.0, 0.0, 0.0)),
                       sh_degree=settings.get("sh_degree", 3),
                       mip2d=settings.get("mip2d", False), filter3d=settings.get("filter3d"),
                       capacity=settings.get("capacity"),
                       check_capacity=settings.get("check_capacity", True))
        ctx.frame = frame
        ctx.params = params
        ctx.mean2d_abs = settings.get("mean2d_abs")
        if "frame" in settings:
            settings["frame"] = frame
        return frame.image.clone()

    @staticmethod
    def backward(ctx, dL_dimage):
        g = render_backward(ctx.params, ctx.frame, dL_dimage.float(), mean2d_abs=ctx.mean2d_abs)
        return g["means"], g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], None


def spatial_order(params: dict, *moments: dict, stream=None):
    """The Gaussians re-stored in the Morton order of their means
    (gs_spatial_order, then gs_gather_rows over the parameters and any Adam
    moment dicts given).  Returns (perm, params, *moments) as new tensors;
    perm[k] is the old index of the k-th Gaussian.  Rendering results do not
    depend on the order (ties of exactly equal depth follow the index)."""
    n = params["means"].shape[0]
    dev = params["means"].device
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    ws = torch.empty(max(gsmi.gs_spatial_order_workspace_bytes(n), 16), dtype=torch.uint8,
                     device=dev)
    gsmi.gs_spatial_order(n, params["means"], ws, perm, stream)
    groups = [params] + list(moments)
    src = [g[k].contiguous() for g in groups for k in PARAM_NAMES]
    dst = [torch.empty_like(t) for t in src]
    if n > 0:
        gsmi.gs_gather_rows(n, perm, src, dst, stream)
    out, i = [], 0
    for _ in groups:
        out.append({k: dst[i + j] for j, k in enumerate(PARAM_NAMES)})
        i += len(PARAM_NAMES)
    return (perm[:n], *out)


def to_device(scene: dict, device="cuda") -> dict:
    """numpy scene -> contiguous float32 device tensors."""
    return {k: torch.from_numpy(scene[k]).to(device=device, dtype=torch.float32).contiguous()
            for k in PARAM_NAMES}


class Pipeline:
    """Preallocated buffers for one training step over a fixed set of views.

    ``step()`` enqueues the whole hot path on the current stream with no host
    synchronisation and no allocation: preprocess, bin_sort, render_fwd with
    the L1 loss gradient against ``targets`` (one ``gs_render_fwd_l1`` call),
    render_bwd and one fused Adam step over all parameter groups.  Every view of the set goes into one launch per
    kernel.  ``overflowed()`` reads the pair count once to check the capacity
    after the fact; a captured HIP graph of ``step()`` replays the same work.

    With ``fused`` (the default) the backward and the Adam step run as one
    ``gs_render_bwd_adam`` call: the same update bit for bit, without writing
    the gradients (``grads`` is then left untouched by ``step()``).  With
    ``sparse_adam`` the fused call is ``gs_render_bwd_sparse_adam``: Gaussians
    no view of the set touches keep their parameters and moments.
    """

    def __init__(self, params: dict, cams, targets: torch.Tensor, tile: int = 16,
                 lds_batch: int = 256, bg=(0.0, 0.0, 0.0), sh_degree: int = 3,
                 capacity: int | None = None, lrs: dict | None = None,
                 betas=(0.9, 0.999), eps: float = 1e-15, grads: dict | None = None,
                 fused: bool = True, share: "Pipeline | None" = None,
                 state: tuple | None = None, mean2d_abs: torch.Tensor | None = None,
                 sparse_adam: bool = False, mip2d: bool = False,
                 filter3d: torch.Tensor | None = None, cam_table: torch.Tensor | None = None,
                 cam_index: torch.Tensor | None = None, adam_lr: torch.Tensor | None = None):
        if sparse_adam and not fused:
            raise ValueError("sparse Adam runs fused with the backward pass")
        self.params = params
        self.cams = list(cams)
        dev = params["means"].device
        self.n = params["means"].shape[0]
        self.nv = len(self.cams)
        self.cams_c = gsmi.make_cameras(self.cams)
        # kept alive: the cfg holds their addresses.  With a camera table (one view),
        # every call takes view 0's camera from cam_table[*cam_index] and the L1
        # target from the stack `targets` at that index; with adam_lr the fused
        # Adam step reads its learning rates from the device
        self.filter3d, self.cam_table, self.cam_index, self.adam_lr = (filter3d, cam_table,
                                                                      cam_index, adam_lr)
        self.cfg = gsmi.make_cfg(tile, lds_batch, bg, mip2d=mip2d, filter3d=filter3d,
                                 cam_table=cam_table, cam_index=cam_index, adam_lr=adam_lr)
        self.sh_degree = sh_degree
        self.npx = sum(int(c.width) * int(c.height) for c in self.cams)
        self.targets = targets.contiguous()
        if capacity is None:
            if cam_table is not None:
                raise ValueError("a pipeline with a camera table needs its capacity")
            probe = render(params, self.cams, tile=tile, lds_batch=lds_batch, bg=bg,
                           sh_degree=sh_degree, mip2d=mip2d, filter3d=filter3d)
            capacity = int(int(probe.n_pairs_dev.item()) * 1.2) + 4096
            del probe
        self.capacity = int(capacity)
        u8 = dict(dtype=torch.uint8, device=dev)
        self.proj = torch.empty(max(gsmi.gs_proj_bytes(self.nv, self.n), 16), **u8)
        self.sort_ws = torch.empty(
            max(gsmi.gs_bin_sort_workspace_bytes(self.nv, self.n, self.capacity), 16), **u8)
        self.bwd_ws = torch.empty(
            max(gsmi.gs_render_bwd_workspace_bytes(self.nv, self.n, self.capacity), 16), **u8)
        self.vals = torch.empty(max(self.capacity, 1), dtype=torch.int32, device=dev)
        self.ranges = torch.empty(2 * max(gsmi.gs_total_tiles(self.cams_c, self.cfg), 1),
                                  dtype=torch.int32, device=dev)
        self.n_pairs = torch.zeros(1, dtype=torch.int64, device=dev)
        self.image = torch.empty(3 * self.npx, dtype=torch.float32, device=dev)
        self.final_T = torch.empty(self.npx, dtype=torch.float32, device=dev)
        self.last = torch.empty(self.npx, dtype=torch.int32, device=dev)
        self.dL = torch.empty(3 * self.npx, dtype=torch.float32, device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)
        if share is not None:  # one optimiser state for several pipelines (e.g. per level)
            self.grads, self.m, self.v = share.grads, share.m, share.v
        elif state is not None:  # (m, v, step_dev) carried over, e.g. across densification
            self.grads = zero_grads(params) if grads is None else grads
            self.m, self.v = state[0], state[1]
        else:
            self.grads = zero_grads(params) if grads is None else grads
            self.m = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
            self.v = {k: torch.zeros_like(params[k]) for k in PARAM_NAMES}
        self.lrs = lrs or dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2,
                               sh=2.5e-3)
        self.betas, self.eps = betas, eps
        self.step_no = 0
        # the step count lives on the device so a captured graph replays as new steps
        self.step_dev = (share.step_dev if share is not None else
                         state[2] if state is not None else
                         torch.zeros(1, dtype=torch.int32, device=dev))
        # |d mean2D| per Gaussian from the fused backward (densification statistics)
        self.mean2d_abs = mean2d_abs
        self.fused = fused
        self.sparse_adam = sparse_adam
        self.track_loss = True   # False: the fused step skips the loss value (gradient only)
        self.graph = None

    def forward(self, stream=None, l1: bool = False):
        """Preprocess, bin_sort and the forward blend.  With ``l1`` the forward also
        writes the L1 loss gradient (``gs_render_fwd_l1``; the loss value too when
        ``track_loss``), so the backward that follows is called with ``l1_done``."""
        p = self.params
        gsmi.gs_preprocess(self.cams_c, self.cfg, self.n, p["means"], p["log_scales"],
                           p["quats"], p["opacity_logits"], p["sh"], self.sh_degree, self.proj,
                           stream)
        gsmi.gs_bin_sort(self.cams_c, self.cfg, self.n, self.proj, self.capacity, self.sort_ws,
                         None, self.vals, self.ranges, self.n_pairs, stream)
        if l1:
            if self.track_loss:
                self.loss.zero_()
            gsmi.gs_render_fwd_l1(self.cams_c, self.cfg, self.n, self.proj, self.ranges,
                                  self.vals, self.image, self.final_T, self.last, self.targets,
                                  1.0 / self.image.numel(), self.dL,
                                  self.loss if self.track_loss else None, stream)
        else:
            gsmi.gs_render_fwd(self.cams_c, self.cfg, self.n, self.proj, self.ranges, self.vals,
                               self.image, self.final_T, self.last, stream)

    def _l1(self, stream):
        if self.track_loss:
            self.loss.zero_()
        gsmi.gs_l1_loss_grad(self.image, self.targets, 1.0 / self.image.numel(), self.dL,
                             self.loss if self.track_loss else None, stream)

    def backward(self, stream=None, accumulate: bool = False, l1_done: bool = False):
        """L1 loss gradient (unless the forward wrote it: ``l1_done``) and
        gs_render_bwd; gradients are written, or added to ``self.grads`` with
        ``accumulate`` (several views sharing one buffer)."""
        p, g = self.params, self.grads
        if not l1_done:
            self._l1(stream)
        gsmi.gs_render_bwd(self.cams_c, self.cfg, self.n, p["means"], p["log_scales"],
                           p["quats"], p["opacity_logits"], p["sh"], self.sh_degree, self.proj,
                           self.ranges, self.vals, self.final_T, self.last, self.dL, g["means"],
                           g["log_scales"], g["quats"], g["opacity_logits"], g["sh"], None,
                           self.capacity, self.bwd_ws, stream, accumulate=accumulate)

    def adam(self, stream=None, step: int | None = None):
        """Adam over all parameter groups; the step count is the device counter
        unless ``step`` is given explicitly."""
        if self.lrs.get("sh_rest", self.lrs["sh"]) != self.lrs["sh"]:
            raise ValueError("a separate SH learning rate above degree 0 needs the fused step")
        groups = [(self.params[k], self.grads[k], self.m[k], self.v[k], self.lrs[k])
                  for k in PARAM_NAMES]
        if step is None:
            gsmi.gs_adam_step_device(groups, self.step_dev, self.betas[0], self.betas[1],
                                     self.eps, stream)
        else:
            gsmi.gs_adam_step(groups, step, self.betas[0], self.betas[1], self.eps, stream)
        self.step_no += 1

    def backward_adam(self, stream=None, l1_done: bool = False):
        """L1 loss gradient (unless ``l1_done``), then the backward pass fused with
        the Adam step (device step counter)."""
        p = self.params
        if not l1_done:
            self._l1(stream)
        gsmi.gs_render_bwd_adam(
            self.cams_c, self.cfg, self.n, p["means"], p["log_scales"], p["quats"],
            p["opacity_logits"], p["sh"], self.sh_degree, self.proj, self.ranges, self.vals,
            self.final_T, self.last, self.dL, [self.m[k] for k in PARAM_NAMES],
            [self.v[k] for k in PARAM_NAMES],
            [self.lrs[k] for k in PARAM_NAMES] + [self.lrs.get("sh_rest", self.lrs["sh"])],
            self.step_dev, self.betas[0], self.betas[1], self.eps, self.mean2d_abs,
            self.capacity, self.bwd_ws, stream, sparse=self.sparse_adam)
        self.step_no += 1

    def step(self, stream=None, adam_step: int | None = None):
        if self.graph is not None and stream is None and adam_step is None:
            self.graph.replay()
            self.step_no += 1
            return
        if self.sparse_adam and adam_step is not None:
            raise ValueError("sparse Adam takes its step count from the device counter")
        self.forward(stream, l1=True)
        if self.fused and adam_step is None:
            self.backward_adam(stream, l1_done=True)
        else:
            self.backward(stream, l1_done=True)
            self.adam(stream, adam_step)

    def set_view(self, cam, target: torch.Tensor):
        """Point a one-view pipeline at another view of the same resolution."""
        if len(self.cams) != 1 or (int(cam.width), int(cam.height)) != (
                int(self.cams[0].width), int(self.cams[0].height)):
            raise ValueError("set_view needs a one-view pipeline and a view of its resolution")
        if self.graph is not None:
            raise ValueError("a captured graph replays its own view")
        self.cams = [cam]
        self.cams_c = gsmi.make_cameras(self.cams)
        self.targets = target.reshape(-1)

    def capture(self):
        """Capture one whole step into a HIP graph; later ``step()`` calls replay it.
        The capacity must already be large enough (``overflowed()`` checks after)."""
        self.forward(l1=True)            # warm every code path once (no parameter update)
        self.backward(l1_done=True)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.forward(l1=True)
            if self.fused:
                self.backward_adam(l1_done=True)
            else:
                self.backward(l1_done=True)
                self.adam()
        self.step_no -= 1                # capturing ran nothing
        self.graph = g
        return g

    def overflowed(self) -> bool:
        return int(self.n_pairs.item()) > self.capacity
