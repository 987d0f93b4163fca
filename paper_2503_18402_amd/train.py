"""Optimisation loop under the frequency-guided resolution schedule (Sec. 4.2;
supplementary Eq. 6-7, "Ground Truth Downsampling", "Learning Rate").

One iteration renders one training view at the scheduled resolution, takes
the L1 loss against the view's ground truth downsampled to that resolution,
and runs the backward pass fused with Adam.  The schedule comes from the
views' frequency map (``gs_frequency_map``, Eq. 2) and the knots of Eq. 7
(``gs_resolution_schedule``); iteration k renders at the integer factor
floor(r(k)); X(F_r) is normalised per pixel by default (see
``gs_resolution_schedule``: with the literal sum of unnormalised DFT magnitudes
natural-image spectra give r_m near a^(1/3), so floor(r) would stay 1).  The
position learning rate is held at its initial value while
floor(r) > 1 and decays exponentially to its final value from the first
full-resolution iteration on.  With ``schedule=False`` every iteration renders
at full resolution and the position rate decays from the start: the
backbone's loop, for comparison.

Two forms of the step: the fused pipeline (``raster.Pipeline``: the L1
gradient written by the forward kernel, the backward fused with Adam), and,
with ``autograd=True``, the differentiable rasterizer as a
``torch.autograd.Function`` (``raster.RasterizeFn``) under a torch L1 loss and
``loss.backward()``, followed by the library's multi-group Adam step.  Both
take the same operations in the same order, so they give the same parameters
bit for bit.  With ``graphs=True`` the fused form runs from one HIP graph per
resolution level: the views, their targets and the per-iteration learning
rates sit in device tables, a device counter picks each iteration's entries,
and every iteration is one replay (bit-identical to the eager loop).  Eager
stepping is the default: on this workload a replay per iteration measured
about 5% slower than launching the step's kernels one by one.

Everything here marshals buffers and calls the C ABI; the arithmetic runs in
the library's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import gsmi, raster


@dataclass
class View:
    """A pinhole camera (the fields the rasterizer reads)."""
    R: np.ndarray
    t: np.ndarray
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int
    near: float = 0.2


def downscale_view(cam, f: int) -> View:
    """The view at integer factor f: floor(W/f) x floor(H/f), focal lengths
    divided by f, principal point at the new image centre."""
    W, H = int(cam.width) // f, int(cam.height) // f
    return View(np.asarray(cam.R, np.float64), np.asarray(cam.t, np.float64), cam.fx / f,
                cam.fy / f, W / 2.0, H / 2.0, W, H, float(getattr(cam, "near", 0.2)))


class ResolutionSchedule:
    """r(k) of Eq. 7 for the ground-truth views ``gt`` (device [N,3,H,W])."""

    def __init__(self, gt: torch.Tensor, iters: int, a: float = 4.0, m: int = 4,
                 r_max: float = 0.0, norm: str = "mean"):
        n, _, H, W = gt.shape
        mag = torch.empty(H, W, dtype=torch.float64, device=gt.device)
        ws = torch.empty(gsmi.gs_frequency_map_workspace_bytes(H, W), dtype=torch.uint8,
                         device=gt.device)
        gsmi.gs_frequency_map(gt.contiguous(), H, W, mag, ws)
        self.mag = mag.cpu().numpy()
        self.iters = iters
        self.r_knots, self.s_knots = gsmi.gs_resolution_schedule(self.mag, iters, a=a, m=m,
                                                                 r_max=r_max, norm=norm)

    def r(self, k: float) -> float:
        return gsmi.gs_schedule_resolution(k, self.r_knots, self.s_knots)

    def factor(self, k: int) -> int:
        return max(1, int(math.floor(self.r(k))))


def downsample(gt: torch.Tensor, h: int, w: int) -> torch.Tensor:
    """Anti-aliased resize of device images [N,3,H,W] to [N,3,h,w]."""
    n, c, H, W = gt.shape
    out = torch.empty(n, c, h, w, dtype=torch.float32, device=gt.device)
    gsmi.gs_downsample_aa(gt.contiguous(), n * c, H, W, h, w, out)
    return out


def psnr(params: dict, cams, gt: torch.Tensor, sh_degree: int = 3, tile: int = 16,
         mip2d: bool = False, filter3d: torch.Tensor | None = None) -> float:
    """Mean PSNR over the views at full resolution (images in [0, 1])."""
    vals = []
    for k, c in enumerate(cams):
        img = raster.render(params, [c], tile=tile, sh_degree=sh_degree, mip2d=mip2d,
                            filter3d=filter3d).image
        mse = torch.mean((img.view_as(gt[k]) - gt[k]) ** 2).item()
        vals.append(-10.0 * math.log10(max(mse, 1e-12)))
    return float(np.mean(vals))


P_FIN_INIT_FACTOR = 5.0   # Sec. 4.3: the budget of Eq. 5 starts at 5 P_init

DEFAULT_LRS = dict(means=1.6e-4, log_scales=5e-3, quats=1e-3, opacity_logits=5e-2, sh=2.5e-3,
                   sh_rest=2.5e-3 / 20.0)


@dataclass
class DensifyConfig:
    """Densification every ``every`` iterations in [start, stop).  ``schedule``:
    densify the top k = P_i - N' candidates with P_i from Eq. 4 (else every
    candidate: the backbone); ``momentum``: grow the budget P_fin by Eq. 5
    from ``p_fin`` (default 5 P_init), else keep ``p_fin`` fixed.  grad_thr
    applies to the 2D-mean gradient in normalised device coordinates (the
    pixel gradient times half the rendered width), so it does not depend on
    the resolution; max_scale = percent_dense * scene extent."""
    every: int = 100
    start: int = 100
    stop: int | None = None
    grad_thr: float = 2e-4
    min_opacity: float = 0.005
    percent_dense: float = 0.01
    extent: float = 1.0
    schedule: bool = True
    momentum: bool = True
    p_fin: float | None = None
    gamma: float = 0.98
    eta: float = 1.0
    seed: int = 0


class Trainer:
    """``iters`` optimisation steps of ``params`` (device tensors, replaced in
    the dict as densification grows them) against ground-truth views ``gt``
    (device [N,3,H,W]) seen from ``cams``.  ``means_lr`` = (initial, final)
    position learning rates; ``r_max`` caps the schedule's downsampling factor
    (0: the smaller image side); ``sparse_adam``: Gaussians the iteration's
    view does not touch keep their parameters and moments; ``mip``: the
    Mip-Splatting backbone's primitives (2D mip filter, and the 3D smoothing
    filter recomputed from the full-resolution views at the start and after
    every densification step)."""

    def __init__(self, params: dict, cams, gt: torch.Tensor, iters: int, schedule: bool = True,
                 a: float = 4.0, m: int = 4, lrs: dict | None = None,
                 means_lr=(1.6e-4, 1.6e-6), sh_degree: int = 3, seed: int = 0,
                 capacity_margin: float = 2.0, norm: str = "mean",
                 densify: DensifyConfig | None = None, r_max: float = 0.0,
                 sparse_adam: bool = False, mip: bool = False, filter3d_scale: float = 0.2,
                 autograd: bool = False, spatial: bool = False, graphs: bool = False):
        self.params, self.cams, self.gt, self.iters = params, list(cams), gt, iters
        # with ``spatial``: Gaussians stored in the spatial (Morton) order of their
        # means, restored after every densification step (the caller's dict is
        # updated in place).  Off by default: at the 50k-300k Gaussians of this
        # loop the binning of spatially ordered Gaussians at full resolution
        # takes its LDS-rectangle route, which costs more there than ranking
        # every pair globally, and the loop measured about 5% slower
        self.spatial = spatial
        if spatial:
            _, ordered = raster.spatial_order(params)
            params.update(ordered)
        self.sh_degree = sh_degree
        self.lrs = dict(DEFAULT_LRS if lrs is None else lrs)
        self.means_lr = means_lr
        self.capacity_margin = capacity_margin
        if autograd and sparse_adam:
            raise ValueError("sparse Adam runs fused with the backward pass")
        self.sparse_adam = sparse_adam
        self.autograd = autograd
        self.graphs = graphs and not autograd
        self.leaves = None
        self.mip, self.filter3d_scale = mip, filter3d_scale
        self.filter3d = None
        self._f3_scratch = torch.zeros(1, dtype=torch.int32, device=params["means"].device)
        self.sched = (ResolutionSchedule(gt, iters, a=a, m=m, r_max=r_max, norm=norm)
                      if schedule else None)
        self.factors = np.array([self.sched.factor(k) if schedule else 1 for k in range(iters)])
        # first iteration at full resolution: the position rate decays from there
        full = np.nonzero(self.factors == 1)[0]
        self.k_full = int(full[0]) if full.size else iters
        self.rng = np.random.default_rng(seed)
        self.dcfg = densify
        dev = params["means"].device
        self.p_init = float(params["means"].shape[0])
        if densify is not None:
            self.p_fin = (float(densify.p_fin) if densify.p_fin is not None
                          else P_FIN_INIT_FACTOR * self.p_init)
            self.zgen = torch.Generator(device=dev).manual_seed(densify.seed)
        self.log = []
        self.lr_log = []   # the position learning rate given to each iteration's step
        # graph mode: the view of each iteration and its six learning rates as device
        # tables, the iteration counter, and the current entries the step reads
        self.k_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.cam_index = torch.zeros(1, dtype=torch.int32, device=dev)
        self.adam_lr = torch.zeros(6, dtype=torch.float32, device=dev)
        self.view_seq = self._view_sequence()
        self.seq_dev = torch.tensor(self.view_seq, dtype=torch.int32, device=dev)
        self.lr_table = torch.tensor([self._lrs6(k) for k in range(iters)], dtype=torch.float32,
                                     device=dev).reshape(iters, 6)
        self.graph_of = {}
        self.step_dev = torch.zeros(1, dtype=torch.int32, device=dev)
        self.m = {k: torch.zeros_like(params[k]) for k in raster.PARAM_NAMES}
        self.v = {k: torch.zeros_like(params[k]) for k in raster.PARAM_NAMES}
        self.gt_levels = {}
        for f in sorted(set(self.factors.tolist()), reverse=True):
            views = [downscale_view(c, f) for c in self.cams]
            h, w = views[0].height, views[0].width
            self.gt_levels[f] = (views, gt if f == 1 else downsample(gt, h, w))
        self._build_levels(0)

    def _view_sequence(self):
        """The view of every iteration: shuffled passes over the views."""
        seq, order = [], []
        for _ in range(self.iters):
            if not order:
                order = list(self.rng.permutation(len(self.cams)))
            seq.append(int(order.pop()))
        return seq

    def _lrs6(self, k: int):
        """The six learning rates of iteration k: the position rate of the
        schedule, then scales, rotations, opacities, SH degree 0 and above."""
        return [self.means_lr_at(k), self.lrs["log_scales"], self.lrs["quats"],
                self.lrs["opacity_logits"], self.lrs["sh"], self.lrs.get("sh_rest", self.lrs["sh"])]

    def _capture(self, f: int):
        """One HIP graph of level f's step: pick the iteration's view and learning
        rates from the device tables, forward with the L1 gradient, backward fused
        with Adam, pair-count and densification statistics, advance the counter."""
        views, _, pipe = self.levels[f]
        pipe.forward(l1=True)           # warm every code path once (no parameter update)
        pipe.backward(l1_done=True)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            torch.index_select(self.seq_dev, 0, self.k_dev, out=self.cam_index)
            torch.index_select(self.lr_table, 0, self.k_dev, out=self.adam_lr.view(1, 6))
            pipe.forward(l1=True)
            pipe.backward_adam(l1_done=True)
            torch.maximum(pipe.pairs_max, pipe.n_pairs, out=pipe.pairs_max)
            gsmi.gs_densify_stats(1, pipe.n, pipe.proj, self.mean2d, self.accum, self.count,
                                  scale=0.5 * views[0].width)
            self.k_dev.add_(1)
        self.graph_of[f] = g

    def _build_levels(self, k0: int):
        """Pipelines for the levels still ahead of iteration k0, sized for the
        current Gaussians, sharing the optimiser state."""
        n = self.params["means"].shape[0]
        dev = self.params["means"].device
        if self.mip:
            self.filter3d = torch.empty(n, device=dev)
            self.update_filter3d()
        self.mean2d = torch.zeros(n, device=dev)
        self.accum = torch.zeros(n, device=dev)
        self.count = torch.zeros(n, device=dev)
        self.levels = {}
        first = None
        probe_views = np.linspace(0, len(self.cams) - 1, min(4, len(self.cams))).astype(int)
        for f in sorted(set(self.factors[k0:].tolist()), reverse=True):
            views, gt_f = self.gt_levels[f]
            tile = self.tile_for(f)
            cap = 0
            for vi in probe_views:
                probe = raster.render(self.params, [views[vi]], tile=tile, sh_degree=self.sh_degree,
                                      mip2d=self.mip, filter3d=self.filter3d)
                cap = max(cap, int(probe.n_pairs_dev.item()))
                del probe
            capacity = int(cap * self.capacity_margin) + 4096
            if self.autograd:
                settings = dict(cams=[views[0]], tile=tile, lds_batch=self.lds_batch_for(f),
                                sh_degree=self.sh_degree, mip2d=self.mip, filter3d=self.filter3d,
                                capacity=capacity, check_capacity=False,
                                mean2d_abs=self.mean2d, frame=None)
                pairs_max = torch.zeros(1, dtype=torch.int64, device=dev)
                self.levels[f] = (views, gt_f, dict(settings=settings, capacity=capacity,
                                                    pairs_max=pairs_max))
                continue
            table = dict(cam_table=gsmi.camera_table(views, dev), cam_index=self.cam_index,
                         adam_lr=self.adam_lr) if self.graphs else {}
            targets = gt_f.reshape(-1) if self.graphs else gt_f[0].reshape(-1)
            pipe = raster.Pipeline(self.params, [views[0]], targets, tile=tile,
                                   lds_batch=self.lds_batch_for(f), sh_degree=self.sh_degree,
                                   capacity=capacity, lrs=self.lrs,
                                   share=first, state=(self.m, self.v, self.step_dev),
                                   mean2d_abs=self.mean2d, sparse_adam=self.sparse_adam,
                                   mip2d=self.mip, filter3d=self.filter3d, **table)
            pipe.pairs_max = torch.zeros(1, dtype=torch.int64, device=dev)
            pipe.track_loss = False   # the loop needs the gradient, not the loss value
            first = first or pipe
            self.levels[f] = (views, gt_f, pipe)
        if self.graphs:
            self.graph_of = {}
            for f in self.levels:
                self._capture(f)

    @staticmethod
    def tile_for(f: int) -> int:
        """Tile size at downsampling factor f: 8 below full resolution (few
        tiles: split them finer), 16 at full resolution."""
        return 8 if f >= 2 else 16

    @staticmethod
    def lds_batch_for(f: int) -> int:
        """Gaussians staged in LDS per blend step at downsampling factor f."""
        return 128

    def update_filter3d(self):
        """Recompute the 3D smoothing filter (in place) from the current means
        and the full-resolution views."""
        gsmi.gs_filter3d_variance(gsmi.make_cameras(self.cams), self.params["means"].shape[0],
                                  self.params["means"], self.filter3d_scale, self.filter3d,
                                  self._f3_scratch)

    def _check_capacity(self):
        for _, _, lvl in self.levels.values():
            pmax, cap = ((lvl["pairs_max"], lvl["capacity"]) if self.autograd
                         else (lvl.pairs_max, lvl.capacity))
            if int(pmax.item()) > cap:
                raise RuntimeError("pair capacity overflowed during training")

    # ---- the autograd form.  The SH coefficients are two leaves, degree 0 and
    # the higher degrees, so that Adam takes them as separate groups with their
    # own learning rates (the fused step's lr[4] and lr[5]).
    GROUPS6 = ("means", "log_scales", "quats", "opacity_logits", "sh_dc", "sh_rest")

    def _split(self):
        p, L = self.params, {}
        for n in raster.PARAM_NAMES[:4]:
            L[n] = p[n].detach().requires_grad_(True)
        L["sh_dc"] = p["sh"][:, :1].clone().requires_grad_(True)
        L["sh_rest"] = p["sh"][:, 1:].clone().requires_grad_(True)
        self.leaves = L
        self.m6, self.v6 = {}, {}
        for d6, d5 in ((self.m6, self.m), (self.v6, self.v)):
            for n in raster.PARAM_NAMES[:4]:
                d6[n] = d5[n]
            d6["sh_dc"] = d5["sh"][:, :1].clone()
            d6["sh_rest"] = d5["sh"][:, 1:].clone()

    def _merge(self):
        L = self.leaves
        for n in raster.PARAM_NAMES[:4]:
            self.params[n] = L[n].detach()
        self.params["sh"] = torch.cat([L["sh_dc"].detach(), L["sh_rest"].detach()], 1)
        for d6, d5 in ((self.m6, self.m), (self.v6, self.v)):
            d5["sh"] = torch.cat([d6["sh_dc"], d6["sh_rest"]], 1)
        self.leaves = None

    def _autograd_step(self, k: int, f: int, v: int):
        views, gt_f, lvl = self.levels[f]
        L, st = self.leaves, lvl["settings"]
        st["cams"] = [views[v]]
        self.mean2d.zero_()
        sh = torch.cat([L["sh_dc"], L["sh_rest"]], 1)
        img = raster.RasterizeFn.apply(L["means"], L["log_scales"], L["quats"],
                                       L["opacity_logits"], sh, st)
        loss = (img - gt_f[v].reshape(-1)).abs().mean()
        loss.backward()
        lr = [self.means_lr_at(k), self.lrs["log_scales"], self.lrs["quats"],
              self.lrs["opacity_logits"], self.lrs["sh"], self.lrs.get("sh_rest", self.lrs["sh"])]
        gsmi.gs_adam_step_device([(L[n], L[n].grad, self.m6[n], self.v6[n], lr[i])
                                  for i, n in enumerate(self.GROUPS6)], self.step_dev,
                                 0.9, 0.999, 1e-15)
        for n in self.GROUPS6:
            L[n].grad = None
        frame = st["frame"]
        torch.maximum(lvl["pairs_max"], frame.n_pairs_dev, out=lvl["pairs_max"])
        self.lr_log.append(lr[0])
        return frame

    def means_lr_at(self, k: int) -> float:
        """Position learning rate at iteration k (supplementary, "Learning
        Rate"): the initial value up to the first iteration rendered at
        floor(r) = 1, then the backbone's exponential decay to the final value
        over the remaining iterations."""
        lr0, lr1 = self.means_lr
        if k <= self.k_full:
            return lr0
        t = (k - self.k_full) / max(1, self.iters - self.k_full)
        return math.exp((1.0 - t) * math.log(lr0) + t * math.log(lr1))

    def _densify(self, k: int):
        from .densify import densify_step
        c = self.dcfg
        # Eq. 4 takes the modulated factor floor(r^(i)), the one rendered at
        # iteration k (Sec. 5, "Implementation Details")
        r = float(self.factors[k])

        def k_of(kept, cand):
            if not c.schedule:
                return cand
            if c.momentum:
                self.p_fin = gsmi.gs_primitive_budget(self.p_fin, cand, c.gamma, c.eta)
            target = gsmi.gs_primitive_target(k, self.iters, r, self.p_init, self.p_fin)
            return int(round(target)) - kept

        self._check_capacity()
        if self.autograd:
            self._merge()
        n = self.params["means"].shape[0]
        z = torch.randn(n, 2, 3, generator=self.zgen, device=self.accum.device)
        newp, newm, newv, info = densify_step(self.params, self.m, self.v, self.accum, self.count,
                                              z, c.grad_thr, c.min_opacity,
                                              c.percent_dense * c.extent, k_of)
        if self.spatial:
            _, newp, newm, newv = raster.spatial_order(newp, newm, newv)
        for name in raster.PARAM_NAMES:
            self.params[name] = newp[name]
            self.m[name] = newm[name]
            self.v[name] = newv[name]
        info.update(iteration=k, r=r, p_fin=getattr(self, "p_fin", None))
        self.log.append(info)
        self._build_levels(k)
        if self.autograd:
            self._split()

    def run(self) -> dict:
        """Run all iterations; returns the wall time (and the part of it spent
        in densification steps, pipeline rebuilds included), the iterations
        per factor and the primitive count."""
        c = self.dcfg
        stop = (c.stop if c.stop is not None else self.iters // 2) if c else 0
        t_densify = 0.0
        if self.autograd:
            self._split()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(self.iters):
            if c is not None and c.start <= k < stop and k > 0 and (k - c.start) % c.every == 0:
                torch.cuda.synchronize()
                td = time.perf_counter()
                self._densify(k)
                torch.cuda.synchronize()
                t_densify += time.perf_counter() - td
            v = self.view_seq[k]
            f = int(self.factors[k])
            if self.graphs:
                self.graph_of[f].replay()
                self.lr_log.append(self._lrs6(k)[0])
                continue
            if self.autograd:
                views = self.levels[f][0]
                frame = self._autograd_step(k, f, v)
                n_now, proj = frame.n, frame.proj
            else:
                views, gt_f, pipe = self.levels[f]
                pipe.set_view(views[v], gt_f[v])
                pipe.lrs["means"] = self.means_lr_at(k)
                self.lr_log.append(pipe.lrs["means"])
                pipe.step()
                torch.maximum(pipe.pairs_max, pipe.n_pairs, out=pipe.pairs_max)
                n_now, proj = pipe.n, pipe.proj
            if c is not None and k < stop:
                gsmi.gs_densify_stats(1, n_now, proj, self.mean2d, self.accum, self.count,
                                      scale=0.5 * views[v].width)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if self.autograd:
            self._merge()
        self._check_capacity()
        if self.mip:
            self.update_filter3d()   # for rendering the trained model
        return dict(seconds=wall, s_per_iter=wall / max(1, self.iters),
                    iters_per_factor={int(f): int((self.factors == f).sum())
                                      for f in sorted(set(self.factors.tolist()))},
                    k_full=self.k_full, n_gaussians=int(self.params["means"].shape[0]),
                    densify_steps=len(self.log), densify_seconds=t_densify)
