"""One densification step of the resolution-guided primitive schedule
(Sec. 4.3, Eq. 4-5; supplementary "Densification of DashGaussian"): the four
C calls with the two device counts read in between and the new arrays
allocated here.  Marshalling only; the arithmetic runs in the library."""
from __future__ import annotations

import torch

from . import gsmi
from .raster import PARAM_NAMES


def densify_step(params: dict, m: dict, v: dict, accum: torch.Tensor, count: torch.Tensor,
                 z: torch.Tensor, grad_thr: float, min_opacity: float, max_scale: float,
                 k_of, stream=None):
    """k_of(n_kept, n_candidates) -> k, the number of candidates to densify.
    Returns (params, m, v, info) with new tensors (the inputs are untouched)."""
    n = params["means"].shape[0]
    dev = params["means"].device
    ws = torch.empty(max(gsmi.gs_densify_workspace_bytes(n), 16), dtype=torch.uint8, device=dev)
    counts = torch.zeros(2, dtype=torch.int64, device=dev)
    gsmi.gs_densify_classify(n, accum, count, params["opacity_logits"], grad_thr, min_opacity,
                             ws, counts, stream)
    n_pruned, n_cand = (int(x) for x in counts.cpu())
    k = int(max(0, min(int(k_of(n - n_pruned, n_cand)), n_cand)))
    n_new_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    gsmi.gs_densify_plan(n, k, n_cand, params["log_scales"], max_scale, ws, n_new_dev, stream)
    n_new = int(n_new_dev.item())
    newp = {name: torch.empty((n_new,) + tuple(params[name].shape[1:]), dtype=torch.float32,
                              device=dev) for name in PARAM_NAMES}
    newm = {name: torch.empty_like(newp[name]) for name in PARAM_NAMES}
    newv = {name: torch.empty_like(newp[name]) for name in PARAM_NAMES}
    info = dict(n=n, n_pruned=n_pruned, n_candidates=n_cand, k=k, n_new=n_new)
    if n_new == 0:  # everything pruned (or nothing given): no rows to write
        return newp, newm, newv, info
    gsmi.gs_densify_apply(n, [params[k_] for k_ in PARAM_NAMES], [m[k_] for k_ in PARAM_NAMES],
                          [v[k_] for k_ in PARAM_NAMES], z, ws,
                          [newp[k_] for k_ in PARAM_NAMES], [newm[k_] for k_ in PARAM_NAMES],
                          [newv[k_] for k_ in PARAM_NAMES], stream)
    return newp, newm, newv, info
