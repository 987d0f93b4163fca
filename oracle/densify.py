"""Oracle of the resolution-guided primitive schedule (Sec. 4.3, Eq. 4 and
Eq. 5; supplementary Eq. 8 and "Densification of DashGaussian").

Test infrastructure only: imported by tests/ (and bench.py's CPU baseline),
never by the product path.  FP64 arithmetic; the decisions that pick
integers (prune, candidacy, ranking, split vs clone) are taken in float32,
the precision the device takes them in.

Readings (the paper leaves these open):
* Densification score: the backbone's, the mean over the iterations where the
  Gaussian was seen of the norm of its 2D-mean gradient (accumulated sum /
  count), compared with a threshold.
* Prune: opacity below min_opacity (the backbone's opacity prune).
* P_add of Eq. 5 at a densification step is the number of unpruned Gaussians
  meeting the score threshold (those the backbone would densify).
* Selection: the k = clamp(P_i - N', 0, P_add) candidates of highest score,
  ties broken by ascending index.
* Clone if the largest scale is at most max_scale (the backbone's
  percent_dense * scene extent), else split into two children at
  mu + R(q) diag(s) z_j (z_j ~ N(0, I), given as input), scales s / 1.6,
  other parameters copied; the parent is removed.
* Output layout: Gaussians in index order; a pruned one writes nothing, a kept
  one itself, a cloned one itself then its copy, a split one its two
  children.  Adam moments are copied for kept and cloned originals and start
  at zero for copies and children.
"""
from __future__ import annotations

import numpy as np

from . import project

SPLIT_SCALE = 1.6   # the backbone's split shrink: s / (0.8 * 2)


def primitive_target(i: float, S: float, r: float, p_init: float, p_fin: float) -> float:
    """Eq. 4: P_i = P_init + (P_fin - P_init) / r^(2 - i/S)."""
    return p_init + (p_fin - p_init) / r ** (2.0 - i / S)


def budget_update(p_fin_prev: float, p_add: float, gamma: float = 0.98, eta: float = 1.0) -> float:
    """Eq. 5: P_fin <- max(P_fin, gamma P_fin + eta P_add)."""
    return max(p_fin_prev, gamma * p_fin_prev + eta * p_add)


def classify(accum, count, opacity_logits, grad_thr: float, min_opacity: float):
    """Scores (float32), prune and candidate masks."""
    accum = np.asarray(accum, np.float32)
    count = np.asarray(count, np.float32)
    score = np.where(count > 0, accum / np.maximum(count, np.float32(1)), np.float32(0))
    score = score.astype(np.float32)
    op = (1.0 / (1.0 + np.exp(-np.asarray(opacity_logits, np.float64)))).astype(np.float32)
    prune = op < np.float32(min_opacity)
    cand = (~prune) & (count > 0) & (score >= np.float32(grad_thr))
    return score, prune, cand


def select_top(score, cand, k: int) -> np.ndarray:
    """Mask of the k candidates of highest score (ties: ascending index)."""
    idx = np.nonzero(cand)[0]
    order = idx[np.lexsort((idx, -score[idx].astype(np.float64)))]
    sel = np.zeros(cand.shape, bool)
    sel[order[:max(0, min(k, idx.size))]] = True
    return sel


def densify(params: dict, moments: dict, accum, count, z, grad_thr: float, min_opacity: float,
            max_scale: float, k: int):
    """One densification step.  params / moments: dicts of arrays (moments
    maps 'm_<name>' / 'v_<name>'); z: [N, 2, 3] standard normal samples.
    Returns (new params, new moments, info)."""
    n = params["means"].shape[0]
    score, prune, cand = classify(accum, count, params["opacity_logits"], grad_thr, min_opacity)
    sel = select_top(score, cand, k)
    s32 = np.exp(params["log_scales"].astype(np.float32)).astype(np.float32)
    split = sel & (s32.max(axis=1) > np.float32(max_scale))
    clone = sel & ~split
    s = np.exp(params["log_scales"].astype(np.float64))
    q = params["quats"].astype(np.float64)
    R = project.quat_to_rot(q / np.linalg.norm(q, axis=1, keepdims=True))   # [N, 3, 3]
    out = {k_: [] for k_ in params}
    mom = {k_: [] for k_ in moments}
    zero = {k_: np.zeros_like(v[0]) for k_, v in moments.items()}
    for g in range(n):
        if prune[g]:
            continue
        if split[g]:
            for j in range(2):
                for name, arr in params.items():
                    if name == "means":
                        out[name].append(arr[g] + R[g] @ (s[g] * z[g, j]))
                    elif name == "log_scales":
                        out[name].append(arr[g] - np.log(SPLIT_SCALE))
                    else:
                        out[name].append(arr[g])
                for name in moments:
                    mom[name].append(zero[name])
            continue
        for name, arr in params.items():
            out[name].append(arr[g])
        for name, arr in moments.items():
            mom[name].append(arr[g])
        if clone[g]:
            for name, arr in params.items():
                out[name].append(arr[g])
            for name in moments:
                mom[name].append(zero[name])
    new = {name: np.array(v, dtype=np.float64).reshape((-1,) + params[name].shape[1:])
           for name, v in out.items()}
    newm = {name: np.array(v, dtype=np.float64).reshape((-1,) + moments[name].shape[1:])
            for name, v in mom.items()}
    info = dict(n_pruned=int(prune.sum()), n_kept=int(n - prune.sum()), p_add=int(cand.sum()),
                n_selected=int(sel.sum()), n_split=int(split.sum()), n_clone=int(clone.sum()),
                n_new=int(new["means"].shape[0]))
    return new, newm, info
