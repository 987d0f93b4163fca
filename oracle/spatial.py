"""The spatial storage order of the Gaussians: a Morton (Z-order) curve over
their means.  Test infrastructure only: imported by tests/, never by the
product path.

This is a storage order of the rasterizer's data, not part of the paper's
method: every image and gradient is the same for any order of the Gaussians,
up to the tie-break of exactly equal depths, which follows the stored index.
It is written out here, from its definition, so that the device's
permutation can be checked bit for bit.

Definition.  The decisions that produce integers are taken in float32, in
this order (the precision and order the device takes them in):
  lo_a = min_i m_ia and hi_a = max_i m_ia for each axis a (exact);
  s_a = 1024 / (hi_a - lo_a), both operations rounded to float32
        (s_a = 0 when hi_a = lo_a);
  q_ia = min(1023, max(0, floor((m_ia - lo_a) * s_a))), the subtraction and
        the product each rounded to float32;
  code_i interleaves the ten bits of q_ix, q_iy, q_iz: bit b of q_ix goes to
        bit 3b, of q_iy to bit 3b + 1, of q_iz to bit 3b + 2;
  the order is the stable ascending sort of code (equal codes keep ascending
  index): perm[k] is the index of the k-th Gaussian.
"""
from __future__ import annotations

import numpy as np

BITS = 10


def quantise(means) -> np.ndarray:
    """q [N,3] int64 cell coordinates of the means in their bounding box."""
    m = np.asarray(means, np.float32)
    if m.shape[0] == 0:
        return np.zeros((0, 3), np.int64)
    lo = m.min(axis=0)
    hi = m.max(axis=0)
    ext = (hi - lo).astype(np.float32)
    s = np.where(ext > 0, np.float32(1 << BITS) / np.where(ext > 0, ext, np.float32(1)),
                 np.float32(0)).astype(np.float32)
    d = (m - lo[None, :]).astype(np.float32)
    t = (d * s[None, :]).astype(np.float32)
    return np.clip(np.floor(t).astype(np.int64), 0, (1 << BITS) - 1)


def morton_codes(means) -> np.ndarray:
    """30-bit interleaved codes [N] (int64)."""
    q = quantise(means)
    code = np.zeros(q.shape[0], np.int64)
    for b in range(BITS):
        for a in range(3):
            code |= ((q[:, a] >> b) & 1) << (3 * b + a)
    return code


def morton_order(means) -> np.ndarray:
    """The permutation [N] (int64): Gaussians sorted by code, ties by index."""
    code = morton_codes(means)
    return np.argsort(code, kind="stable")
