"""(tile | depth) keys, their stable ascending sort and the per-tile ranges.

Plain definition, written out: for every Gaussian i with a non-empty tile
rectangle, in ascending i, and for every tile (tx, ty) of its rectangle in
row-major order, emit key = ((ty * grid_w + tx) << 32) | bits(z_f32_i) with
value i.  Sort the pairs by key, stably, so equal keys keep ascending i.
ranges[t] = [first, last + 1) of tile t in the sorted list, [0, 0) when the
tile received nothing.  For several views the view index sits above the tile
index: key = ((view_tile_base + tile) << 32) | bits(z), i.e. tiles of all views
are numbered consecutively view after view.
"""
from __future__ import annotations

import numpy as np


def depth_bits(z_f32: np.ndarray) -> np.ndarray:
    return np.asarray(z_f32, np.float32).view(np.uint32).astype(np.uint64)


def emit_pairs(rect: np.ndarray, tiles_touched: np.ndarray, z_f32: np.ndarray, grid_w: int,
               tile_base: int = 0):
    """Keys and values in emission order (Gaussian index ascending, tiles row-major)."""
    keys, vals = [], []
    zb = depth_bits(z_f32)
    for i in np.nonzero(np.asarray(tiles_touched) > 0)[0]:
        x0, y0, x1, y1 = (int(v) for v in rect[i])
        ty, tx = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
        t = (tile_base + ty * grid_w + tx).ravel().astype(np.uint64)
        keys.append((t << np.uint64(32)) | zb[i])
        vals.append(np.full(t.shape[0], i, np.uint32))
    if not keys:
        return np.zeros(0, np.uint64), np.zeros(0, np.uint32)
    return np.concatenate(keys), np.concatenate(vals)


def sort_pairs(keys: np.ndarray, vals: np.ndarray):
    """Stable ascending sort by key (equal keys keep emission order)."""
    o = np.argsort(keys, kind="stable")
    return keys[o], vals[o]


def tile_ranges(sorted_keys: np.ndarray, n_tiles: int) -> np.ndarray:
    """[n_tiles, 2] uint32 ranges by a linear scan of the sorted keys."""
    r = np.zeros((n_tiles, 2), np.uint32)
    t = (sorted_keys >> np.uint64(32)).astype(np.int64)
    for i in range(t.shape[0]):
        if i == 0 or t[i] != t[i - 1]:
            r[t[i], 0] = i
        if i == t.shape[0] - 1 or t[i] != t[i + 1]:
            r[t[i], 1] = i + 1
    return r


def bin_sort(rect, tiles_touched, z_f32, grid_w: int, grid_h: int):
    """Keys, values and ranges for one view."""
    k, v = emit_pairs(rect, tiles_touched, z_f32, grid_w)
    k, v = sort_pairs(k, v)
    return k, v, tile_ranges(k, grid_w * grid_h)


def bin_sort_views(rects, tiles_touched, z_f32s, grids):
    """Several views: tiles numbered consecutively view after view."""
    ks, vs = [], []
    base = 0
    for rect, tt, z, (gw, gh) in zip(rects, tiles_touched, z_f32s, grids):
        k, v = emit_pairs(rect, tt, z, gw, tile_base=base)
        ks.append(k)
        vs.append(v)
        base += gw * gh
    k = np.concatenate(ks) if ks else np.zeros(0, np.uint64)
    v = np.concatenate(vs) if vs else np.zeros(0, np.uint32)
    k, v = sort_pairs(k, v)
    return k, v, tile_ranges(k, base)
