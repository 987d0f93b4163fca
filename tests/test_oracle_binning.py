"""Pins for the oracle's keys / sort / ranges (CPU only): Python's built-in
``sorted`` over explicitly enumerated (key, value) tuples, and ranges found by
brute force over all tiles."""
import numpy as np

from oracle import binning, project
from paper_2503_18402_amd import scenes


def _brute(rects, tt, z, gw, gh):
    pairs = []
    for i in range(len(tt)):
        if tt[i] <= 0:
            continue
        x0, y0, x1, y1 = rects[i]
        for ty in range(y0, y1 + 1):
            for tx in range(x0, x1 + 1):
                key = ((ty * gw + tx) << 32) | int(np.float32(z[i]).view(np.uint32))
                pairs.append((key, i))
    pairs = sorted(pairs, key=lambda kv: (kv[0], kv[1]))
    ranges = []
    for t in range(gw * gh):
        idx = [j for j, (k, _) in enumerate(pairs) if (k >> 32) == t]
        ranges.append((idx[0], idx[-1] + 1) if idx else (0, 0))
    return pairs, ranges


def test_random_rects_match_sorted():
    rng = np.random.default_rng(0)
    gw, gh, n = 7, 5, 60
    x0 = rng.integers(0, gw, n); x1 = np.minimum(gw - 1, x0 + rng.integers(0, 3, n))
    y0 = rng.integers(0, gh, n); y1 = np.minimum(gh - 1, y0 + rng.integers(0, 3, n))
    rects = np.stack([x0, y0, x1, y1], 1)
    tt = (x1 - x0 + 1) * (y1 - y0 + 1)
    tt[rng.random(n) < 0.2] = 0
    z = rng.uniform(0.5, 4.0, n).astype(np.float32)
    z[5] = z[9] = z[20]           # ties resolve by index
    k, v, r = binning.bin_sort(rects, tt, z, gw, gh)
    pairs, ranges = _brute(rects, tt, z, gw, gh)
    assert [int(x) for x in k] == [p[0] for p in pairs]
    assert [int(x) for x in v] == [p[1] for p in pairs]
    assert [tuple(int(a) for a in row) for row in r] == ranges


def test_small_scene_projection_pairs():
    sc, cam = scenes.small_scene()
    sc = scenes.subset(sc, slice(0, 400))
    P = project.project(sc, cam, tile=16)
    gw, gh = (cam.width + 15) // 16, (cam.height + 15) // 16
    k, v, r = binning.bin_sort(P["rect"], P["tiles_touched"], P["depth_f32"], gw, gh)
    pairs, ranges = _brute(P["rect"], P["tiles_touched"], P["depth_f32"], gw, gh)
    assert len(pairs) == int(P["tiles_touched"].sum()) == k.shape[0]
    assert [int(x) for x in v] == [p[1] for p in pairs]
    assert [tuple(int(a) for a in row) for row in r] == ranges


def test_views_stack_tiles():
    rng = np.random.default_rng(1)
    rects = [np.array([[0, 0, 1, 0], [1, 1, 1, 1]]), np.array([[0, 0, 0, 0]])]
    tts = [np.array([2, 1]), np.array([1])]
    zs = [np.array([2.0, 1.0], np.float32), np.array([3.0], np.float32)]
    k, v, r = binning.bin_sort_views(rects, tts, zs, [(2, 2), (1, 1)])
    tiles = [int(x >> np.uint64(32)) for x in k]
    assert tiles == [0, 1, 3, 4]
    assert [int(x) for x in v] == [0, 0, 1, 0]
    assert r.shape == (5, 2) and tuple(r[2]) == (0, 0) and tuple(r[4]) == (3, 4)


def test_empty():
    k, v, r = binning.bin_sort(np.zeros((0, 4), int), np.zeros(0, int), np.zeros(0, np.float32), 3, 2)
    assert k.shape == (0,) and v.shape == (0,) and not r.any()
