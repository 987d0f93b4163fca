"""Pins of the spatial storage order (oracle/spatial.py): the codes against a
bit-by-bit brute force, the order against Python's sorted() over (code,
index), its locality, and the degenerate inputs."""
import numpy as np

from oracle import spatial


def _brute_code(q):
    c = 0
    for b in range(10):
        for a in range(3):
            c |= ((int(q[a]) >> b) & 1) << (3 * b + a)
    return c


def test_codes_and_order_against_brute_force():
    rng = np.random.default_rng(0)
    m = rng.uniform(-4, 4, size=(300, 3)).astype(np.float32)
    m[50:60] = m[0]                       # equal means: equal codes, ties by index
    q = spatial.quantise(m)
    # the quantisation by its definition, one Gaussian at a time in float32
    f = np.float32
    lo, hi = m.min(0), m.max(0)
    for i in range(0, 300, 7):
        for a in range(3):
            s = f(f(1024) / f(hi[a] - lo[a]))
            t = f(f(m[i, a] - lo[a]) * s)
            assert q[i, a] == min(1023, max(0, int(np.floor(t))))
    codes = spatial.morton_codes(m)
    assert [int(c) for c in codes] == [_brute_code(qi) for qi in q]
    perm = spatial.morton_order(m)
    assert list(perm) == sorted(range(300), key=lambda i: (int(codes[i]), i))
    assert list(perm[np.isin(perm, np.arange(50, 60)) | (perm == 0)]) == [0] + list(range(50, 60))


def test_order_is_local():
    rng = np.random.default_rng(1)
    m = rng.uniform(-4, 4, size=(20000, 3)).astype(np.float32)
    perm = spatial.morton_order(m)
    step_sorted = np.linalg.norm(np.diff(m[perm], axis=0), axis=1).mean()
    step_random = np.linalg.norm(np.diff(m, axis=0), axis=1).mean()
    assert step_sorted < 0.1 * step_random
    assert np.array_equal(np.sort(perm), np.arange(20000))


def test_degenerate_inputs():
    assert spatial.morton_order(np.zeros((0, 3), np.float32)).shape == (0,)
    assert list(spatial.morton_order(np.ones((5, 3), np.float32))) == [0, 1, 2, 3, 4]
    # one axis flat: its cells are all 0, the others still order the points
    m = np.stack([np.arange(8, dtype=np.float32)[::-1], np.zeros(8, np.float32),
                  np.zeros(8, np.float32)], 1)
    assert list(spatial.morton_order(m)) == list(range(7, -1, -1))
    # the box's far corner lands in the last cell, not past it
    q = spatial.quantise(np.array([[0, 0, 0], [1, 2, 3]], np.float32))
    assert q.tolist() == [[0, 0, 0], [1023, 1023, 1023]]
