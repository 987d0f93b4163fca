"""Pins for the oracle's Adam step and L1 loss (CPU only).

Adam: the first step moves each element by exactly -lr g/(|g| + eps) (bias
corrections make m_hat = g and v_hat = g^2), and ten steps match
torch.optim.Adam run in float64 on the CPU (an independent implementation).
Sparse Adam: rows outside the mask are untouched, and eight steps over
changing row sets match torch.optim.SparseAdam (the library's lazy Adam) with
eps negligible (it adds eps before the bias correction of v).
L1: central differences of the loss value.
"""
import numpy as np
import torch

from oracle import adam, loss


def test_first_step_closed_form():
    rng = np.random.default_rng(0)
    p = rng.normal(size=100)
    g = rng.normal(size=100)
    lr, eps = 1e-2, 1e-8
    p1, m, v = adam.adam_step(p, g, np.zeros(100), np.zeros(100), 1, lr, eps=eps)
    assert np.abs(p1 - (p - lr * g / (np.abs(g) + eps))).max() < 1e-15


def test_matches_torch_adam():
    rng = np.random.default_rng(1)
    p0 = rng.normal(size=(40,))
    grads = rng.normal(size=(10, 40))
    lr, b1, b2, eps = 3e-3, 0.9, 0.999, 1e-15
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros(40), np.zeros(40)
    for k in range(10):
        t.grad = torch.tensor(grads[k], dtype=torch.float64)
        opt.step()
        p, m, v = adam.adam_step(p, grads[k], m, v, k + 1, lr, b1, b2, eps)
    assert np.abs(p - t.detach().numpy()).max() < 1e-14


def test_sparse_adam_matches_torch_sparse_adam():
    rng = np.random.default_rng(5)
    n, w = 30, 4
    p0 = rng.normal(size=(n, w))
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-30
    t = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.SparseAdam([t], lr=lr, betas=(b1, b2), eps=eps)
    p, m, v = p0.copy(), np.zeros((n, w)), np.zeros((n, w))
    for k in range(8):
        rows = rng.uniform(size=n) < 0.6
        rows[k] = True                      # a row seen every step ...
        rows[n - 1] = False                 # ... and one never seen
        g = rng.normal(size=(n, w)) * rows[:, None]
        g[np.nonzero(rows)[0][0]] = 0.0     # a visible row whose gradient is zero
        idx = torch.tensor(np.nonzero(rows)[0])
        t.grad = torch.sparse_coo_tensor(idx[None], torch.tensor(g[rows]), (n, w)).coalesce()
        opt.step()
        prev = p.copy()
        p, m, v = adam.sparse_adam_step(p, g, m, v, rows, k + 1, lr, b1, b2, eps)
        assert np.array_equal(p[~rows], prev[~rows])
    assert np.abs(p - t.detach().numpy()).max() < 1e-13
    assert np.array_equal(p[n - 1], p0[n - 1])


def test_sparse_adam_with_every_row_is_adam():
    rng = np.random.default_rng(6)
    p, g, m, v = (rng.normal(size=(7, 3)) for _ in range(4))
    v = np.abs(v)
    a = adam.adam_step(p, g, m, v, 3, 1e-2)
    b = adam.sparse_adam_step(p, g, m, v, np.ones(7, bool), 3, 1e-2)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_l1_grad_fd():
    rng = np.random.default_rng(2)
    C = rng.uniform(size=(3, 5, 4))
    tg = rng.uniform(size=(3, 5, 4))
    val, g = loss.l1(C, tg)
    h = 1e-7
    for idx in [(0, 0, 0), (1, 2, 3), (2, 4, 1)]:
        e = np.zeros_like(C)
        e[idx] = h
        fd = (loss.l1(C + e, tg)[0] - loss.l1(C - e, tg)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-8
    assert abs(val - np.abs(C - tg).mean()) < 1e-15
