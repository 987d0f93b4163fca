"""Pins for the oracle's Adam step and L1 loss (CPU only).

Adam: the first step moves each element by exactly -lr g/(|g| + eps) (bias
corrections make m_hat = g and v_hat = g^2), and ten steps match
torch.optim.Adam run in float64 on the CPU (an independent implementation).
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
