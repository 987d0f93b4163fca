"""The Adam update by definition (the "primitive update" after each rendering
and back-propagation, Sec. 1 and Sec. 5.2; the backbones use Adam).

    m <- b1 m + (1 - b1) g
    v <- b2 v + (1 - b2) g^2
    p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)

elementwise, FP64, t the 1-based step.
"""
from __future__ import annotations

import numpy as np


def adam_step(p, g, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-15):
    p = np.asarray(p, np.float64).copy()
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p -= lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def sparse_adam_step(p, g, m, v, rows, step: int, lr: float, beta1: float = 0.9,
                     beta2: float = 0.999, eps: float = 1e-15):
    """Sparse (lazy) Adam, the optimiser of the Taming backbone: the rows
    (first axis) where ``rows`` is true take the Adam update above with the
    global step t; the other rows keep p, m and v unchanged."""
    rows = np.asarray(rows, bool)
    p1, m1, v1 = adam_step(p, g, m, v, step, lr, beta1, beta2, eps)
    keep = ~rows
    p1[keep] = np.asarray(p, np.float64)[keep]
    m1[keep] = np.asarray(m, np.float64)[keep]
    v1[keep] = np.asarray(v, np.float64)[keep]
    return p1, m1, v1
