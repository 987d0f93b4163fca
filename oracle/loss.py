"""L1 photometric loss and its gradient (the loss the backbones train with).

L = mean |C - target| over the 3HW image values; dL/dC = sign(C - target)/(3HW)
with sign(0) = 0.
"""
from __future__ import annotations

import numpy as np


def l1(C, target):
    d = np.asarray(C, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(np.abs(d))), np.sign(d) / d.size
