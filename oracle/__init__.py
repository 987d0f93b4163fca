"""FP64 CPU oracle for the tile-based differentiable Gaussian rasterizer.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.

It is a plain, slow, obviously-correct restatement of what the rasterizer
computes, written from the paper's definition of splat-and-blend rendering
(Sec. 3, Eq. 1: C(u) = sum_i T_i w_i c_i with T_i = prod_{j<i}(1 - w_j) and
w_i = o_i G2D_i(u)) and from the conventions the rasterizer fixes where the
paper is silent (EWA projection, SH colour, 1/255 cutoff, 0.99 clamp, T<1e-4
exit).  Every floating-point step runs in float64 on the float32 inputs,
except the one value that is defined in float32 on purpose: the depth whose
bits form the sort key (``project.depth_f32``).

Modules
-------
sh       real spherical-harmonic basis up to degree 3 and its derivative
project  per-Gaussian EWA projection, colour, culling, tile rectangles
render   per-pixel brute-force forward blend and its analytic backward
binning  (tile|depth) keys, stable sort and tile ranges by definition
adam     the Adam update by definition
loss     L1 loss and its gradient

Parity pins for every function live in ``tests/test_oracle_*.py``.
"""
