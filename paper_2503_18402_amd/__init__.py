"""MI355X (gfx950) differentiable tile-based Gaussian rasterizer.

The per-iteration hot path of 3DGS optimisation (render, back-propagate,
Adam) that DashGaussian's resolution and primitive schedules make cheaper,
as hand-written HIP kernels behind the C ABI in ``include/gs.h``.

Modules: ``gsmi`` (ctypes binding of the C ABI), ``raster`` (buffers,
batched multi-view rendering, autograd), ``scenes`` (seeded synthetic
inputs), ``build`` (hipcc build of ``libgsmi.so``).
"""
__all__ = ["gsmi", "raster", "scenes", "build"]
