"""FP64 CPU oracle of the differentiable Gaussian-splat rasterizer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg may import, call, link or execute anything in this
folder.  It shares no code with the GPU library and never imports it.

  oracle.oracle -- tiled forward, hand-derived backward (plain C, FP64)
  oracle.dense  -- dense per-pixel brute force with autograd (PyTorch CPU, FP64)
"""
