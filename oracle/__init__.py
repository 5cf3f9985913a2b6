"""FP64 CPU oracle of the differentiable Gaussian-splat rasterizer.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the package smoke check and the
benchmark's CPU-baseline leg may import, call, link or execute anything in this
folder.  It shares no code with the GPU library and never imports it.

  oracle.oracle -- tiled forward, hand-derived backward (plain C, FP64)
  oracle.dense  -- dense per-pixel brute force with autograd (PyTorch CPU, FP64)
  oracle.update -- sparse Adam, pose step and Sim(3) relocation (numpy, FP64)
  oracle.hierarchy_cut -- level-of-detail cut of the Gaussian hierarchy
  oracle.ba     -- local bundle adjustment with a dense Schur complement (numpy, FP64)
"""
