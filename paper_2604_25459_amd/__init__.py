"""MI355X-native batched 3D Gaussian Splatting for rigid-body simulation
environments (the batch renderer of GS-Playground, arXiv 2604.25459).

Submodules:
  synth  -- seeded synthetic scenes, cameras, poses and serving traces
  gsr    -- ctypes binding of libgsr.so (HIP kernels + C ABI in csrc/)
  build  -- compiles libgsr.so for gfx950
"""
