"""MI355X-native differentiable 3D Gaussian splatting (the mapping hot path of LVI-GS, arXiv 2411.02703).

Submodules (imported on demand so that the input generator works without the HIP library):
  binding   - ctypes binding of libgs.so (the C ABI in include/libgs.h)
  rasterize - torch.autograd.Function around the rasteriser
  step      - plain per-view and batched graph-captured optimisation iterations
  scenes    - seeded synthetic inputs
  build     - builds libgs.so for gfx950
"""
__all__ = ["binding", "rasterize", "step", "scenes", "build"]
