"""MI355X-native (gfx950) hot path of TideGS out-of-core 3DGS training.

Submodules:
  synth     seeded synthetic scenes, cameras and trajectories
  _lib      ctypes binding of libtide.so (the C ABI in include/tide.h)
  raster    torch-facing driver: rasterizer forward/backward, loss, Adam
  build     builds libtide.so with hipcc for gfx950
"""
__all__ = ["synth", "raster", "build"]
