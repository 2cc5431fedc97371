"""MI355X-native tile-based 3D Gaussian Splatting renderer (HIP, gfx950).

Submodules:
  scenes  seeded synthetic inputs (no renderer arithmetic)
  gs      ctypes binding of the C ABI in include/gs.h (libgs.so)
  build   builds libgs.so with hipcc
"""
