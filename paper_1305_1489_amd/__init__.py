"""MI355X-native HDG hot path: HIP kernels for gfx950 behind a C ABI (include/hdg.h).

Submodules:
  _lib     ctypes binding of libhdg (same names as the C calls)
  driver   end-to-end orchestration of the stages over the binding
  build    in-tree build of libhdg.so with hipcc
"""
