"""MI355X-native micromagnetic hot path (arXiv 2411.18194 method).

``mmp``     ctypes binding of the HIP library libmmp.so (C ABI: include/mmp.h)
``inputs``  seeded synthetic problem generators
``build``   compiles the library in-tree for gfx950
"""
