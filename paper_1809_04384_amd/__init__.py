"""MI355X-native DH^2 compression of the Helmholtz single-layer Galerkin matrix.

The compute path lives in the native library libdh2.so (HIP kernels for
gfx950 + host C++, C ABI in include/dh2.h); paper_1809_04384_amd.dh2 is a
thin ctypes binding with the same entry points.
"""
