"""Lattice Landau-de Gennes force and FIRE relaxation on MI355X (gfx950).

The compute lives in liblqfire.so (HIP kernels behind the C ABI of
include/lqfire.h); lqfire.py is its ctypes binding, synth.py draws seeded
synthetic inputs, build.py compiles the library, serve.py runs many small
minimizations at once.
"""
