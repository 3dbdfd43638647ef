"""MI355X-native parallel-tempering Metropolis for the 3D +-J Edwards-Anderson
model over bit-packed temperature replicas (arXiv:1311.5582).

The simulation runs in hand-written HIP kernels for gfx950 behind the C ABI
declared in include/ea.h; `paper_1311_5582_amd.binding` is the thin ctypes
layer over it.  Importing this package loads nothing: the shared library is
opened on first use of the binding and its absence is an error.
"""
__all__ = ["binding", "inputs"]
