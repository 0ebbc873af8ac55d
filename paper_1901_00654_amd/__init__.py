"""MI355X-native matrix-free multigrid-preconditioned spline smoothing.

Implements the hot path of arXiv:1901.00654 (tensor-product cubic B-spline
smoothing of scattered d-dimensional data, solved by a geometric-multigrid
preconditioned CG without assembling the matrix) as hand-written HIP
kernels for gfx950 behind the C ABI declared in include/tsmg.h.

Submodules:
- ``tsmg``       ctypes binding of the C ABI (same names as the header).
- ``build``      compiles the HIP library in-tree.
- ``workloads``  seeded synthetic inputs (no method arithmetic).

The binding is imported lazily so ``workloads`` stays importable without the
compiled library.
"""
