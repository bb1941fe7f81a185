"""MI355X-native nodal discontinuous Galerkin core for the 3-D compressible
Euler equations on periodic Cartesian hexahedral meshes (Kirby & Mavriplis,
"GPU-Accelerated Discontinuous Galerkin Methods": the explicit DG
right-hand side of Section II and the five-stage low-storage Runge-Kutta
stage update of Sections IV-V).

    paper_2006_15698_amd.dg      ctypes binding of libdg.so (same names as
                                 include/dg.h) plus the Solver convenience
                                 class and the autograd RHS
    paper_2006_15698_amd.build   builds libdg.so in-tree with hipcc (gfx950)

Every step of the hot path runs in the HIP kernels of libdg.so; PyTorch only
provides device memory and the stream.  Importing ``dg`` raises ImportError if
libdg.so has not been built.
"""
