"""ORACLE -- test infrastructure only.

A plain, slow, float64 CPU implementation of what the GPU path computes: the
dense Gaussian kernel and its alpha = 1 diffusion-maps normalisation (Eq. (2),
Alg. 1), the hierarchical approximation K~ = D + S + UV (Eq. (3)) built by the
same compression algorithm as the GPU library, its matrix-vector product, and
the float64 Lanczos eigensolver (Sec. 2.2).

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import
this package.  It shares no code with the HIP library and imports nothing from it.
"""
