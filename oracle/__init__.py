"""CPU oracle for polyharmonic-spline (PHS) interpolation — TEST INFRASTRUCTURE.

This package is the plain, slow, FP64 statement of what the accelerated path
computes: dense kernel matrices, a direct factorisation on the complement of the
polynomial space, the Vecchia/Matern inverse-Cholesky factor built point by
point, and a projected PCG used only to predict iteration counts.

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import it.  It shares no code with the HIP library and never imports the
product package; the two meet only through the seeded input generators.

Modules
-------
phs_dense   definition of the interpolation problem and its direct solution
vecchia     ordering, ordered nearest neighbours, Matern kernel, sparse factor
pcg         projected preconditioned CG (reference iteration counts)

Readings of passages where the paper is silent or garbled are listed in the
docstring of each function that takes them.  Functions without an independent
pin say "parity unpinned" in their docstring.
"""
