"""Plain FP64 CPU oracle for the nodal IP-DG right-hand side (test infrastructure).

This package is a slow, obviously-correct NumPy restatement of the method of
Zafeiris, Georgoulis & Papadakis, "Parallel nodal interior-penalty
discontinuous Galerkin methods for the subsonic compressible Navier-Stokes
equations" (arXiv 2508.17917).  It exists only to check the HIP path: the
tests, the smoke check and the CPU-baseline leg of the benchmark may import
it; the product path (the C-ABI library and its Python binding) never does,
and the two share no code.

Layout: every nodal field is an array of shape (4, Np, K) -- conserved
variable, node, element -- which is deliberately not the device layout.

Functions whose result no independent pin fixes say "parity unpinned" in
their docstring.  Everything else is pinned by the CPU tests in
``tests/test_oracle_*.py`` against closed forms, invariants, library
routines or brute force.
"""
