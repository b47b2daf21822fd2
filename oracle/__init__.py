"""CPU oracle for the deflated Hutchinson / hierarchical-probing trace estimator.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library or its Python binding
imports, calls or links anything in this directory; only the test suite, the
smoke check and the CPU-baseline leg of the benchmark use it.

Contents (each function cites the passage of Gambhir, Stathopoulos & Orginos,
"Deflation as a Method of Variance Reduction for Estimating the Trace of a
Matrix Inverse", arXiv:1603.05988, that it follows):

- ``lattice``   dense Wilson-Dirac matrix on small lattices (complex128).
- ``rng``       SplitMix64 counter generator, Z4 noise indices, hierarchical
                probing colours and Hadamard signs.
- ``estimator`` Hutchinson quadratic forms, deflation (T_D, z^H P z), sample
                and exact variances (Section 1 eq. variance, Section 5.2,
                Algorithm 1).
- ``theory``    Theorem 1 (Delta matrix), the Section 2 3x3 example, the free
                Wilson spectrum used in Section 6.
- ``stencil``   an independent plain-C FP64 Wilson stencil with BiCGStab, for
                lattices too large for dense algebra and for CPU timing.

All arithmetic is FP64 (the paper fixes no precision).
"""
