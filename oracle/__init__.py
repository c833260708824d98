"""Plain FP64 CPU oracle for the HDG hot path (TEST INFRASTRUCTURE ONLY).

This package is the correctness reference for the HIP library: a slow,
straightforward NumPy/SciPy implementation of what the paper (Fu, Gatica,
Sayas, "Matlab tools for HDG in three dimensions") computes, in float64
throughout.  Only the test-suite, the package smoke check and the benchmark's
CPU-baseline leg may import it; the library never does, and the two share no
code (inputs come from :mod:`hdg_inputs`, which holds no method arithmetic).

Modules
  quadrature  Stroud conical-product rules on the reference tetrahedron and
              triangle (eq 3.1, the face rule of Section 4)
  poly        dense multivariate polynomials (exact values and gradients)
  basis       orthonormal hierarchical Dubiner bases (eq 3.3; Section 4,
              "Bases, faces, and boundaries")
  mesh        expansion of the basic mesh (Section 2, "Data structure")
  local       per-element blocks (Sections 3-4), local solver and static
              condensation (eq 5.1-5.6)
  globalsys   assembly (eq 6.5), boundary data (eq 6.3, 6.4), Dirichlet
              elimination, global solve, reconstruction (Section 6),
              postprocessing (eq 9.11) and errors (eq 10.1-10.2)
  brute       the uncondensed system eq 1.2a-e solved directly
  convection  HDG for convection-diffusion (eq 9.1 matrices; the conservative method with the
              numerical total flux), non-symmetric local solves and trace system
  bdm         hybridized BDM: the HDG local matrices with tau = 0 and the degree-k modes of
              u deleted (Section 9, "BDM"), condensed and uncondensed
  projection  the L2 projection onto M_h (eq 9.12), the HDG projection (eq 9.13) and the
              superconvergence diagnostics eps_u, eps_uhat (eq 10.2)
"""
