"""FP64 CPU oracle of the CPR two-stage preconditioned FGMRES solve phase.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) imports, calls or links anything here; only the tests,
the package's smoke check and the benchmark's CPU-baseline leg do.  It shares no
code with the HIP path: the two meet only at the seeded input generator in
``workloads/``, which holds none of the method's arithmetic.

The oracle is plain and slow on purpose.  It follows Zhao, Feng, Zhang and Shu,
"Parallel Multi-Stage Preconditioners with Adaptive Setup for the Black Oil
Model" (arXiv 2201.01970): the CPR method (Section 3.1, eq. (CPR), Algorithm
"CPR method"), the adaptive-setup GMRES (Section 4, Algorithms "ASCPR-GMRES"
and "ASCPR"), and the multi-colour Gauss-Seidel built on the matrix of strong
connections (Section 5, eq. (strong-matrix), Algorithms "VerticesSplitting",
"VerticesGrouping", "PGS-SCM").  The paper leaves the pressure AMG's
coarsening to its UA-AMG library; here it is classical Ruge-Stueben
coarsening and interpolation written out from the textbook definition.

Every sum whose rounding matters is written with an explicit order (stored
column order, left to right); products and sums are separate operations.

Modules:
  sparse    CSR container and ordered row sums
  strength  RS strength and the paper's strong-connection matrix
  coloring  VerticesSplitting / VerticesGrouping
  rs        C/F splitting, interpolation, Galerkin product
  amg       hierarchy, multi-colour GS sweep, V-cycle, dense coarse solve
  cpr       pressure restriction/prolongation, block-GS stage 2, CPR apply
  fgmres    flexible GMRES(m)
  ascpr     the adaptive-setup rule and a Newton-sequence driver

Parity status: every function is pinned by tests under tests/ except the
iterate values of a whole solve, which the paper does not print ("parity
unpinned" for iterate values; they are pinned only through the properties
listed in the tests).
"""
