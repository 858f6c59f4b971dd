"""Plain FP64 CPU oracle for extrapolated geometric multigrid on B-spline (IGA)
discretisations of the Poisson problem.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import, call, link or run anything in this
package.  It shares no code with the GPU library: it has its own B-spline
evaluation (Cox-de Boor recursion), its own quadrature assembly (element
scatter), its own prolongation (collocation at Greville points instead of knot
insertion), sparse Galerkin products, CSR smoothers and Householder-QR
extrapolation.

Every function cites the passage of the paper (arXiv 2412.20205, "Vector
extrapolation methods applied to geometric multigrid solvers for isogeometric
analysis") that it follows.  Functions whose result no independent pin checks
say "parity unpinned" in their docstring.
"""
