"""Reference oracle: a plain, slow FP64 CPU implementation of the solver path.

This package is TEST INFRASTRUCTURE. Only the test-suite, the smoke check and
the benchmark's CPU-baseline leg may import it. The GPU library shares no code,
tables or constants with it; both sides are written independently from the
paper (Phillips & Fischer, "Optimal Chebyshev Smoothers and One-sided
V-cycles") and from the standard spectral-element definitions.

Modules
  gll        GLL nodes, weights, derivative and interpolation matrices
  sem        spectral-element Poisson operator on (deformed) hexahedral boxes
  chebyshev  Chebyshev smoothers of the 1st kind (Alg. 1) and 4th / opt. 4th
             kind (Alg. 2), with the beta table of the supplementary material
  mg         multigrid V-cycles, symmetric and one-sided (Sec. 2, eqs.
             recursive-v-cycle-err-prop / recursive-ftc-err)
  krylov     preconditioned and flexible conjugate gradients
  fd2d       2D finite-difference Poisson with Galerkin geometric multigrid (Sec. 3)
  analysis   gamma^{-1}, approximation constants, critical C (Sec. 2, Lemma 2.1)
  adjoint    gradients of ||u - u_t||^2 with respect to the load and the
             geometric factors
  lanczos    largest eigenvalue of S A

Parity status: every function is pinned by tests against closed forms,
brute-force constructions or values printed in the paper, except the batched
and mixed-precision paths, which exist only on the GPU side and are checked
against this FP64 oracle (parity unpinned against the paper, which has no such
runs).
"""
