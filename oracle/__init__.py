"""CPU oracle for the multilevel deflation (MADP) preconditioned FGMRES solver.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plainly written FP64
(complex128) reference that the GPU library is checked against.  Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark may import it;
the product path (the C-ABI library and its Python binding) never does.  It
shares no code with the GPU path: operators are assembled as SciPy CSR matrices
row by row from the discretisation rules, and every solver step follows the
order of the paper's Algorithm 1.

Modules
  stencils   exact-rational Galerkin recursion for the coarse-level stencils
             (Sec. 3.3, the 7x7 stencils of the third level and Appendix A)
  operators  CSR assembly: 5-point Helmholtz/CSLP with Sommerfeld ghost points
             (Sec. 2.1), re-discretised 5x5/7x7 coarse operators with the
             boundary rule of Sec. 3.3, deflation vectors Z, multigrid transfers
  krylov     GMRES / FGMRES with modified Gram-Schmidt (Algorithm 1)
  multigrid  V-cycle approximation of the CSLP inverse (Sec. 3.2, 4.4)
  madp       the MADP hierarchy, preconditioner application and outer solve

Parity status of every function is recorded in its docstring; functions that
no pin other than the GPU comparison checks say "parity unpinned".
"""
