"""CPU oracle for the low-rank stochastic-Galerkin Navier-Stokes solver
(Elman & Su, "A low-rank solver for the stochastic unsteady Navier-Stokes
problem").

THIS PACKAGE IS TEST INFRASTRUCTURE.  It is a plain, slow, FP64 numpy/scipy
restatement of what the paper computes, written to check the GPU library.
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it.  The product path (``paper_1906_06785_amd``) never
imports, calls or links anything here, and this package imports nothing from
the product path.  Shared inputs come from ``synthetic_inputs`` only.

Modules:
  mesh     step-domain mesh, Q2-Q1 finite elements (sec. 3.2, eq. 3.7-3.8, sec. 6.1)
  gpc      Legendre chaos basis and the G_l, H_l matrices (eq. 3.9)
  system   all-at-once operator, right-hand side, direct reference solves
           (eq. 3.10-3.12, eq. 4.12, Alg. 3.1)
  tt       tensor-train algebra: TT-SVD, rounding, add, dot, Kronecker apply
           (sec. 4.1, eq. 4.1-4.7, Alg. 4.1)
  solver   mean-based LSC preconditioner, inner mean solve, low-rank flexible
           GMRES, refinement (Alg. 4.2, sec. 5, eq. 5.2, 5.19-5.23)

Parity status of each function is stated in its docstring; functions whose
result has no independent pin say "parity unpinned".
"""
