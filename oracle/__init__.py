"""FP64 CPU oracle for the space-time Fast Diagonalization solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product (the ``stfd`` C library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark use it.
It shares no code with the GPU path: it is written from the paper's
definitions in plain numpy/scipy, slowly and in the order the paper states
things, so that it can be checked against the paper by eye.

Modules
  time_matrices   A_t, M_t, C_t of the modified Hilbert transformation H_T
                  (Sec. 2, definitions after the global system (2.x)), two
                  routes: the truncated eigen-series with exact per-mode
                  coefficients, and the exactly summed series (log-tan kernel)
                  integrated element pair by element pair.
  space_matrices  P1 mass, stiffness and M^{1,0} matrices (Sec. 2).
  load            piecewise-constant projection Q_h^0 f and the assembled load
                  F~ = M^{1,0} F C_t^T (Sec. 2).
  solvers         the full Kronecker system K_h (Sec. 2, 3.1), the Fast
                  Diagonalization algorithm (Sec. 4.4, Algorithm FD), the
                  Bartels-Stewart algorithm with the complex Schur form
                  (Sec. 4.3, Algorithm BSc) and FP64 iterative refinement on
                  the K_h residual.
  errors          space-time L2(Q) and H1(Q) errors of a discrete solution.
  lshape          the L-shape example of Sec. 5: its manufactured solution and
                  source, the homogenisation of its Dirichlet data, and one
                  table row (dof, mesh sizes, errors) per refinement level.

Parity status of each function is stated in its docstring; every function is
pinned by a test in ``tests/test_oracle_*.py`` against something other than
itself (printed paper values, closed forms, brute force, library routines).
"""
