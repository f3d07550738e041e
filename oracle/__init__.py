"""CPU FP64 oracle for matrix-free 3D SIMP compliance topology optimisation.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may import or run anything in this package.  The GPU library never
calls it, and it shares no code with the GPU library: the only module both sides read
is ``synth_inputs`` (seeded problem inputs, no method arithmetic).

Everything here is plain, slow and written to be checked against the paper by eye:
explicit element stiffness by Gauss quadrature, an explicitly assembled sparse global
stiffness, an explicit sparse filter matrix, and textbook solvers.  All floating point
is float64.

Modules
  fem      geometry, element stiffness, SIMP modulus, assembly, constrained operator
  solvers  direct solve, Jacobi-PCG, Lanczos extremes, iterative refinement
  topopt   compliance, sensitivities, density filter, OC bisection, SIMP loop
  nn       3D convolutions, the U-Net preconditioner, its loss/gradients, flexible CG

Parity status: every function is pinned by the ``-m "not gpu"`` tests in
``tests/test_oracle_*.py`` except where a function's docstring says "parity unpinned".
"""
