"""CPU FP64 oracle for tensor-product B-spline smoothing (arXiv:1901.00654).

TEST INFRASTRUCTURE ONLY. This package exists to check the GPU library
against a plain, slow, independently written implementation of what the
paper computes. Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it. The product path never imports, calls
or links anything here, and nothing here imports the product package.

What is here, each module citing the passage it follows:

- ``bspline``  univariate B-splines on uniform extended knots by the
               Cox-de Boor recursion, and their derivatives (Sec. 2.1).
- ``system``   Phi, the 1D Gram matrices Psi^p_r, Lambda, A = Phi'Phi +
               lambda*Lambda and b = Phi'y, assembled as scipy.sparse
               matrices (Sec. 2.2, 2.4), prolongation from the subdivision
               formula (eq. 2.5, 2.6), the grid hierarchy (Sec. 3.2.1).
- ``mg``       the assembled-matrix V-cycle (Alg. 7 with the Jacobi
               smoother of Alg. 6), MGCG (Alg. 8), plain CG, the damping
               parameter from a short Lanczos estimate of the largest
               eigenvalue of D^-1 A (a reading: the paper gives no value),
               the direct solve.
- ``matfree``  a matrix-free CPU apply and per-coefficient sampled outputs
               for sizes where assembly is too large.

Parity status of every function is stated in its docstring; a function with
no independent pin says "parity unpinned".
"""
