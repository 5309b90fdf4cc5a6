"""CPU FP64 oracle for the Lindblad steady-state / spectrum / gradient path.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import anything from this package.  The
library path (the HIP kernels behind the C ABI and its Python binding) never
imports it, and it never imports the library: the two share no code.  The only
common module is ``lind_inputs``, which defines seeded inputs and holds none of
the method's arithmetic.

Everything here is plain, slow and written to be checked by eye against the
paper (arXiv 2608.30860, "Well-conditioned iterative methods for large open
quantum systems"):

* ``oracle.lindblad`` -- the operators L, S, K, Phi, the Lyapunov solve, the
  dense column-stacked superoperator, dense steady states and spectra
  (plain definitions).
* ``oracle.krylov``   -- matrix-free reference solvers for sizes where the dense
  superoperator does not fit: the steady state as the fixed point of Phi
  (Algorithm "steady state as fixed point of Phi" with the eigendecomposition
  no-jump resolvent), right-preconditioned GMRES with the deflated no-jump
  preconditioner, and shift-invert Arnoldi for the low-lying spectrum.
* ``oracle.gradient`` -- gradients of <O> = Re Tr(O rho_inf): dense forward
  sensitivity (one linear solve per real direction), the adjoint formula, and
  central finite differences.
* ``oracle.dynamics`` -- the resolvent (lambda - L)^{-1} (dense definition, the
  series of the resolvent corollary, right-preconditioned GMRES), the contraction
  norm of K R^S_lambda, and the implicit Euler step (I - dt L)^{-1}.

Parity status of every function is stated in its docstring.  Nothing in the
oracle is "parity unpinned" except the matrix-free spectrum at sizes where no
dense reference exists (certified there only by its own residual).
"""
from . import lindblad, krylov, gradient, dynamics  # noqa: F401
