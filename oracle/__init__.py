"""CPU FP64 oracle for the substructuring Schur-complement solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the GPU solver
neither imports it nor shares any code with it.

Plain, slow, obviously correct numpy/scipy implementations of what the
solver computes (arXiv:2306.00094):

* ``monolithic_solve`` -- u* = A^{-1} b for the discrete system of the
  section "A discretized weak formulation" (A symmetric positive definite
  when the Dirichlet collar is non-empty), by a banded Cholesky factorisation
  in the natural node order (LAPACK routine used as one step).
* ``jacobi_pcg`` -- the paper's baseline solver: CG on the whole system
  with the diagonal of A as preconditioner (section "Considered solver
  strategies"), x0 = 0, independent columns, the same stopping rule as below.
* ``DDOracle`` -- the same substructuring method the GPU runs:
  - factor each interior block A^k_{Omega Omega} = L_k L_k^T
    (block Cholesky splitting, eq. splittingBlockCholesky);
  - Schur complement S = K_GG - sum_k R_k^T K_GI^k (K_II^k)^{-1} K_IG^k R_k
    applied matrix-free (eq. subSchurComplement; the sum over subdomains of
    eq. SchurComplement with the interface parametrised by one global
    interface vector);
  - reduced forcing g = b_G - sum_k R_k^T K_GI^k (K_II^k)^{-1} b_I^k
    (eq. subForcing);
  - preconditioned conjugate gradients on S u_G = g with the exact diagonal
    of S as Jacobi preconditioner, x0 = 0, every right-hand side column an
    independent CG;
  - back substitution u_I^k = (K_II^k)^{-1} (b_I^k - K_IG^k u_G)
    (eq. backwardSubstitution).

Readings where the paper is silent (the paper's own solver is the dual
FETI method; it fixes no primal preconditioner, no norm for its 1e-10
tolerance and no multi-RHS scheme):
  * stop column c when ||r_G,c||_2 <= tol * ||b_c||_2 -- after exact back
    substitution ||b - A u|| equals ||r_G||, so tol is the relative residual
    of the full system;
  * Jacobi preconditioner with the exact diagonal of S.

Two further solvers of the same discrete system, each in its own module and
pinned by its own tests:
* ``feti_oracle.FETIOracle`` -- the paper's one-level FETI (section "FETI",
  Algorithm 1) on zeta-weighted subdomain matrices (tests/test_feti_oracle.py);
* ``bdd_oracle.BDDOracle`` -- the primal interface problem with the balancing
  Neumann-Neumann preconditioner built from the same pinned pseudoinverses
  (tests/test_bdd_oracle.py).

Pins of this oracle (tests/test_oracle.py): brute-force dense inverses on
tiny systems, explicit dense Schur complements, DD-vs-monolithic agreement,
CG termination in at most n_G steps, symmetry of S; for jacobi_pcg: the
first iterates of a 2x2 system worked by hand in exact fractions, one-step
convergence on diagonal systems, termination in n steps, agreement with the
banded Cholesky solution.
"""
from .dd_oracle import (DDOracle, cholesky, monolithic_solve, rel_err,  # noqa: F401
                        full_residual, jacobi_pcg)
