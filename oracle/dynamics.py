"""Resolvent of the Lindbladian and the implicit Euler step, plain FP64 references.

TEST INFRASTRUCTURE ONLY (see the package docstring).

* ``resolvent_dense``   -- (lambda - L)^{-1} B by a dense solve with the n^2 x n^2 superoperator
  (the plain definition; small n).
* ``resolvent_series``  -- Corollary "Resolvent of the Lindbladian" (eq. thm-main):
  R^L_lambda = R^S_lambda sum_k (K R^S_lambda)^k, truncated.
* ``contraction_norm``  -- the trace-norm-induced norm of K R^S_lambda (Theorem "contraction");
  for a completely positive map T it equals || T^*(I) ||_inf, and
  (K R^S_lambda)^*(I) = R^{S*}_lambda(sum_j L_j^+ L_j), with S*(Y) = G^+ Y + Y G.
* ``resolvent_gmres``   -- (lambda - L) X = B by right-preconditioned GMRES with R^S_lambda
  (eq. right-precond-identity), matrix-free, for sizes with no dense superoperator.
* ``implicit_euler_dense`` -- rho_{k+1} = (I - dt L)^{-1} rho_k (eq. resolvent of the implicit
  solver section), dense solves.
"""
from __future__ import annotations

import numpy as np

from .krylov import gmres
from .lindblad import EigResolvent, K_apply, dag, lindblad_apply, no_jump_generator, superop_dense, unvec, vec


def resolvent_dense(H, Ls, lam, B):
    """X = (lambda - L)^{-1} B from the dense superoperator (column stacking)."""
    n = H.shape[0]
    Lsup = superop_dense(H, Ls)
    A = lam * np.eye(n * n, dtype=np.complex128) - Lsup
    return unvec(np.linalg.solve(A, vec(B)), n)


def resolvent_series(H, Ls, lam, B, terms=200):
    """Truncated eq. thm-main: R^S_lambda applied to sum_{k < terms} (K R^S_lambda)^k B."""
    G = no_jump_generator(H, Ls)
    R = EigResolvent(G)
    acc = np.zeros_like(B, dtype=np.complex128)
    term = B.astype(np.complex128)
    for _ in range(terms):
        acc = acc + term
        term = K_apply(Ls, R.resolvent(term, lam))
    return R.resolvent(acc, lam)


def contraction_norm(H, Ls, lam):
    """|| K R^S_lambda ||_{1 -> 1} = || R^{S*}_lambda(sum_j L_j^+ L_j) ||_inf  (CP map)."""
    G = no_jump_generator(H, Ls)
    Radj = EigResolvent(dag(G))
    W = sum(dag(L) @ L for L in Ls)
    Y = Radj.resolvent(W, lam)
    Y = 0.5 * (Y + dag(Y))
    return float(np.max(np.linalg.eigvalsh(Y)))


def resolvent_gmres(H, Ls, lam, B, tol=1e-12, m=40, max_cycles=50):
    """(lambda - L) X = B by GMRES right-preconditioned with R^S_lambda (matrix-free)."""
    G = no_jump_generator(H, Ls)
    R = EigResolvent(G)

    def A(X):
        return lam * X - lindblad_apply(H, Ls, X)

    def P(X):
        return R.resolvent(X, lam)

    return gmres(A, B.astype(np.complex128), P, m=m, max_cycles=max_cycles,
                 atol=tol * max(1e-300, np.linalg.norm(B)))


def implicit_euler_dense(H, Ls, rho0, dt, steps):
    """States rho_1 .. rho_steps of rho_{k+1} = (I - dt L)^{-1} rho_k, dense solves."""
    n = H.shape[0]
    A = np.eye(n * n, dtype=np.complex128) - dt * superop_dense(H, Ls)
    out = []
    x = vec(rho0.astype(np.complex128))
    for _ in range(steps):
        x = np.linalg.solve(A, x)
        out.append(unvec(x, n))
    return out
