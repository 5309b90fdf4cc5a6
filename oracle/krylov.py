"""Matrix-free FP64 reference solvers for sizes where the dense superoperator
does not fit (n >~ 48).

TEST INFRASTRUCTURE ONLY (see the package docstring).

These follow the paper's algorithms step by step, in plain NumPy, with the
no-jump resolvent of eq. (lyapu_eig_solution) (class ``EigResolvent``):

* ``steady_state_phi``  -- Algorithm "Steady state as the fixed point of Phi":
  explicitly restarted Arnoldi(m) on Phi = -K S^{-1}; keep the Ritz vector whose
  Ritz value is nearest 1; rho = -S^{-1} xi, hermitise, normalise; stop on the
  residual; restart from xi; return the running best.
* ``gmres``              -- right-preconditioned restarted GMRES (Section A.2).
* ``low_spectrum``       -- Algorithm "Low-lying spectrum via shift-invert Arnoldi":
  the outer Arnoldi is ARPACK (scipy.sparse.linalg.eigs, a library primitive) on
  OP = (mu - L~_eta)^{-1}; each OP application is a right-preconditioned GMRES
  solve with P_mu = Precond(., mu, eta); eigenvalues of L are mu - 1/nu.

Parity: the results are certified by their own residuals (||L rho||, ||L v - lambda v||)
and checked against the dense definitions in ``oracle.lindblad`` at n <= 48 in the
oracle's own tests.  At sizes with no dense reference the spectrum is
"parity unpinned" beyond its residual certificate.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla

from .lindblad import (EigResolvent, K_apply, S_apply, dag, deflated_apply, hermitize,
                       lindblad_apply, max_norm, no_jump_generator, trace_norm)


def _ritz_nearest_one(theta):
    """Index of the Ritz value nearest 1; ties broken toward real, then Im >= 0."""
    dist = np.abs(theta - 1.0)
    best = np.min(dist)
    cand = [i for i in range(len(theta)) if dist[i] <= best * (1 + 1e-9) + 1e-14]
    cand.sort(key=lambda i: (abs(theta[i].imag), -theta[i].imag))
    return cand[0]


def arnoldi(op, v0, m):
    """m steps of Arnoldi with modified Gram-Schmidt plus one re-orthogonalisation
    pass, in the Hilbert-Schmidt product.  Returns (V list of m+1, H (m+1) x m)."""
    V = [v0 / np.linalg.norm(v0)]
    Hm = np.zeros((m + 1, m), dtype=np.complex128)
    for k in range(m):
        w = op(V[k])
        for _ in range(2):
            for j in range(k + 1):
                h = np.vdot(V[j].reshape(-1), w.reshape(-1))
                Hm[j, k] += h
                w = w - h * V[j]
        Hm[k + 1, k] = np.linalg.norm(w)
        if Hm[k + 1, k] == 0:
            return V, Hm[: k + 2, : k + 1]
        V.append(w / Hm[k + 1, k])
    return V, Hm


def steady_state_phi(H, Ls, tol=1e-10, m=30, max_restarts=200, rho0=None, norm="trace",
                     return_info=False):
    """Algorithm "Steady state as the fixed point of Phi" (Section A.2), FP64.

    Start vector: xi_0 = -S(rho_0) (so that -S^{-1} xi_0 = rho_0); rho_0 = I/n by default.
    Stopping norm: the trace norm of L(rho_hat) by default ("max" for the paper's
    max-norm test)."""
    n = H.shape[0]
    G = no_jump_generator(H, Ls)
    R = EigResolvent(G)
    sinv = R.sinv

    def phi(xi):
        return -K_apply(Ls, sinv(xi))

    if rho0 is None:
        rho0 = np.eye(n, dtype=np.complex128) / n
    xi = -S_apply(G, rho0)
    best = (np.inf, None)
    n_phi = 0
    for j in range(max_restarts):
        V, Hm = arnoldi(phi, xi, m)
        n_phi += Hm.shape[1]
        k = Hm.shape[1]
        theta, Y = np.linalg.eig(Hm[:k, :k])
        i = _ritz_nearest_one(theta)
        y = Y[:, i]
        xi = sum(y[t] * V[t] for t in range(k))
        rho = -sinv(xi)
        rho = hermitize(rho)
        rho = rho / np.trace(rho).real
        r = lindblad_apply(H, Ls, rho)
        res = trace_norm(r) if norm == "trace" else max_norm(r)
        if res < best[0]:
            best = (res, rho)
        if res < tol:
            break
        xi = xi / np.linalg.norm(xi)
    if return_info:
        return best[1], dict(resid=best[0], n_phi=n_phi, restarts=j + 1, kappa=R.kappa())
    return best[1]


def gmres(apply_A, b, apply_P=None, x0=None, m=30, max_cycles=50, atol=1e-12):
    """Right-preconditioned restarted GMRES(m): solve A x = b with x = P y.
    Least squares by a dense solve of the small Hessenberg problem."""
    if apply_P is None:
        apply_P = lambda X: X  # noqa: E731
    x = np.zeros_like(b) if x0 is None else x0.copy()
    for _ in range(max_cycles):
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        if beta < atol:
            break
        V, Hm = arnoldi(lambda v: apply_A(apply_P(v)), r, m)
        k = Hm.shape[1]
        e1 = np.zeros(Hm.shape[0], dtype=np.complex128)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(Hm, e1, rcond=None)
        x = x + apply_P(sum(y[t] * V[t] for t in range(k)))
    return x


def low_spectrum(H, Ls, k, mu=0.0, eta=1.0, tol=1e-10, inner_tol=1e-13, seed=5):
    """Algorithm "Low-lying spectrum via shift-invert Arnoldi" (Section A.2).

    Returns (eigenvalues of L sorted by |lambda|, list of eigenvector matrices).
    Outer Arnoldi: ARPACK on OP = (mu - L~_eta)^{-1}; inner: right-preconditioned GMRES
    with Precond(., mu, eta)."""
    n = H.shape[0]
    G = no_jump_generator(H, Ls)
    R = EigResolvent(G)
    I = np.eye(n, dtype=np.complex128)
    W = R.resolvent(I, mu)
    trW = np.trace(W)

    def P(X):
        Z = R.resolvent(X, mu)
        return Z + (eta * np.trace(Z) / (1.0 - eta * trW)) * W

    def A(X):
        return mu * X - deflated_apply(H, Ls, X, eta)

    def op(x):
        X = x.reshape(n, n)
        B = gmres(A, X, P, m=40, max_cycles=40, atol=inner_tol * max(1.0, np.linalg.norm(X)))
        return B.reshape(-1)

    LO = spla.LinearOperator((n * n, n * n), matvec=op, dtype=np.complex128)
    rng = np.random.default_rng(seed)
    v0 = rng.standard_normal(n * n) + 1j * rng.standard_normal(n * n)
    nu, W_ = spla.eigs(LO, k=k, which="LM", v0=v0, tol=tol, ncv=max(2 * k + 1, 20))
    lam = mu - 1.0 / nu
    order = np.argsort(np.abs(lam))
    vecs = [W_[:, i].reshape(n, n) / np.linalg.norm(W_[:, i]) for i in order]
    return lam[order], vecs


def eigen_residual(H, Ls, lam, X):
    """max-norm of L(X) - lambda X (Algorithm "Low-lying spectrum" stopping test)."""
    return max_norm(lindblad_apply(H, Ls, X) - lam * X)
