"""Gradients of J = Re Tr(O rho_inf) with respect to H and the jump operators.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Convention: for a complex matrix parameter Z, the gradient g satisfies
dJ = Re Tr(g^+ dZ) for every complex direction dZ, i.e. g = dJ/dRe Z + i dJ/dIm Z
(the convention PyTorch uses for real losses of complex tensors).

Three independent routes:
* ``grad_forward_dense``  -- dense forward sensitivity, one solve per real direction:
  L~_eta drho = -(dL) rho_inf with Tr drho = 0, dJ = Re Tr(O drho).  It never uses the
  adjoint formula, so it checks it (Remark "Differentiating the steady state").
* ``grad_adjoint``        -- the adjoint route of that remark: solve L* mu = O - <O> I
  (through the deflated adjoint operator; densely, or matrix-free by ``adjoint_state_gmres``), then
  g_H = i [rho, mu],  g_Lj = L_j {rho, mu} - 2 mu L_j rho.
* ``grad_fd``             -- central finite differences of J along given directions.
"""
from __future__ import annotations

import numpy as np

from .lindblad import dag, hermitize, lindblad_adjoint_apply, steady_state_dense, superop_dense, unvec, vec


def expectation(O, rho):
    return float(np.real(np.trace(O @ rho)))


def dL_apply(H, Ls, dH, dLs, rho):
    """Directional derivative (dL)(rho) of eq. (lindblad_def) for perturbations dH, dL_j."""
    out = -1j * (dH @ rho - rho @ dH)
    for L, dL in zip(Ls, dLs):
        dLdL = dag(dL) @ L + dag(L) @ dL
        out = out + dL @ rho @ dag(L) + L @ rho @ dag(dL) - 0.5 * (dLdL @ rho + rho @ dLdL)
    return out


def grad_forward_dense(H, Ls, O, eta=1.0):
    """Full gradients by dense forward sensitivity (tiny n).  Returns (J, g_H, [g_L])."""
    n = H.shape[0]
    rho = steady_state_dense(H, Ls, eta)
    M = superop_dense(H, Ls)
    vI = vec(np.eye(n, dtype=np.complex128))
    A = M + eta * np.outer(vI, vI.conj())
    Ainv = np.linalg.inv(A)
    J = expectation(O, rho)

    def dJ(dH, dLs):
        rhs = -vec(dL_apply(H, Ls, dH, dLs, rho))
        drho = unvec(Ainv @ rhs, n)
        return float(np.real(np.trace(O @ drho)))

    zeros = [np.zeros((n, n), dtype=np.complex128) for _ in Ls]
    gH = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            E = np.zeros((n, n), dtype=np.complex128)
            E[a, b] = 1.0
            gH[a, b] = dJ(E, zeros) + 1j * dJ(1j * E, zeros)
    gL = []
    for j in range(len(Ls)):
        g = np.zeros((n, n), dtype=np.complex128)
        for a in range(n):
            for b in range(n):
                E = np.zeros((n, n), dtype=np.complex128)
                E[a, b] = 1.0
                dl = list(zeros)
                dl[j] = E
                re = dJ(zeros[0], dl)
                dl[j] = 1j * E
                im = dJ(zeros[0], dl)
                g[a, b] = re + 1j * im
        gL.append(g)
    return J, gH, gL


def adjoint_state_dense(H, Ls, O, rho, eta=1.0):
    """mu solving L*(mu) = O - <O> I, Tr mu = 0, via the deflated adjoint
    (L~_eta)*(X) = L*(X) + eta Tr(X) I solved densely."""
    n = H.shape[0]
    M = superop_dense(H, Ls)
    vI = vec(np.eye(n, dtype=np.complex128))
    A = M + eta * np.outer(vI, vI.conj())
    rhs = O - expectation(O, rho) * np.eye(n)
    mu = unvec(np.linalg.solve(dag(A), vec(rhs)), n)
    return hermitize(mu)


def adjoint_state_gmres(H, Ls, O, rho, eta=1.0, rtol=1e-13, m=40, max_cycles=60):
    """Matrix-free form of ``adjoint_state_dense`` for sizes where the superoperator does not fit:
    the deflated adjoint system (L~_eta)*(mu) = L*(mu) + eta Tr(mu) I = O - <O> I (the adjoint of
    eq. steady_state_linear_problem's operator) solved by the oracle's right-preconditioned GMRES
    with the adjoint no-jump inverse S*^{-1}, S*(X) = G^+ X + X G, as preconditioner (the Remark
    "Differentiating the steady state" preconditions the adjoint solve with the adjoint Lyapunov
    operator).  S*^{-1} is the eigendecomposition solve of eq. lyapu_eig_solution applied to G^+
    (its Lyapunov equation G^+ X + X (G^+)^+ = Y is S*(X) = Y).  Returned hermitised.
    Pinned against ``adjoint_state_dense`` at small n in the oracle's tests."""
    from .krylov import gmres
    from .lindblad import EigResolvent, no_jump_generator

    n = H.shape[0]
    G = no_jump_generator(H, Ls)
    Radj = EigResolvent(dag(G))
    I = np.eye(n, dtype=np.complex128)
    rhs = O - expectation(O, rho) * I

    def A(X):
        return lindblad_adjoint_apply(H, Ls, X) + eta * np.trace(X) * I

    mu = gmres(A, rhs, apply_P=Radj.sinv, m=m, max_cycles=max_cycles, atol=rtol * np.linalg.norm(rhs))
    return hermitize(mu)


def grad_from_adjoint(Ls, rho, mu):
    """g_H = i[rho, mu],  g_Lj = L_j {rho, mu} - 2 mu L_j rho."""
    gH = 1j * (rho @ mu - mu @ rho)
    gL = [L @ (rho @ mu + mu @ rho) - 2.0 * mu @ L @ rho for L in Ls]
    return gH, gL


def grad_adjoint(H, Ls, O, eta=1.0):
    rho = steady_state_dense(H, Ls, eta)
    mu = adjoint_state_dense(H, Ls, O, rho, eta)
    gH, gL = grad_from_adjoint(Ls, rho, mu)
    return expectation(O, rho), gH, gL, mu


def grad_fd(J_of, H, Ls, directions, h=1e-6):
    """Central differences of J along directions [(dH, [dL_j])]; returns array of dJ."""
    out = []
    for dH, dLs in directions:
        Jp = J_of(H + h * dH, [L + h * dL for L, dL in zip(Ls, dLs)])
        Jm = J_of(H - h * dH, [L - h * dL for L, dL in zip(Ls, dLs)])
        out.append((Jp - Jm) / (2 * h))
    return np.array(out)


def directional(gH, gLs, dH, dLs):
    """dJ = Re Tr(g^+ dZ) summed over parameters."""
    s = np.real(np.vdot(gH.reshape(-1), dH.reshape(-1)))
    for g, d in zip(gLs, dLs):
        s += np.real(np.vdot(g.reshape(-1), d.reshape(-1)))
    return float(s)


def random_directions(n, d, count, seed=2):
    """Hermitian directions for H, complex for each L_j, jointly unit-normalised."""
    rng = np.random.default_rng(seed)
    dirs = []
    for _ in range(count):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        dH = 0.5 * (A + dag(A))
        dLs = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(d)]
        nrm = np.sqrt(np.linalg.norm(dH) ** 2 + sum(np.linalg.norm(x) ** 2 for x in dLs))
        dirs.append((dH / nrm, [x / nrm for x in dLs]))
    return dirs
