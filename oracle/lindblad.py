"""Plain FP64 definitions of the Lindbladian and its no-jump / jump split.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Paper references are to arXiv 2608.30860:
  eq. (lindblad_def)               L(rho) = -i[H, rho] + sum_j (L_j rho L_j^+ - 1/2 {L_j^+ L_j, rho})
  eq. (lindblad_decomposition)/(G) L = S + K,  S(X) = G X + X G^+,  K(X) = sum_j L_j X L_j^+,
                                   G = -i H - 1/2 sum_j L_j^+ L_j
  eq. (lyapunov)/(lyapunov_solution)  S(X) = Y  <=>  X = -int_0^inf e^{tG} Y e^{tG^+} dt
  Section 2.2                      Phi = -K S^{-1}
  eq. (steady_state_linear_problem) L~_eta(rho) = L(rho) + eta Tr(rho) I,  L~_eta rho = eta I
  eq. (no-jump-resolvent-precond), (G-lambda)  R^S_lambda = (lambda - S)^{-1},
                                   (lambda - S)(X) = -(G_lambda X + X G_lambda^+), G_lambda = G - lambda/2 I
  eq. (ShermanMorr), Algorithm "Precond"  deflated no-jump preconditioner
  eq. (lyapu_eig_solution), Algorithm "No-jump resolvent via eigendecomposition"

Vectorisation convention (dense superoperators): column stacking,
vec(A X B) = (B^T kron A) vec(X), i.e. ``vec(X) = X.reshape(-1, order="F")``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

# ----------------------------------------------------------------------------
# helpers
# ----------------------------------------------------------------------------

def dag(A: np.ndarray) -> np.ndarray:
    return A.conj().T


def vec(X: np.ndarray) -> np.ndarray:
    return np.asarray(X).reshape(-1, order="F")


def unvec(x: np.ndarray, n: int) -> np.ndarray:
    return np.asarray(x).reshape((n, n), order="F")


def hs_inner(A: np.ndarray, B: np.ndarray) -> complex:
    """Hilbert-Schmidt product <A, B> = Tr(A^+ B)."""
    return complex(np.vdot(A.reshape(-1), B.reshape(-1)))


def trace_norm(A: np.ndarray) -> float:
    """||A||_1 = Tr sqrt(A^+ A) = sum of singular values (Section 1.2 notation)."""
    return float(np.sum(np.linalg.svd(A, compute_uv=False)))


def max_norm(A: np.ndarray) -> float:
    """Entrywise max-norm used by the paper as its stopping criterion."""
    return float(np.max(np.abs(A)))


def hermitize(A: np.ndarray) -> np.ndarray:
    return 0.5 * (A + dag(A))


def trace_distance(A: np.ndarray, B: np.ndarray) -> float:
    """1/2 ||A - B||_1."""
    return 0.5 * trace_norm(A - B)


# ----------------------------------------------------------------------------
# operators (eq. lindblad_def, lindblad_decomposition, G)
# ----------------------------------------------------------------------------

def no_jump_generator(H: np.ndarray, Ls) -> np.ndarray:
    """G = -iH - 1/2 sum_j L_j^+ L_j   (eq. G)."""
    G = -1j * np.asarray(H, dtype=np.complex128)
    for L in Ls:
        G = G - 0.5 * (dag(L) @ L)
    return G


def lindblad_apply(H, Ls, rho):
    """L(rho) written term by term from eq. (lindblad_def); does not go through G."""
    out = -1j * (H @ rho - rho @ H)
    for L in Ls:
        LdL = dag(L) @ L
        out = out + L @ rho @ dag(L) - 0.5 * (LdL @ rho + rho @ LdL)
    return out


def lindblad_adjoint_apply(H, Ls, X):
    """Hilbert-Schmidt adjoint L*(X) = i[H, X] + sum_j (L_j^+ X L_j - 1/2 {L_j^+ L_j, X}).

    Defined by <L*(X), Y> = <X, L(Y)> for all X, Y (Section 1.2 notation for X*)."""
    out = 1j * (H @ X - X @ H)
    for L in Ls:
        LdL = dag(L) @ L
        out = out + dag(L) @ X @ L - 0.5 * (LdL @ X + X @ LdL)
    return out


def S_apply(G, X):
    """No-jump part S(X) = G X + X G^+   (eq. lindblad_decomposition)."""
    return G @ X + X @ dag(G)


def K_apply(Ls, X):
    """Jump part K(X) = sum_j L_j X L_j^+   (eq. lindblad_decomposition)."""
    out = np.zeros_like(X, dtype=np.complex128)
    for L in Ls:
        out = out + L @ X @ dag(L)
    return out


def deflated_apply(H, Ls, rho, eta=1.0):
    """L~_eta(rho) = L(rho) + eta Tr(rho) I   (eq. steady_state_linear_problem)."""
    n = rho.shape[0]
    return lindblad_apply(H, Ls, rho) + eta * np.trace(rho) * np.eye(n)


# ----------------------------------------------------------------------------
# Lyapunov solves
# ----------------------------------------------------------------------------

def lyap_solve(G, Y, mu=0.0):
    """X with (S - mu)(X) = Y, i.e. (G - mu/2) X + X (G - mu/2)^+ = Y.

    mu = 0 gives S^{-1}(Y) (eq. lyapunov).  Uses LAPACK's Bartels-Stewart solver
    through ``scipy.linalg.solve_continuous_lyapunov`` (which solves
    A X + X A^H = Q).  The resolvent of the paper is R^S_mu = (mu - S)^{-1} = -this.
    """
    n = G.shape[0]
    A = G - 0.5 * mu * np.eye(n)
    return sla.solve_continuous_lyapunov(A, Y)


def lyap_solve_kron(G, Y, mu=0.0):
    """Same as ``lyap_solve`` by a dense Kronecker solve (tiny n only):
    (I kron G_mu + conj(G_mu) kron I) vec X = vec Y with G_mu = G - mu/2 I."""
    n = G.shape[0]
    I = np.eye(n)
    Gm = G - 0.5 * mu * I
    A = np.kron(I, Gm) + np.kron(Gm.conj(), I)
    return unvec(np.linalg.solve(A, vec(Y)), n)


def resolvent_S(G, Y, lam=0.0):
    """No-jump resolvent R^S_lambda(Y) = (lambda - S)^{-1} Y   (eq. no-jump-resolvent-precond)."""
    return -lyap_solve(G, Y, lam)


def phi_apply(G, Ls, xi):
    """Phi(xi) = -K(S^{-1} xi)   (Section 2.2)."""
    return -K_apply(Ls, lyap_solve(G, xi))


def precond_apply(G, X, lam, c, W=None):
    """Algorithm "Precond": Z = R^S_lam(X); W = R^S_lam(I);
    return Z + c Tr(Z) / (1 - c Tr W) W   (eq. ShermanMorr for a general shift)."""
    n = G.shape[0]
    Z = resolvent_S(G, X, lam)
    if W is None:
        W = resolvent_S(G, np.eye(n, dtype=np.complex128), lam)
    denom = 1.0 - c * np.trace(W)
    return Z + (c * np.trace(Z) / denom) * W


class EigResolvent:
    """Algorithm "No-jump resolvent via eigendecomposition" (eq. lyapu_eig_solution).

    Precompute once G = U Sigma U^{-1}, V = U^{-+}; then
    R^S_lambda(Y) = U [ (V^+ Y V)_ij / (lambda - s_i - conj(s_j)) ] U^+.
    Used by the matrix-free reference solvers at sizes where ``lyap_solve``
    (one Schur factorisation per call) would be too slow.
    """

    def __init__(self, G):
        s, U = np.linalg.eig(G)
        self.s = s
        self.U = U
        self.V = dag(np.linalg.inv(U))

    def resolvent(self, Y, lam=0.0):
        D = lam - self.s[:, None] - self.s.conj()[None, :]
        Yh = dag(self.V) @ Y @ self.V
        return self.U @ (Yh / D) @ dag(self.U)

    def sinv(self, Y, mu=0.0):
        """(S - mu)^{-1} Y = -R^S_mu(Y)."""
        return -self.resolvent(Y, mu)

    def kappa(self):
        Un = self.U / np.linalg.norm(self.U, axis=0)[None, :]
        return float(np.linalg.cond(Un))


def gauge_shift(H, Ls, c):
    """Remark "Non-uniqueness of the decomposition", eq. lindblad_gauge:
    Lt_j = L_j + c_j I,  Ht = H + (1/2i) sum_j (conj(c_j) Lt_j - c_j Lt_j^+).
    The pair (Ht, Lt) defines the same Lindbladian with another no-jump / jump split."""
    n = H.shape[0]
    I = np.eye(n, dtype=np.complex128)
    Lt = [L + cj * I for L, cj in zip(Ls, c)]
    Ht = H.astype(np.complex128) + sum((np.conj(cj) * L - cj * dag(L)) for L, cj in zip(Lt, c)) / 2j
    return Ht, Lt


# ----------------------------------------------------------------------------
# dense superoperators (column stacking)
# ----------------------------------------------------------------------------

def superop_dense(H, Ls):
    """Dense n^2 x n^2 matrix of L with vec(A X B) = (B^T kron A) vec X:
    -i(I kron H - H^T kron I) + sum_j [conj(L_j) kron L_j - 1/2 I kron L_j^+L_j
    - 1/2 (L_j^+ L_j)^T kron I]."""
    n = H.shape[0]
    I = np.eye(n)
    M = -1j * (np.kron(I, H) - np.kron(H.T, I))
    for L in Ls:
        LdL = dag(L) @ L
        M = M + np.kron(L.conj(), L) - 0.5 * np.kron(I, LdL) - 0.5 * np.kron(LdL.T, I)
    return M


def superop_of_map(fn, n):
    """Dense matrix of any linear map on n x n matrices, column by column."""
    M = np.zeros((n * n, n * n), dtype=np.complex128)
    for k in range(n * n):
        E = unvec(np.eye(n * n, dtype=np.complex128)[:, k], n)
        M[:, k] = vec(fn(E))
    return M


def steady_state_dense(H, Ls, eta=1.0):
    """rho_inf from the deflated linear problem L~_eta rho = eta I solved densely
    (eq. steady_state_linear_problem); <I|rho> = Tr rho = vec(I)^H vec(rho).
    Returned hermitised and trace-normalised."""
    n = H.shape[0]
    M = superop_dense(H, Ls)
    vI = vec(np.eye(n, dtype=np.complex128))
    A = M + eta * np.outer(vI, vI.conj())
    rho = unvec(np.linalg.solve(A, eta * vI), n)
    rho = hermitize(rho)
    return rho / np.trace(rho).real


def steady_state_svd(H, Ls):
    """Null vector of the dense superoperator via its smallest singular value
    (the dense-SVD route of Section 2.1), trace-normalised."""
    n = H.shape[0]
    M = superop_dense(H, Ls)
    _, _, Vh = np.linalg.svd(M)
    rho = unvec(Vh[-1].conj(), n)
    rho = rho / np.trace(rho)
    return hermitize(rho)


def spectrum_dense(H, Ls):
    """All n^2 eigenvalues of L (dense eig)."""
    return np.linalg.eigvals(superop_dense(H, Ls))


def low_spectrum_dense(H, Ls, k, drop_zero=True):
    """k smallest-magnitude eigenvalues of L; the zero mode (steady state) is dropped
    by removing eta*n from the spectrum of L~_eta (Section 4.2, deflating the zero mode).
    Sorted by |lambda| ascending, ties by Im ascending."""
    n = H.shape[0]
    eta = 1.0
    M = superop_dense(H, Ls)
    vI = vec(np.eye(n, dtype=np.complex128))
    ev = np.linalg.eigvals(M + eta * np.outer(vI, vI.conj())) if drop_zero else np.linalg.eigvals(M)
    if drop_zero:
        j = int(np.argmin(np.abs(ev - eta * n)))
        ev = np.delete(ev, j)
    order = np.lexsort((ev.imag, np.round(np.abs(ev), 12)))
    return ev[order][:k]


def low_eigenpairs_dense(H, Ls, k):
    """k smallest-magnitude nonzero eigenpairs of L (dense); eigenvectors as n x n
    matrices with unit Frobenius norm."""
    n = H.shape[0]
    eta = 1.0
    M = superop_dense(H, Ls)
    vI = vec(np.eye(n, dtype=np.complex128))
    ev, W = np.linalg.eig(M + eta * np.outer(vI, vI.conj()))
    j = int(np.argmin(np.abs(ev - eta * n)))
    keep = [i for i in range(len(ev)) if i != j]
    ev = ev[keep]
    W = W[:, keep]
    order = np.lexsort((ev.imag, np.round(np.abs(ev), 12)))[:k]
    vecs = [unvec(W[:, i] / np.linalg.norm(W[:, i]), n) for i in order]
    return ev[order], vecs


def choi(fn, n):
    """Choi matrix sum_ij |i><j| kron fn(|i><j|): PSD iff fn is completely positive."""
    C = np.zeros((n * n, n * n), dtype=np.complex128)
    for i in range(n):
        for j in range(n):
            E = np.zeros((n, n), dtype=np.complex128)
            E[i, j] = 1.0
            C[i * n:(i + 1) * n, j * n:(j + 1) * n] = fn(E)
    return C


def lyap_integral(G, Y, t_max=60.0, steps=6000):
    """-int_0^T e^{tG} Y e^{tG^+} dt by composite Simpson (eq. lyapunov_solution);
    an independent check of the sign and form of S^{-1} for small, stable G."""
    h = t_max / steps
    E = sla.expm(h * G)
    P = np.eye(G.shape[0], dtype=np.complex128)
    acc = np.zeros_like(Y, dtype=np.complex128)
    for k in range(steps + 1):
        w = 1.0 if k in (0, steps) else (4.0 if k % 2 else 2.0)
        acc = acc + w * (P @ Y @ dag(P))
        P = E @ P
    return -(h / 3.0) * acc
