"""Seeded synthetic workloads: Hamiltonians, jump operators, observables, start states.

This module only *defines inputs*. It holds none of the method's arithmetic
(no G, no Lyapunov solve, no Phi, no Krylov step), so both the CPU oracle and the
HIP path may draw their inputs from it without sharing any computation.

Conventions
-----------
* Every matrix is a numpy ``complex128`` array, row-major, shape ``(n, n)``.
* Jump operators come as a list ``[L_1, ..., L_d]`` in the order the workload
  lists them.
* Bosonic modes use the truncated annihilation operator ``a`` with
  ``a[k, k+1] = sqrt(k+1)`` (Fock basis |0>..|n-1>), as in the paper's appendix on
  the benchmark systems.
* Two modes are combined by the row-major Kronecker product:
  ``a1 = a (x) I`` and ``a2 = I (x) a``.
* Random systems use ``numpy.random.default_rng(seed)`` (PCG64).  A complex
  Gaussian matrix with ``E|z|^2 = s2`` draws its real part (n*n, row-major) and then
  its imaginary part, each ``N(0, s2/2)``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "destroy", "kerr_cavity", "two_photon_cavity", "coupled_kerr", "random_dense",
    "random_dense_paper", "thermal_oscillator", "three_level_cyclic", "two_level_decay",
    "random_observable", "random_state", "workload", "WORKLOADS", "complex_gaussian",
    "vacuum", "maximally_mixed",
]


def destroy(n: int) -> np.ndarray:
    """Truncated annihilation operator on n Fock levels."""
    a = np.zeros((n, n), dtype=np.complex128)
    k = np.arange(1, n)
    a[k - 1, k] = np.sqrt(k)
    return a


def vacuum(n: int) -> np.ndarray:
    r = np.zeros((n, n), dtype=np.complex128)
    r[0, 0] = 1.0
    return r


def maximally_mixed(n: int) -> np.ndarray:
    return np.eye(n, dtype=np.complex128) / n


def kerr_cavity(n: int = 32, Delta: float = 0.5, eps: float = 1.0, K: float = 0.1,
                kappa: float = 1.0, gamma_dephasing: float | None = None):
    """Driven Kerr cavity.

    H = Delta a^dag a + eps (a + a^dag) + K a^dag^2 a^2,  L_1 = sqrt(kappa) a,
    and optionally L_2 = sqrt(gamma) a^dag a (dephasing).
    """
    a = destroy(n)
    ad = a.conj().T
    H = Delta * (ad @ a) + eps * (a + ad) + K * (ad @ ad @ a @ a)
    Ls = [np.sqrt(kappa) * a]
    if gamma_dephasing is not None:
        Ls.append(np.sqrt(gamma_dephasing) * (ad @ a))
    return H.astype(np.complex128), [L.astype(np.complex128) for L in Ls]


def two_photon_cavity(n: int = 256, alpha2: float = 4.0, kappa2: float = 1.0, kappa1: float = 1e-3):
    """Two-photon dissipation cavity: H = 0, L_1 = sqrt(k2)(a^2 - alpha^2 I), L_2 = sqrt(k1) a."""
    a = destroy(n)
    H = np.zeros((n, n), dtype=np.complex128)
    L1 = np.sqrt(kappa2) * (a @ a - alpha2 * np.eye(n))
    L2 = np.sqrt(kappa1) * a
    return H, [L1.astype(np.complex128), L2.astype(np.complex128)]


def coupled_kerr(n_mode: int = 40, Delta=(0.3, -0.2), K=(0.05, 0.08), g: float = 0.4,
                 eps: float = 0.8, kappa: float = 1.0, gamma: float = 0.1):
    """Two coupled Kerr cavities on n_mode^2 levels.

    H = sum_k [Delta_k a_k^dag a_k + K_k a_k^dag^2 a_k^2] + g (a1^dag a2 + a1 a2^dag)
        + eps (a1 + a1^dag);
    jumps, in order: sqrt(kappa) a1, sqrt(kappa) a2, sqrt(gamma) a1^dag a1,
    sqrt(gamma) a2^dag a2.
    """
    a = destroy(n_mode)
    I = np.eye(n_mode)
    a1 = np.kron(a, I)
    a2 = np.kron(I, a)
    ops = [a1, a2]
    H = np.zeros((n_mode * n_mode,) * 2, dtype=np.complex128)
    for k in range(2):
        ak = ops[k]
        akd = ak.conj().T
        H += Delta[k] * (akd @ ak) + K[k] * (akd @ akd @ ak @ ak)
    H += g * (a1.conj().T @ a2 + a1 @ a2.conj().T)
    H += eps * (a1 + a1.conj().T)
    Ls = [np.sqrt(kappa) * a1, np.sqrt(kappa) * a2,
          np.sqrt(gamma) * (a1.conj().T @ a1), np.sqrt(gamma) * (a2.conj().T @ a2)]
    return H, [L.astype(np.complex128) for L in Ls]


def complex_gaussian(rng: np.random.Generator, n: int, s2: float) -> np.ndarray:
    """n x n complex Gaussian, E|z|^2 = s2; real part drawn first, then imaginary."""
    sd = np.sqrt(s2 / 2.0)
    re = rng.standard_normal((n, n)) * sd
    im = rng.standard_normal((n, n)) * sd
    return (re + 1j * im).astype(np.complex128)


def random_dense(n: int, d: int, seed: int = 0):
    """Random dense Lindbladian.

    H = (A + A^dag)/2 with A complex Gaussian, E|A_ij|^2 = 1/n;
    L_j complex Gaussian with E|L_ij|^2 = 1/(n d), so sum_j L_j^dag L_j ~ I.
    Draw order: A, then L_1 .. L_d.
    """
    rng = np.random.default_rng(seed)
    A = complex_gaussian(rng, n, 1.0 / n)
    H = 0.5 * (A + A.conj().T)
    Ls = [complex_gaussian(rng, n, 1.0 / (n * d)) for _ in range(d)]
    return H, Ls


def random_dense_paper(n: int, d: int = 3, gamma: float = 0.1, seed: int = 0):
    """The paper's own dense family: real and imaginary parts i.i.d. N(0,1),
    H = (A_0 + A_0^dag)/2, L_j = sqrt(gamma) A_j."""
    rng = np.random.default_rng(seed)
    A = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for _ in range(d + 1)]
    H = 0.5 * (A[0] + A[0].conj().T)
    return H.astype(np.complex128), [np.sqrt(gamma) * A[j].astype(np.complex128) for j in range(1, d + 1)]


def thermal_oscillator(n: int, omega: float = 1.0, kappa: float = 1.0, nbar: float = 0.1):
    """H = omega N, L_1 = sqrt(kappa (1+nbar)) a, L_2 = sqrt(kappa nbar) a^dag."""
    a = destroy(n)
    ad = a.conj().T
    H = omega * (ad @ a)
    return H.astype(np.complex128), [np.sqrt(kappa * (1 + nbar)) * a, np.sqrt(kappa * nbar) * ad]


def three_level_cyclic():
    """Three-level cyclic example of the peripheral-spectrum remark:
    H = 0, L_1 = |0><1|, L_2 = |1><2|, L_3 = |2><0|."""
    n = 3
    H = np.zeros((n, n), dtype=np.complex128)
    Ls = []
    for (i, j) in [(0, 1), (1, 2), (2, 0)]:
        L = np.zeros((n, n), dtype=np.complex128)
        L[i, j] = 1.0
        Ls.append(L)
    return H, Ls


def two_level_decay(gamma: float = 1.0):
    """n = 2, H = 0, L = sqrt(gamma)|0><1| (the left/right preconditioning footnote)."""
    H = np.zeros((2, 2), dtype=np.complex128)
    L = np.zeros((2, 2), dtype=np.complex128)
    L[0, 1] = np.sqrt(gamma)
    return H, [L]


def random_observable(n: int, seed: int = 1) -> np.ndarray:
    """O = (B + B^dag)/2 with B complex Gaussian, E|B_ij|^2 = 1/n."""
    rng = np.random.default_rng(seed)
    B = complex_gaussian(rng, n, 1.0 / n)
    return 0.5 * (B + B.conj().T)


def random_state(n: int, seed: int = 3, hermitian: bool = True) -> np.ndarray:
    """A random test matrix (Hermitian PSD with unit trace by default)."""
    rng = np.random.default_rng(seed)
    B = complex_gaussian(rng, n, 1.0)
    if not hermitian:
        return B
    R = B @ B.conj().T
    return R / np.trace(R).real


# Named workloads (parameters exactly as the benchmark table states them).
WORKLOADS = {
    "kerr32": dict(n=32, d=1),
    "kerr32_linear": dict(n=32, d=1),
    "two_photon256": dict(n=256, d=2),
    "coupled_kerr1600": dict(n=1600, d=4),
    "random2048": dict(n=2048, d=8),
    "kerr512_dephasing": dict(n=512, d=2),
    "random1024_d4": dict(n=1024, d=4),
}


def workload(name: str, n: int | None = None, seed: int = 0):
    """Return (H, Ls, rho0) for a named workload; ``n`` overrides the size where
    the family allows it (used by small parity cases)."""
    if name == "kerr32":
        H, Ls = kerr_cavity(n or 32)
        return H, Ls, maximally_mixed(H.shape[0])
    if name == "kerr32_linear":
        H, Ls = kerr_cavity(n or 32, K=0.0)
        return H, Ls, maximally_mixed(H.shape[0])
    if name == "two_photon256":
        H, Ls = two_photon_cavity(n or 256)
        return H, Ls, vacuum(H.shape[0])
    if name == "coupled_kerr1600":
        m = int(round(np.sqrt(n))) if n else 40
        H, Ls = coupled_kerr(m)
        return H, Ls, maximally_mixed(H.shape[0])
    if name == "random2048":
        H, Ls = random_dense(n or 2048, 8, seed)
        return H, Ls, maximally_mixed(H.shape[0])
    if name == "kerr512_dephasing":
        H, Ls = kerr_cavity(n or 512, gamma_dephasing=0.05)
        return H, Ls, maximally_mixed(H.shape[0])
    if name == "random1024_d4":
        H, Ls = random_dense(n or 1024, 4, seed)
        return H, Ls, maximally_mixed(H.shape[0])
    raise KeyError(name)
