"""Pins for the CPU oracle: closed forms, worked examples printed in the paper,
invariants and brute force -- none of them re-types the oracle's own formulas.

Each test names the passage it follows.  ``test_planted_*`` plant a plausible
mistake in a copy of an oracle function (on the CPU) and check that a pin catches it.
"""
import os

import numpy as np
import pytest

import lind_inputs as li
from oracle import dynamics as od
from oracle import gradient as og
from oracle import krylov as ok
from oracle import lindblad as ol

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def read_golden(name):
    vals = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=")
            nums = [float(x) for x in v.split()]
            vals[k.strip()] = nums if len(nums) > 1 else nums[0]
    return vals


def coherent(n, beta):
    """Truncated coherent state |beta> (unit-normalised)."""
    k = np.arange(n)
    from scipy.special import gammaln
    amp = np.exp(-0.5 * abs(beta) ** 2 + k * np.log(abs(beta) + 0j) - 0.5 * gammaln(k + 1)) * np.exp(1j * k * np.angle(beta))
    amp = amp / np.linalg.norm(amp)
    return np.outer(amp, amp.conj())


# --------------------------------------------------------------------------------------
# operators against the textbook vec identity and closed forms
# --------------------------------------------------------------------------------------

def test_superop_matches_matrix_free():
    """Dense column-stacked superoperator (vec(AXB) = (B^T kron A) vec X) against the
    term-by-term definition, eq. (lindblad_def), on random matrices."""
    H, Ls = li.random_dense(6, 3, seed=11)
    X = li.random_state(6, seed=4, hermitian=False)
    M = ol.superop_dense(H, Ls)
    assert np.allclose(M @ ol.vec(X), ol.vec(ol.lindblad_apply(H, Ls, X)), atol=1e-13)
    # L = S + K with G of eq. (G)
    G = ol.no_jump_generator(H, Ls)
    assert np.allclose(ol.S_apply(G, X) + ol.K_apply(Ls, X), ol.lindblad_apply(H, Ls, X), atol=1e-13)


def test_trace_annihilation_and_hermiticity():
    """Tr L(X) = 0 and L(X^+) = L(X)^+ for every X (identity is a left null vector, Section 2.1)."""
    H, Ls = li.random_dense(7, 2, seed=3)
    X = li.random_state(7, seed=5, hermitian=False)
    LX = ol.lindblad_apply(H, Ls, X)
    assert abs(np.trace(LX)) < 1e-13
    assert np.allclose(ol.lindblad_apply(H, Ls, X.conj().T), LX.conj().T, atol=1e-13)


def test_adjoint_is_hs_adjoint():
    """<L*(X), Y> = <X, L(Y)> (Section 1.2 definition of X*)."""
    H, Ls = li.random_dense(5, 2, seed=8)
    X = li.random_state(5, seed=1, hermitian=False)
    Y = li.random_state(5, seed=2, hermitian=False)
    lhs = ol.hs_inner(ol.lindblad_adjoint_apply(H, Ls, X), Y)
    rhs = ol.hs_inner(X, ol.lindblad_apply(H, Ls, Y))
    assert abs(lhs - rhs) < 1e-12


def test_coherent_state_linear_cavity():
    """Kerr workload with K = 0: the steady state is |beta><beta|, beta = -i eps/(i Delta + kappa/2)."""
    g = read_golden("kerr_linear_coherent.txt")
    beta = -1j * g["eps"] / (1j * g["Delta"] + g["kappa"] / 2)
    assert abs(beta - complex(g["beta_re"], g["beta_im"])) < 1e-15
    H, Ls = li.kerr_cavity(32, Delta=g["Delta"], eps=g["eps"], K=0.0, kappa=g["kappa"])
    ref = coherent(32, beta)
    assert ol.max_norm(ol.lindblad_apply(H, Ls, ref)) < 1e-12
    rho = ol.steady_state_dense(H, Ls)
    assert ol.trace_distance(rho, ref) < 1e-12
    rho_svd = ol.steady_state_svd(H, Ls)
    assert ol.trace_distance(rho_svd, ref) < 1e-10


def test_thermal_state_is_geometric():
    """Damped oscillator at temperature: the truncated birth-death chain is in detailed balance,
    so p_k is exactly proportional to (nbar/(1+nbar))^k."""
    nbar = 0.3
    H, Ls = li.thermal_oscillator(12, omega=1.3, kappa=0.7, nbar=nbar)
    rho = ol.steady_state_dense(H, Ls)
    q = nbar / (1 + nbar)
    p = q ** np.arange(12)
    p /= p.sum()
    assert np.allclose(np.diag(rho).real, p, atol=1e-13)
    assert np.max(np.abs(rho - np.diag(np.diag(rho)))) < 1e-13


def test_thermal_low_spectrum():
    """Damped oscillator spectrum lambda = -i omega l - kappa (m + |l|/2), m >= 0, independent of
    nbar.  With omega = kappa = 1 the eight smallest nonzero moduli are -1, -1/2 +- i, -3/2 +- i,
    -2, -1 +- 2i; at n = 20 and nbar = 0.1 the truncation moves them by far less than 1e-10.
    Both multisets must match (nothing missing, nothing extra)."""
    H, Ls = li.thermal_oscillator(20, omega=1.0, kappa=1.0, nbar=0.1)
    ev = ol.low_spectrum_dense(H, Ls, 8)
    expected = np.array([-1.0, -0.5 - 1j, -0.5 + 1j, -1.5 - 1j, -1.5 + 1j, -2.0, -1 - 2j, -1 + 2j])
    for e in expected:
        assert np.min(np.abs(ev - e)) < 1e-10, e
    for e in ev:
        assert np.min(np.abs(expected - e)) < 1e-10, e
    # sorted by modulus, ties (the conjugate pairs) by Im ascending
    assert np.allclose(ev, expected, atol=1e-10)


def test_thermal_low_eigenpairs():
    """low_eigenpairs_dense: the same eigenvalues as low_spectrum_dense; every eigenvector is a unit
    matrix with L(v) = lambda v checked through the term-by-term L (not the Kronecker matrix that
    produced it); the mode -i omega l - kappa (m + |l|/2) is supported on the entries |k><k'| with
    k - k' = l (the phase-covariant oscillator conserves k - k'; -i[omega N, .] multiplies them by
    -i omega (k - k'))."""
    H, Ls = li.thermal_oscillator(20, omega=1.0, kappa=1.0, nbar=0.1)
    ev, vecs = ol.low_eigenpairs_dense(H, Ls, 8)
    assert np.allclose(ev, ol.low_spectrum_dense(H, Ls, 8), atol=1e-12)
    for lam, v in zip(ev, vecs):
        assert abs(np.linalg.norm(v) - 1) < 1e-12
        assert ol.max_norm(ol.lindblad_apply(H, Ls, v) - lam * v) < 1e-10
        ell = int(round(-lam.imag))  # omega = 1
        k, kp = np.nonzero(np.abs(v) > 1e-8)
        assert np.all(k - kp == ell), (lam, set(k - kp))


def test_three_level_cyclic_golden():
    """Remark "Peripheral spectra of Phi": rho_inf = I/3 and Phi has eigenvalues 1, exp(+-2 pi i/3)."""
    g = read_golden("three_level_cyclic.txt")
    H, Ls = li.three_level_cyclic()
    rho = ol.steady_state_dense(H, Ls)
    assert np.allclose(np.diag(rho).real, g["steady_state_diag"], atol=1e-14)
    G = ol.no_jump_generator(H, Ls)
    P = ol.superop_of_map(lambda X: ol.phi_apply(G, Ls, X), 3)
    ev = np.linalg.eigvals(P)
    per = np.array(g["peripheral_eigs_re"]) + 1j * np.array(g["peripheral_eigs_im"])
    for e in per:
        assert np.min(np.abs(ev - e)) < 1e-12
    assert np.sum(np.abs(np.abs(ev) - 1) < 1e-9) == 3
    # Algorithm 4 (Arnoldi, Ritz value nearest 1) still converges to I/3
    rho_a = ok.steady_state_phi(H, Ls, tol=1e-12, m=8)
    assert np.allclose(rho_a, np.eye(3) / 3, atol=1e-12)


def test_two_level_footnote_golden():
    """Footnote on left vs right preconditioning: R K rho = (gamma/lambda) rho_11 |0><0| and
    K R rho = gamma/(gamma+lambda) rho_11 |0><0| (resolvent R = (lambda - S)^{-1}, G_lambda = G - lambda/2)."""
    g = read_golden("two_level_footnote.txt")
    H, Ls = li.two_level_decay(g["gamma"])
    G = ol.no_jump_generator(H, Ls)
    rho = li.random_state(2, seed=9)
    lam = g["lambda"]
    RK = ol.resolvent_S(G, ol.K_apply(Ls, rho), lam)
    KR = ol.K_apply(Ls, ol.resolvent_S(G, rho, lam))
    E00 = np.array([[1, 0], [0, 0]], dtype=complex)
    assert np.allclose(RK, g["RK_coefficient"] * rho[1, 1] * E00, atol=1e-14)
    assert np.allclose(KR, g["KR_coefficient"] * rho[1, 1] * E00, atol=1e-14)


def test_lyapunov_three_ways():
    """S^{-1} by LAPACK Bartels-Stewart, by the Kronecker definition, and by the integral form
    eq. (lyapunov_solution); plus the residual G X + X G^+ = Y."""
    H, Ls = li.random_dense(5, 3, seed=21)
    Ls = [4 * L for L in Ls]  # faster decay -> shorter quadrature
    G = ol.no_jump_generator(H, Ls)
    Y = li.random_state(5, seed=6, hermitian=False)
    X1 = ol.lyap_solve(G, Y)
    X2 = ol.lyap_solve_kron(G, Y)
    X3 = ol.lyap_integral(G, Y, t_max=40.0, steps=8000)
    assert np.allclose(ol.S_apply(G, X1), Y, atol=1e-13)
    assert np.allclose(X1, X2, atol=1e-12)
    assert np.allclose(X1, X3, atol=1e-9)
    # shifted form: (S - mu) X = Y
    Xm = ol.lyap_solve(G, Y, mu=0.7)
    assert np.allclose(ol.S_apply(G, Xm) - 0.7 * Xm, Y, atol=1e-13)
    # eigendecomposition route (eq. lyapu_eig_solution)
    R = ol.EigResolvent(G)
    assert np.allclose(R.sinv(Y), X1, atol=1e-12)
    assert np.allclose(R.sinv(Y, 0.7), Xm, atol=1e-12)


def test_hermitian_in_hermitian_out_and_cp():
    """Hermitian Y gives Hermitian X (Section A.1), -S^{-1} and Phi are completely positive
    (eq. lyapunov_solution; Theorem 1), Phi is trace preserving (Appendix lemma)."""
    H, Ls = li.random_dense(4, 2, seed=31)
    G = ol.no_jump_generator(H, Ls)
    Y = li.random_state(4, seed=2)
    X = ol.lyap_solve(G, Y)
    assert np.allclose(X, X.conj().T, atol=1e-14)
    C1 = ol.choi(lambda E: -ol.lyap_solve(G, E), 4)
    C2 = ol.choi(lambda E: ol.phi_apply(G, Ls, E), 4)
    assert np.min(np.linalg.eigvalsh(ol.hermitize(C1))) > -1e-12
    assert np.min(np.linalg.eigvalsh(ol.hermitize(C2))) > -1e-12
    Z = li.random_state(4, seed=3, hermitian=False)
    assert abs(np.trace(ol.phi_apply(G, Ls, Z)) - np.trace(Z)) < 1e-13


def test_phi_spectrum_in_unit_disk_and_fixed_point():
    """Theorem 1: Phi is CPTP with spectrum in the closed unit disk, 1 simple; its fixed point
    xi_inf = K rho_inf and rho_inf = -S^{-1} xi_inf / Tr(.)."""
    H, Ls = li.random_dense(5, 3, seed=41)
    G = ol.no_jump_generator(H, Ls)
    P = ol.superop_of_map(lambda X: ol.phi_apply(G, Ls, X), 5)
    ev = np.linalg.eigvals(P)
    assert np.max(np.abs(ev)) < 1 + 1e-12
    assert np.sum(np.abs(ev - 1) < 1e-8) == 1
    rho = ol.steady_state_dense(H, Ls)
    xi = ol.K_apply(Ls, rho)
    assert np.allclose(ol.phi_apply(G, Ls, xi), xi, atol=1e-13)
    back = -ol.lyap_solve(G, xi)
    assert np.allclose(back / np.trace(back), rho, atol=1e-12)


def test_sherman_morrison_exact():
    """eq. (ShermanMorr): Precond(X, lam, c) is exactly ((lam - S) - c |I><I|)^{-1} X."""
    H, Ls = li.random_dense(4, 2, seed=51)
    G = ol.no_jump_generator(H, Ls)
    X = li.random_state(4, seed=7, hermitian=False)
    for lam, c in [(0.0, 1.0), (0.3, 1.0), (0.0, 2.5)]:
        Z = ol.precond_apply(G, X, lam, c)
        back = lam * Z - ol.S_apply(G, Z) - c * np.trace(Z) * np.eye(4)
        assert np.allclose(back, X, atol=1e-12)


def test_deflation_moves_zero_to_eta_n():
    """Section 4.2: L~_eta keeps every nonzero eigenvalue and sends 0 to eta n."""
    H, Ls = li.random_dense(4, 2, seed=61)
    n = 4
    ev = np.sort_complex(ol.spectrum_dense(H, Ls))
    eta = 0.7
    M = ol.superop_dense(H, Ls)
    vI = ol.vec(np.eye(n))
    ev2 = np.linalg.eigvals(M + eta * np.outer(vI, vI.conj()))
    j0 = np.argmin(np.abs(ev))
    assert np.min(np.abs(ev2 - eta * n)) < 1e-10
    rest = np.delete(ev, j0)
    for e in rest:
        assert np.min(np.abs(ev2 - e)) < 1e-9


def test_contraction_theorem():
    """Theorem 2: ||K R^S_lambda|| = ||(R^S_lambda)*(sum L^+L)||_inf < 1 for lambda > 0, and = 1
    at lambda = 0 (Remark "Loss of the contraction at zero shift")."""
    H, Ls = li.random_dense(5, 2, seed=71)
    G = ol.no_jump_generator(H, Ls)
    n = 5
    KR = ol.superop_of_map(lambda X: ol.K_apply(Ls, ol.resolvent_S(G, X, 0.0)), n)
    # adjoint applied to I, unvec back
    for lam in [0.0, 0.1, 1.0]:
        KRl = ol.superop_of_map(lambda X: ol.K_apply(Ls, ol.resolvent_S(G, X, lam)), n)
        dual_I = ol.unvec(KRl.conj().T @ ol.vec(np.eye(n)), n)
        norm = np.max(np.linalg.eigvalsh(ol.hermitize(dual_I)))
        if lam == 0.0:
            assert abs(norm - 1) < 1e-12
        else:
            assert norm < 1 - 1e-6
    del KR


def test_resolvent_series():
    """Corollary (Resolvent of the Lindbladian): R^L_lambda = R^S_lambda sum_k (K R^S_lambda)^k, lambda > 0."""
    H, Ls = li.random_dense(4, 2, seed=81)
    G = ol.no_jump_generator(H, Ls)
    lam = 2.0
    n = 4
    b = li.random_state(n, seed=3, hermitian=False)
    term = b.copy()
    acc = np.zeros_like(b)
    for _ in range(400):
        acc = acc + term
        term = ol.K_apply(Ls, ol.resolvent_S(G, term, lam))
    series = ol.resolvent_S(G, acc, lam)
    M = ol.superop_dense(H, Ls)
    exact = ol.unvec(np.linalg.solve(lam * np.eye(n * n) - M, ol.vec(b)), n)
    assert np.allclose(series, exact, atol=1e-10)


def test_dephasing_closed_form():
    """Linear cavity with dephasing: <N> = eps^2 Gamma / (kappa (Delta^2 + Gamma^2/4)),
    Gamma = kappa + gamma (closed Heisenberg equations for <a> and <a^dag a>)."""
    D, e, k, gm = 0.5, 1.0, 1.0, 0.05
    H, Ls = li.kerr_cavity(40, Delta=D, eps=e, K=0.0, kappa=k, gamma_dephasing=gm)
    rho = ol.steady_state_dense(H, Ls)
    a = li.destroy(40)
    N = a.conj().T @ a
    Gm = k + gm
    ref = e ** 2 * Gm / (k * (D ** 2 + Gm ** 2 / 4))
    assert abs(np.trace(N @ rho).real - ref) < 1e-11


def test_coupled_cavities_product_coherent():
    """Two coupled linear cavities (K = 0, gamma = 0): the steady state is a product of coherent
    states with (i D1 + k/2) b1 + i g b2 = -i eps, (i D2 + k/2) b2 + i g b1 = 0."""
    m = 8
    D1, D2, g, eps, k = 0.3, -0.2, 0.4, 0.3, 1.0
    H, Ls = li.coupled_kerr(m, Delta=(D1, D2), K=(0.0, 0.0), g=g, eps=eps, kappa=k, gamma=0.0)
    A = np.array([[1j * D1 + k / 2, 1j * g], [1j * g, 1j * D2 + k / 2]])
    b1, b2 = np.linalg.solve(A, np.array([-1j * eps, 0.0]))
    ref = np.kron(coherent(m, b1), coherent(m, b2))
    r = ol.lindblad_apply(H, Ls[:2], ref)
    assert ol.max_norm(r) < 1e-5  # truncation at 8 levels per mode
    rho = ol.steady_state_dense(H, Ls[:2])
    assert ol.trace_distance(rho, ref) < 1e-4


def test_phi_arnoldi_matches_dense():
    """Algorithm "Steady state as the fixed point of Phi" (plain) against the dense null vector."""
    H, Ls = li.random_dense(20, 8, seed=0)
    rho_d = ol.steady_state_dense(H, Ls)
    rho_a, info = ok.steady_state_phi(H, Ls, tol=1e-12, m=20, return_info=True)
    assert ol.trace_distance(rho_a, rho_d) < 1e-11
    assert info["resid"] < 1e-12
    # Kerr cavity (the 32-level workload)
    H, Ls, _ = li.workload("kerr32")
    rho_d = ol.steady_state_dense(H, Ls)
    rho_a = ok.steady_state_phi(H, Ls, tol=1e-11, m=30)
    assert ol.trace_distance(rho_a, rho_d) < 1e-10


def test_gmres_deflated_steady_state():
    """Algorithm "Steady state via preconditioned GMRES" reaches the dense steady state."""
    H, Ls = li.random_dense(10, 3, seed=5)
    n = 10
    G = ol.no_jump_generator(H, Ls)
    I = np.eye(n, dtype=complex)
    W = ol.resolvent_S(G, I, 0.0)

    def P(X):
        return ol.precond_apply(G, X, 0.0, 1.0, W)

    def A(X):
        return -ol.deflated_apply(H, Ls, X, 1.0)

    rho = ok.gmres(A, -I, P, m=20, atol=1e-13)
    rho = ol.hermitize(rho) / np.trace(rho).real
    assert ol.trace_distance(rho, ol.steady_state_dense(H, Ls)) < 1e-11


def test_low_spectrum_matches_dense():
    """Algorithm "Low-lying spectrum via shift-invert Arnoldi" (plain) against dense eig."""
    H, Ls = li.random_dense(7, 3, seed=2)
    ref = ol.low_spectrum_dense(H, Ls, 4)
    lam, vecs = ok.low_spectrum(H, Ls, 5)  # one extra: a conjugate pair may straddle the cut
    for e in ref:
        assert np.min(np.abs(lam - e)) < 1e-9
    for l, v in zip(lam, vecs):
        assert ok.eigen_residual(H, Ls, l, v) < 1e-8


def test_gradient_three_routes():
    """Remark "Differentiating the steady state": the adjoint gradients equal the dense forward
    sensitivities and central finite differences."""
    H, Ls = li.random_dense(4, 2, seed=13)
    O = li.random_observable(4, seed=1)
    J, gH_f, gL_f = og.grad_forward_dense(H, Ls, O)
    J2, gH_a, gL_a, mu = og.grad_adjoint(H, Ls, O)
    assert abs(J - J2) < 1e-14
    assert np.allclose(gH_a, gH_f, atol=1e-10)
    for a, b in zip(gL_a, gL_f):
        assert np.allclose(a, b, atol=1e-10)
    dirs = og.random_directions(4, 2, 8)
    Jof = lambda H_, Ls_: og.expectation(O, ol.steady_state_dense(H_, Ls_))  # noqa: E731
    fd = og.grad_fd(Jof, H, Ls, dirs)
    ad = np.array([og.directional(gH_a, gL_a, dH, dL) for dH, dL in dirs])
    assert np.linalg.norm(ad - fd) / np.linalg.norm(fd) < 1e-7


def test_gradient_dephasing_closed_form():
    """d<N>/d(Delta, eps, kappa, gamma) from the adjoint gradients (chain rule through
    H = Delta N + eps(a + a^dag), L1 = sqrt(kappa) a, L2 = sqrt(gamma) N) against the
    derivatives of the closed form <N> = eps^2 Gamma/(kappa(Delta^2 + Gamma^2/4))."""
    D, e, k, gm = 0.5, 1.0, 1.0, 0.05
    n = 30
    H, Ls = li.kerr_cavity(n, Delta=D, eps=e, K=0.0, kappa=k, gamma_dephasing=gm)
    a = li.destroy(n)
    N = a.conj().T @ a
    J, gH, gL, _ = og.grad_adjoint(H, Ls, N)

    def f(D, e, k, gm):
        Gm = k + gm
        return e ** 2 * Gm / (k * (D ** 2 + Gm ** 2 / 4))

    h = 1e-6
    ref = [(f(D + h, e, k, gm) - f(D - h, e, k, gm)) / (2 * h),
           (f(D, e + h, k, gm) - f(D, e - h, k, gm)) / (2 * h),
           (f(D, e, k + h, gm) - f(D, e, k - h, gm)) / (2 * h),
           (f(D, e, k, gm + h) - f(D, e, k, gm - h)) / (2 * h)]
    zero = np.zeros_like(H)
    got = [og.directional(gH, gL, N, [zero, zero]),
           og.directional(gH, gL, a + a.conj().T, [zero, zero]),
           og.directional(gH, gL, zero, [a / (2 * np.sqrt(k)), zero]),
           og.directional(gH, gL, zero, [zero, N / (2 * np.sqrt(gm))])]
    assert np.allclose(got, ref, rtol=1e-7, atol=1e-9)


# --------------------------------------------------------------------------------------
# planted mistakes: each must be caught by one of the pins above
# --------------------------------------------------------------------------------------

def _lindblad_wrong_commutator(H, Ls, rho):
    out = +1j * (H @ rho - rho @ H)  # planted: sign of the Hamiltonian term
    for L in Ls:
        LdL = L.conj().T @ L
        out = out + L @ rho @ L.conj().T - 0.5 * (LdL @ rho + rho @ LdL)
    return out


def _lindblad_transposed_jump(H, Ls, rho):
    out = -1j * (H @ rho - rho @ H)
    for L in Ls:
        LdL = L.conj().T @ L
        out = out + L.conj().T @ rho @ L - 0.5 * (LdL @ rho + rho @ LdL)  # planted: L^+ rho L
    return out


def _lindblad_dropped_half(H, Ls, rho):
    out = -1j * (H @ rho - rho @ H)
    for L in Ls:
        LdL = L.conj().T @ L
        out = out + L @ rho @ L.conj().T - (LdL @ rho + rho @ LdL)  # planted: dropped 1/2
    return out


@pytest.mark.parametrize("bad", [_lindblad_wrong_commutator, _lindblad_transposed_jump, _lindblad_dropped_half])
def test_planted_lindblad_mistakes_are_caught(bad):
    g = read_golden("kerr_linear_coherent.txt")
    beta = complex(g["beta_re"], g["beta_im"])
    H, Ls = li.kerr_cavity(32, K=0.0)
    ref = coherent(32, beta)
    caught = ol.max_norm(bad(H, Ls, ref)) > 1e-6
    X = li.random_state(6, seed=1, hermitian=False)
    H6, L6 = li.random_dense(6, 2, seed=1)
    caught = caught or abs(np.trace(bad(H6, L6, X))) > 1e-8
    assert caught


def test_planted_phi_sign_is_caught():
    """Phi with the wrong sign (+K S^{-1}) fails the three-level golden spectrum."""
    g = read_golden("three_level_cyclic.txt")
    H, Ls = li.three_level_cyclic()
    G = ol.no_jump_generator(H, Ls)
    P = ol.superop_of_map(lambda X: ol.K_apply(Ls, ol.lyap_solve(G, X)), 3)
    ev = np.linalg.eigvals(P)
    assert np.min(np.abs(ev - 1.0)) > 1e-3


def test_planted_resolvent_shift_is_caught():
    """A resolvent with G - lambda (instead of G - lambda/2) fails the two-level footnote."""
    g = read_golden("two_level_footnote.txt")
    H, Ls = li.two_level_decay(g["gamma"])
    G = ol.no_jump_generator(H, Ls)
    rho = li.random_state(2, seed=9)
    lam = g["lambda"]
    wrong = -ol.lyap_solve(G - 0.5 * lam * np.eye(2), ol.K_apply(Ls, rho), lam)
    assert abs(wrong[0, 0] - g["RK_coefficient"] * rho[1, 1]) > 1e-3


# --------------------------------------------------------------------------------------
# resolvent and implicit Euler (oracle.dynamics)
# --------------------------------------------------------------------------------------
def test_resolvent_three_routes():
    """(lambda - L)^{-1} B three ways: dense LU of the superoperator, the series of the resolvent
    corollary (Lyapunov solves only), and right-preconditioned GMRES; lambda spans the three
    shifts of the resolvent benchmark (lambda_max * 10^{0,-1,-2}, lambda_max = spectral radius)."""
    for H, Ls in [li.random_dense(6, 2, seed=5), li.kerr_cavity(8)]:
        n = H.shape[0]
        lam_max = float(np.max(np.abs(ol.spectrum_dense(H, Ls))))
        B = li.random_state(n, seed=9, hermitian=False)
        for lam in [lam_max, lam_max / 10, lam_max / 100]:
            X = od.resolvent_dense(H, Ls, lam, B)
            res = lam * X - ol.lindblad_apply(H, Ls, X) - B
            assert np.max(np.abs(res)) < 1e-11 * max(1, np.max(np.abs(B)))
            terms = int(np.ceil(np.log(1e-15) / np.log(od.contraction_norm(H, Ls, lam)))) + 5
            S = od.resolvent_series(H, Ls, lam, B, terms=min(terms, 20000))
            assert np.max(np.abs(S - X)) < 1e-9 * np.max(np.abs(X))
            Y = od.resolvent_gmres(H, Ls, lam, B, tol=1e-13)
            assert np.max(np.abs(Y - X)) < 1e-9 * np.max(np.abs(X))


def test_contraction_norm_footnote_and_brute_force():
    """Left/right preconditioning footnote: n = 2, H = 0, L = sqrt(gamma)|0><1| gives
    ||K R^S_lambda|| = gamma / (gamma + lambda); and the CP-map norm formula against the dual map
    built column by column on a random system."""
    g = 0.7
    H, Ls = li.two_level_decay(g)
    for lam in [0.01, 0.3, 2.0]:
        assert abs(od.contraction_norm(H, Ls, lam) - g / (g + lam)) < 1e-13
    H, Ls = li.random_dense(5, 3, seed=17)
    G = ol.no_jump_generator(H, Ls)
    for lam in [0.05, 1.0]:
        KR = ol.superop_of_map(lambda X: ol.K_apply(Ls, ol.resolvent_S(G, X, lam)), 5)
        dual_I = ol.hermitize(ol.unvec(KR.conj().T @ ol.vec(np.eye(5)), 5))
        assert abs(od.contraction_norm(H, Ls, lam) - np.max(np.linalg.eigvalsh(dual_I))) < 1e-12
        assert od.contraction_norm(H, Ls, lam) < 1


def ie_two_level_closed_form(g, dt, k, rho0):
    """Implicit Euler for L = sqrt(g)|0><1|, H = 0: rho_11 -> rho_11 / (1 + g dt),
    rho_01 -> rho_01 / (1 + g dt / 2), trace kept."""
    r = rho0.astype(np.complex128).copy()
    p1 = r[1, 1] / (1 + g * dt) ** k
    c = r[0, 1] / (1 + g * dt / 2) ** k
    out = np.array([[1 - p1, c], [np.conj(c), p1]], dtype=np.complex128)
    return out


def test_implicit_euler_two_level_closed_form():
    """eq. resolvent (implicit solver section) on the two-level decay, against the per-step
    closed form, and its first-order agreement with exp(t L) (scipy.linalg.expm)."""
    import scipy.linalg as sl
    g, dt = 0.8, 0.25
    H, Ls = li.two_level_decay(g)
    plus = 0.5 * np.array([[1, 1], [1, 1]], dtype=np.complex128)
    for rho0 in [np.diag([0.0, 1.0]).astype(np.complex128), plus]:
        states = od.implicit_euler_dense(H, Ls, rho0, dt, 6)
        for k, r in enumerate(states, 1):
            assert np.allclose(r, ie_two_level_closed_form(g, dt, k, rho0), atol=1e-14)
    H, Ls = li.kerr_cavity(6)
    rho0 = li.random_state(6, seed=4)
    t = 0.5
    ex = ol.unvec(sl.expm(t * ol.superop_dense(H, Ls)) @ ol.vec(rho0), 6)
    errs = []
    for steps in [50, 100, 200]:
        errs.append(np.max(np.abs(od.implicit_euler_dense(H, Ls, rho0, t / steps, steps)[-1] - ex)))
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8  # first order in dt
    assert errs[2] < 1e-2


def test_implicit_euler_trace_hermiticity_and_steady_limit():
    """Each step keeps the trace and Hermiticity (L is trace-annihilating and Hermiticity-
    preserving); long steps converge to the steady state (the fixed point of (I - dt L)^{-1})."""
    H, Ls, _ = li.workload("kerr32")
    H, Ls = H[:12, :12], [L[:12, :12] for L in Ls]
    rho0 = li.random_state(12, seed=6)
    states = od.implicit_euler_dense(H, Ls, rho0, 0.3, 5)
    for r in states:
        assert abs(np.trace(r) - np.trace(rho0)) < 1e-13
        assert np.max(np.abs(r - r.conj().T)) < 1e-13
    far = od.implicit_euler_dense(H, Ls, rho0, 50.0, 60)[-1]
    assert ol.trace_distance(far / np.trace(far), ol.steady_state_dense(H, Ls)) < 1e-10


def test_planted_explicit_euler_sign_is_caught():
    """Plant (I + dt L) instead of (I - dt L) in a copy of the implicit Euler step: the two-level
    closed form catches it."""
    g, dt = 0.8, 0.25
    H, Ls = li.two_level_decay(g)
    rho0 = np.diag([0.0, 1.0]).astype(np.complex128)
    A = np.eye(4, dtype=np.complex128) + dt * ol.superop_dense(H, Ls)
    bad = ol.unvec(np.linalg.solve(A, ol.vec(rho0)), 2)
    assert not np.allclose(bad, ie_two_level_closed_form(g, dt, 1, rho0), atol=1e-6)


# --------------------------------------------------------------------------------------
# gauge-shifted split (Remark "Non-uniqueness of the decomposition")
# --------------------------------------------------------------------------------------
def test_gauge_shift_keeps_the_lindbladian():
    """Every shift c gives an admissible split of the same L (the remark's direct computation):
    the dense superoperators agree, and G changes by -B - sum|c_j|^2/2 with B = sum conj(c_j) L_j."""
    H, Ls = li.random_dense(5, 3, seed=23)
    c = [0.3 - 0.2j, -1.1 + 0.4j, 0.05j]
    Ht, Lt = ol.gauge_shift(H, Ls, c)
    assert np.allclose(Ht, Ht.conj().T, atol=1e-15)
    assert np.allclose(ol.superop_dense(Ht, Lt), ol.superop_dense(H, Ls), atol=1e-13)
    G, Gt = ol.no_jump_generator(H, Ls), ol.no_jump_generator(Ht, Lt)
    B = sum(np.conj(cj) * L for L, cj in zip(Ls, c))
    assert np.allclose(Gt, G - B - 0.5 * sum(abs(cj) ** 2 for cj in c) * np.eye(5), atol=1e-13)


def test_gauge_three_level_golden():
    """Conclusion: on the three-level example, c = (1, 0, 0) leaves 1 simple in the shifted Phi and
    brings every other eigenvalue to modulus <= sqrt(3/8), the pair becoming 1/2 +- i/(2 sqrt 2)."""
    g = read_golden("three_level_gauge.txt")
    H, Ls = li.three_level_cyclic()
    c = np.array(g["gauge_re"]) + 1j * np.array(g["gauge_im"])
    Ht, Lt = ol.gauge_shift(H, Ls, c)
    Gt = ol.no_jump_generator(Ht, Lt)
    P = ol.superop_of_map(lambda X: ol.phi_apply(Gt, Lt, X), 3)
    ev = np.linalg.eigvals(P)
    assert np.sum(np.abs(ev - 1) < 1e-9) == 1
    others = ev[np.abs(ev - 1) >= 1e-9]
    assert np.max(np.abs(others)) <= g["bound"] + 1e-12
    for re, im in zip(g["pair_re"], g["pair_im"]):
        assert np.min(np.abs(ev - (re + 1j * im))) < 1e-12
    assert abs(g["bound"] - np.sqrt(3 / 8)) < 1e-15


def test_gauge_repairs_singular_split():
    """Conclusion: the shifted S is singular only if some psi has L_j psi = -c_j psi for all j; the
    two-level decay (Theorem 1, first case: S singular at c = 0) is repaired by any c != 0 and its
    steady state |0><0| comes out of the shifted Phi-Arnoldi."""
    H, Ls = li.two_level_decay(1.0)
    G = ol.no_jump_generator(H, Ls)
    assert np.min(np.abs(np.linalg.eigvals(G).real)) < 1e-14
    Ht, Lt = ol.gauge_shift(H, Ls, [0.5])
    Gt = ol.no_jump_generator(Ht, Lt)
    assert np.min(np.abs(np.linalg.eigvals(Gt).real)) > 0.1
    rho = ok.steady_state_phi(Ht, Lt, tol=1e-12, m=3)
    assert np.allclose(rho, np.diag([1.0, 0.0]), atol=1e-12)


def test_planted_gauge_sign_is_caught():
    """Plant the wrong sign of the Hamiltonian correction in a copy of gauge_shift."""
    H, Ls = li.random_dense(4, 2, seed=29)
    c = [0.4 + 0.1j, -0.3j]
    n = 4
    Lt = [L + cj * np.eye(n) for L, cj in zip(Ls, c)]
    bad_H = H - sum((np.conj(cj) * L - cj * L.conj().T) for L, cj in zip(Lt, c)) / 2j
    assert not np.allclose(ol.superop_dense(bad_H, Lt), ol.superop_dense(H, Ls), atol=1e-6)


def test_adjoint_state_gmres_matches_dense():
    """The matrix-free adjoint state (right-preconditioned GMRES on the deflated adjoint system)
    equals the dense solve of the same system, and the gradients built from it equal the dense
    forward sensitivities (Remark "Differentiating the steady state")."""
    for n, d, seed in [(12, 2, 7), (16, 3, 8)]:
        H, Ls = li.random_dense(n, d, seed)
        O = li.random_observable(n, seed=1)
        rho = ol.steady_state_dense(H, Ls)
        mu_d = og.adjoint_state_dense(H, Ls, O, rho)
        mu_g = og.adjoint_state_gmres(H, Ls, O, rho)
        assert np.max(np.abs(mu_g - mu_d)) <= 1e-11 * np.max(np.abs(mu_d))
        _, gH, gL = og.grad_forward_dense(H, Ls, O)
        gH2, gL2 = og.grad_from_adjoint(Ls, rho, mu_g)
        assert np.max(np.abs(gH2 - gH)) <= 1e-10 * np.max(np.abs(gH))
        for a, b in zip(gL2, gL):
            assert np.max(np.abs(a - b)) <= 1e-10 * np.max(np.abs(b))


def test_coupled_kerr_truncation_converged():
    """The two-cavity workload is truncation-converged well before 20 levels per mode (the reference
    the 40 x 40 GPU state is compared with): the oracle's Algorithm 4 states at 16 and 20 levels per
    mode, zero-padded, agree to 1e-10 in trace distance, and both are certified by their residuals."""
    def embed(rho, ms, mb):
        R = rho.reshape(ms, ms, ms, ms)
        out = np.zeros((mb, mb, mb, mb), dtype=np.complex128)
        out[:ms, :ms, :ms, :ms] = R
        return out.reshape(mb * mb, mb * mb)
    st = {}
    for ms in (16, 20):
        H, Ls = li.coupled_kerr(ms)
        rho, info = ok.steady_state_phi(H, Ls, tol=1e-12, return_info=True)
        assert info["resid"] <= 1e-12
        st[ms] = rho
    assert ol.trace_distance(embed(st[16], 16, 20), st[20]) < 1e-10
