"""GPU parity of the steady state by preconditioned GMRES (method "gmres", Algorithm "Steady state via
preconditioned GMRES") and of the gauge-shifted split (Remark "Non-uniqueness of the decomposition")
against the CPU oracle.

Tolerances as for the Phi-Arnoldi steady state: ||L rho||_1 bound <= tol, trace distance <= 1e-8 to
the oracle; the shifted Phi's spectrum on the three-level example to 1e-12 (the paper prints it).
"""
import os

import numpy as np
import pytest

import lind_inputs as li
from oracle import gradient as og
from oracle import krylov as ok
from oracle import lindblad as ol

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
GOLD = os.path.join(os.path.dirname(__file__), "golden")


def T(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex128)).to("cuda:0")


def N(t):
    return t.detach().cpu().numpy()


def make(H, Ls, **kw):
    from paper_2608_30860_amd import Lindblad
    return Lindblad(T(H), T(np.stack(Ls)), **kw)


def read_golden(name):
    vals = {}
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split("=")
            nums = [float(x) for x in v.split()]
            vals[k.strip()] = nums if len(nums) > 1 else nums[0]
    return vals


# ------------------------------------------------------------------ GMRES steady state -----------
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("bf16x3", 1e-10)])
@pytest.mark.parametrize("n,d", [(24, 8), (96, 3)])
def test_gmres_method_random(prec, tol, n, d):
    print(f"[case] gmres steady random n={n} d={d} {prec}", flush=True)
    H, Ls = li.random_dense(n, d, 0)
    m = make(H, Ls, prec=prec, method="gmres")
    r = m.steady_state(tol)
    rho = N(r.rho)
    print("info", r.info)
    assert ol.trace_norm(ol.lindblad_apply(H, Ls, rho)) < tol
    ref = ol.steady_state_dense(H, Ls) if n <= 24 else ok.steady_state_phi(H, Ls, tol=1e-13)
    assert ol.trace_distance(rho, ref) < 1e-8
    m.close()


def test_gmres_method_kerr32_and_three_level():
    H, Ls, _ = li.workload("kerr32")
    m = make(H, Ls, method="gmres")
    rho = N(m.steady_state(1e-10).rho)
    assert ol.trace_distance(rho, ol.steady_state_dense(H, Ls)) < 1e-8
    m.close()
    H, Ls = li.three_level_cyclic()
    m = make(H, Ls, method="gmres", m=8)
    assert np.allclose(N(m.steady_state(1e-12).rho), np.eye(3) / 3, atol=1e-12)
    m.close()


def test_gmres_method_random2048():
    """Full size, BF16x3 preconditioner, FP64 operator: the same state as Phi-Arnoldi."""
    print("[case] gmres steady random n=2048", flush=True)
    H, Ls, _ = li.workload("random2048")
    m = make(H, Ls, prec="bf16x3", method="gmres")
    r = m.steady_state(1e-8)
    print("info", r.info)
    m2 = make(H, Ls, prec="bf16x3")
    r2 = m2.steady_state(1e-8)
    a, b = r.rho, r2.rho
    ev = torch.linalg.eigvalsh(0.5 * ((a - b) + (a - b).conj().T))
    assert float(0.5 * ev.abs().sum()) < 1e-8
    assert r.info["resid_trace"] <= 1e-8
    m.close()
    m2.close()


# ------------------------------------------------------------------ gauge-shifted split ----------
def test_gauge_keeps_lindbladian_state_and_gradients():
    H, Ls = li.random_dense(24, 3, 5)
    c = [0.4 - 0.3j, -0.8 + 0.1j, 0.25j]
    mg = make(H, Ls, gauge=c)
    m0 = make(H, Ls)
    X = li.random_state(24, seed=3, hermitian=False)
    assert np.max(np.abs(N(mg.apply(T(X))) - ol.lindblad_apply(H, Ls, X))) < 1e-12 * np.max(np.abs(ol.lindblad_apply(H, Ls, X)))
    Ht, Lt = ol.gauge_shift(H, Ls, c)
    assert np.max(np.abs(N(mg.factor("G")) - ol.no_jump_generator(Ht, Lt))) < 1e-13
    rg, r0 = N(mg.steady_state(1e-11).rho), N(m0.steady_state(1e-11).rho)
    assert ol.trace_distance(rg, r0) < 1e-10
    O = li.random_observable(24, seed=1)
    Jg, gHg, gLg, _, _ = mg.steady_grad(T(O), 1e-12)
    J0, gH0, gL0, _, _ = m0.steady_grad(T(O), 1e-12)
    assert abs(Jg - J0) < 1e-11
    num = np.linalg.norm(N(gHg) - N(gH0)) ** 2 + sum(np.linalg.norm(N(a) - N(b)) ** 2 for a, b in zip(gLg, gL0))
    den = np.linalg.norm(N(gH0)) ** 2 + sum(np.linalg.norm(N(b)) ** 2 for b in gL0)
    assert np.sqrt(num / den) < 1e-8
    Jr, gHr, gLr = og.grad_forward_dense(H, Ls, O)
    assert abs(Jg - Jr) < 1e-10
    mg.close()
    m0.close()


def test_gauge_three_level_spectrum_golden():
    """The shifted Phi of the three-level example, assembled from lind_phi on the 9 unit matrices."""
    g = read_golden("three_level_gauge.txt")
    H, Ls = li.three_level_cyclic()
    c = list(np.array(g["gauge_re"]) + 1j * np.array(g["gauge_im"]))
    m = make(H, Ls, gauge=c, m=8)
    P = np.zeros((9, 9), dtype=np.complex128)
    for k in range(9):
        E = np.zeros((3, 3), dtype=np.complex128)
        E[k % 3, k // 3] = 1.0  # column stacking
        P[:, k] = N(m.phi(T(E))).reshape(-1, order="F")
    ev = np.linalg.eigvals(P)
    assert np.sum(np.abs(ev - 1) < 1e-9) == 1
    assert np.max(np.abs(ev[np.abs(ev - 1) >= 1e-9])) <= g["bound"] + 1e-12
    for re, im in zip(g["pair_re"], g["pair_im"]):
        assert np.min(np.abs(ev - (re + 1j * im))) < 1e-12
    assert np.allclose(N(m.steady_state(1e-12).rho), np.eye(3) / 3, atol=1e-12)
    m.close()


def test_gauge_repairs_two_level_decay():
    """Theorem 1, first case (singular S at c = 0, reported as ESINGULAR) becomes solvable."""
    from paper_2608_30860_amd import LindError
    H, Ls = li.two_level_decay(1.0)
    with pytest.raises(LindError):
        make(H, Ls)
    m = make(H, Ls, gauge=[0.5], m=4)
    assert np.allclose(N(m.steady_state(1e-12).rho), np.diag([1.0, 0.0]), atol=1e-12)
    m.close()
