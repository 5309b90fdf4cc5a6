"""Failure paths and determinism of the steady-state driver (all forced from the host; no kernel is
made to fail).

* Algorithm "Steady state as the fixed point of Phi" returns its running best iterate: with the
  restart cap or the time limit hit, lind_steady_state returns LIND_ENOCONV and still writes the
  best state and its residual; that state resumes the solve through rho0 (a checkpoint).
* lind_create refuses non-finite H or L_j with LIND_EINVAL.
* The reductions use no atomics: two FP64 (or BF16x3) solves, on one context or on two contexts
  built from the same input, agree bit for bit.
* An Arnoldi breakdown (the Krylov space invariant after one step) ends the cycle with the exact
  fixed point instead of a division by the zero norm.
"""
import numpy as np
import pytest
import torch

import lind_inputs as li
from oracle import lindblad as ol
from paper_2608_30860_amd import Lindblad
from paper_2608_30860_amd.lindx import LIND_EINVAL, LIND_ENOCONV, LIND_OK, LindError

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _dev(H, Ls):
    return torch.from_numpy(H).to(DEV), torch.from_numpy(np.stack(Ls)).to(DEV)


def _colsum(R):
    return float(np.sum(np.linalg.norm(R, axis=0)))


def test_enoconv_writes_best_iterate_and_resumes():
    H, Ls = li.random_dense(48, 4, 3)
    Ht, Lt = _dev(H, Ls)
    m = Lindblad(Ht, Lt, m=6, max_restarts=1, refine_max=0)
    r = m.steady_state(1e-12, raise_on_noconv=False)
    print("first call", r.info, flush=True)
    assert r.info["status"] == LIND_ENOCONV
    rho = r.rho.cpu().numpy()
    # the written iterate is the state the residual belongs to: Hermitian, trace 1, and its FP64
    # residual bound recomputed on the host is the reported one
    assert np.max(np.abs(rho - rho.conj().T)) == 0.0
    assert abs(np.trace(rho) - 1) < 1e-13
    cs = _colsum(ol.lindblad_apply(H, Ls, rho))
    assert abs(cs - r.info["resid_trace"]) <= 1e-8 * cs + 1e-15
    assert r.info["resid_trace"] > 1e-12
    # resume from the best iterate, one restart per call, until the tolerance is met
    state, calls = r.rho, 0
    while r.info["status"] == LIND_ENOCONV and calls < 60:
        r = m.steady_state(1e-12, rho0=state, raise_on_noconv=False)
        state = r.rho
        calls += 1
    print("resumed calls", calls, r.info, flush=True)
    assert r.info["status"] == LIND_OK
    ref = ol.steady_state_dense(H, Ls)
    assert ol.trace_distance(r.rho.cpu().numpy(), ref) < 1e-10
    m.close()


def test_time_limit_returns_best_iterate():
    H, Ls = li.random_dense(64, 4, 4)
    Ht, Lt = _dev(H, Ls)
    m = Lindblad(Ht, Lt, m=30, time_limit_s=1e-9)
    r = m.steady_state(1e-14, raise_on_noconv=False)
    assert r.info["status"] == LIND_ENOCONV
    rho = r.rho.cpu().numpy()
    assert np.all(np.isfinite(rho)) and abs(np.trace(rho) - 1) < 1e-13
    cs = _colsum(ol.lindblad_apply(H, Ls, rho))
    assert abs(cs - r.info["resid_trace"]) <= 1e-8 * cs + 1e-15
    m.close()


@pytest.mark.parametrize("where", ["H", "L"])
def test_nonfinite_input_is_einval(where):
    H, Ls = li.random_dense(32, 2, 5)
    if where == "H":
        H = H.copy()
        H[3, 5] = np.nan
    else:
        Ls = [L.copy() for L in Ls]
        Ls[1][7, 2] = np.inf
    Ht, Lt = _dev(H, Ls)
    with pytest.raises(LindError) as e:
        Lindblad(Ht, Lt)
    assert e.value.code == LIND_EINVAL
    assert "non-finite" in str(e.value)


@pytest.mark.parametrize("prec,n,d", [("fp64", 256, 4), ("bf16x3", 256, 4), ("fp64", 2048, 8)])
def test_solves_are_bitwise_deterministic(prec, n, d):
    H, Ls = li.random_dense(n, d, 0)
    Ht, Lt = _dev(H, Ls)
    a = Lindblad(Ht, Lt, prec=prec)
    r1 = a.steady_state(1e-10 if prec == "fp64" else 1e-8)
    r2 = a.steady_state(1e-10 if prec == "fp64" else 1e-8)
    b = Lindblad(Ht, Lt, prec=prec)
    r3 = b.steady_state(1e-10 if prec == "fp64" else 1e-8)
    print(prec, n, d, r1.info["resid_trace"], r3.info["resid_trace"], flush=True)
    assert torch.equal(r1.rho, r2.rho)
    assert torch.equal(r1.rho, r3.rho)
    assert r1.info["n_phi"] == r2.info["n_phi"] == r3.info["n_phi"]
    for which in ["G", "T", "Z", "U", "V", "s"]:  # the factorisation itself
        assert torch.equal(a.factor(which), b.factor(which)), which
    a.close()
    b.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3"])
def test_invariant_krylov_space_at_the_first_step(prec):
    """With L_1 = I and H diagonal every diagonal state is steady and Phi is the identity on
    diagonal matrices, so the first Krylov vector (the start I/n turned into -S(I/n)) spans an
    invariant space: the Arnoldi step's norm is zero (up to rounding) and the driver must stop
    there with the Ritz value 1 and return I/n, without dividing by the zero norm."""
    n = 4
    H = np.diag([0.3, -0.1, 0.7, 0.2]).astype(np.complex128)
    Ls = [np.eye(n, dtype=np.complex128)]
    Ht, Lt = _dev(H, Ls)
    m = Lindblad(Ht, Lt, prec=prec, m=8)
    r = m.steady_state(1e-12)
    print(prec, r.info, flush=True)
    rho = r.rho.cpu().numpy()
    assert r.info["status"] == LIND_OK
    assert np.all(np.isfinite(rho))
    assert ol.trace_distance(rho, np.eye(n) / n) <= 1e-12
    assert r.info["n_phi"] <= 3
    m.close()
