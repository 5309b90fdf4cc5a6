"""Kernel-level GPU tests through include/lind_internal.h: each kernel against a plain NumPy
evaluation of the same operation on the same seeded inputs."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def lib():
    from paper_2608_30860_amd.lindx import load_library
    L = load_library()
    vp, ci, cd, ll = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    L.lindx_gemm.argtypes = [ci, ci, ci, ci, ci, vp, ll, ll, ci, vp, ll, ll, ci, vp, ll, cd, cd, ci, ci, ci, vp]
    L.lindx_schur.argtypes = [vp, vp, ci, ci, vp]
    L.lindx_small_eig.argtypes = [vp, ci, vp, vp, vp]
    L.lindx_trevec.argtypes = [vp, vp, ci, vp]
    L.lindx_ritz_near.argtypes = [vp, ci, cd, cd, vp, ctypes.POINTER(ci), vp]
    L.lindx_triinv.argtypes = [vp, vp, ci, vp]
    L.lindx_trisylv.argtypes = [vp, vp, ci, cd, cd, vp]
    L.lindx_trisylv_blk.argtypes = [vp, vp, ci, cd, cd, cd, ctypes.POINTER(cd), vp]
    L.lindx_p4_test.argtypes = [vp, vp, ci, ci, ci, ci, ci, ci, ci, vp, vp, vp, vp]
    L.lindx_cgs2.argtypes = [vp, ll, ci, vp, ll, vp, vp, ci, vp]
    L.lindx_cgs2_small.argtypes = [vp, ll, ci, vp, ll, vp, vp, vp]
    return L


def T(a, dtype=torch.complex128):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0").to(dtype)


def P(t):
    return ctypes.c_void_p(t.data_ptr())


def crand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def op(X, o):
    return X if o == 0 else X.conj().swapaxes(-1, -2)


@pytest.mark.parametrize("prec,tol", [(0, 1e-13), (1, 2e-5), (2, 3e-4)])
@pytest.mark.parametrize("M,N,K,nb", [(37, 45, 29, 1), (130, 70, 200, 1), (64, 64, 64, 3), (200, 200, 200, 2),
                                      (1, 1, 1, 1), (1024, 1024, 96, 1), (300, 260, 72, 8), (1024, 1024, 64, 4),
                                      (2048, 1040, 96, 1), (1536, 1538, 64, 2), (2050, 1030, 40, 1),
                                      (2047, 1031, 96, 1), (256, 256, 256, 1), (96, 80, 250, 1),
                                      (512, 256, 256, 1)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (2, 0), (0, 2), (2, 2)])
def test_gemm(prec, tol, M, N, K, nb, opA, opB):
    """Complex products against NumPy, relative to the largest entry.  The four large shapes fill
    more than 128 tiles of 128 x 128, where the FP64 and FP32 products run the direct-to-LDS
    kernels: ragged edges in m, n and k, a split-K batch reduction, and an odd shape that the FP32
    one must hand to the register-staged kernel (its 16-byte chunks need even sizes).  Single
    products on at most 128 tiles of 32 x 32 (130 x 70 x 200, 256^3, 96 x 80 x 250, 512 x 256 x 256)
    run with their K split into chunks summed by the reduction (FP64 and FP32)."""
    print(f"[case] gemm prec={prec} {M}x{N}x{K} nb={nb} ops={opA},{opB}", flush=True)
    rng = np.random.default_rng(M * 7 + N + K + nb)
    Ash = (nb, M, K) if opA == 0 else (nb, K, M)
    Bsh = (nb, K, N) if opB == 0 else (nb, N, K)
    A = crand(rng, *Ash)
    B = crand(rng, *Bsh)
    C0 = crand(rng, M, N)
    ref = sum(op(A[b], opA) @ op(B[b], opB) for b in range(nb))
    alpha = 0.5 - 0.25j
    dt = torch.complex128 if prec == 0 else torch.complex64
    for beta in (0, 1):
        for out64 in ((0,) if prec == 0 else (0, 1)):
            At, Bt = T(A, dt), T(B, dt)
            Ct = T(C0, torch.complex128 if (prec == 0 or out64) else torch.complex64)
            lda = Ash[2]
            ldb = Bsh[2]
            rc = lib().lindx_gemm(prec, M, N, K, nb, P(At), lda, Ash[1] * Ash[2], opA, P(Bt), ldb, Bsh[1] * Bsh[2],
                                  opB, P(Ct), N, alpha.real, alpha.imag, beta, out64, 0, None)
            assert rc == 0
            torch.cuda.synchronize()
            got = Ct.cpu().numpy().astype(np.complex128)
            want = alpha * ref + (C0 if beta else 0)
            if prec > 0 and not (prec == 0 or out64):
                want = want  # complex64 output
            err = np.max(np.abs(got - want)) / np.max(np.abs(want))
            assert err < tol, (beta, out64, err)


@pytest.mark.parametrize("M,N,K,nb", [(37, 45, 29, 1), (130, 70, 200, 1), (128, 128, 64, 1), (300, 260, 72, 1),
                                      (1, 1, 1, 1), (256, 384, 1000, 1), (64, 64, 64, 3), (300, 260, 72, 8),
                                      (1024, 1024, 64, 4), (4100, 2050, 40, 1), (2048, 2050, 40, 4)])
@pytest.mark.parametrize("opA,opB", [(0, 0), (2, 0), (0, 2), (2, 2)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_p4_gemm(M, N, K, nb, opA, opB, mode):
    """pre-split BF16 product: planes out (row-major / transposed), split-K partials out, and the
    fused divide; relative to the largest entry, 3e-4 as for the on-the-fly BF16x3 product.  The
    two largest shapes are ragged in m and n over many tiles, one of them split-K."""
    if mode != 2 and nb != 1:
        pytest.skip("batched products only reduce into split-K partials")
    print(f"[case] p4 {M}x{N}x{K} nb={nb} ops={opA},{opB} mode={mode}", flush=True)
    rng = np.random.default_rng(M * 5 + N + 3 * K + nb + 11 * mode)
    Ash = (nb, M, K) if opA == 0 else (nb, K, M)
    Bsh = (nb, K, N) if opB == 0 else (nb, N, K)
    A = crand(rng, *Ash)
    B = crand(rng, *Bsh)
    ref = sum(op(A[b], opA) @ op(B[b], opB) for b in range(nb))
    for div in ((False, True) if mode != 2 else (False,)):
        dr = crand(rng, M) + 3.0 if div else None
        dc = crand(rng, N) + 3.0 if div else None
        want = ref / (dr[:, None] + dc[None, :]) if div else ref
        Ct = T(np.zeros((M, N)))
        At, Bt = T(A), T(B)  # keep the device copies alive across the call
        drt, dct = (T(dr), T(dc)) if div else (None, None)
        rc = lib().lindx_p4_test(P(At), P(Bt), M, N, K, nb, opA, opB, mode,
                                 P(drt) if div else None, P(dct) if div else None, P(Ct), None)
        assert rc == 0
        got = Ct.cpu().numpy()
        err = np.max(np.abs(got - want)) / np.max(np.abs(want))
        assert err < 3e-4, (div, err)


@pytest.mark.parametrize("n,K,nb", [(37, 29, 1), (130, 200, 1), (256, 64, 1), (300, 72, 4), (1, 5, 1), (2048, 96, 1)])
@pytest.mark.parametrize("mode", [0, 1, 2])
def test_p4_gemm_hermitian(n, K, nb, mode):
    """Hermitian products A A^H (summed over batches, and divided by d_m + conj(d_n)) from the upper
    tiles only: against the full product, and exactly Hermitian"""
    if mode != 2 and nb != 1:
        pytest.skip("batched products only reduce into split-K partials")
    print(f"[case] p4 hermitian n={n} K={K} nb={nb} mode={mode}", flush=True)
    rng = np.random.default_rng(n + K + nb + mode)
    A = crand(rng, nb, n, K)
    ref = sum(A[b] @ A[b].conj().T for b in range(nb))
    div = mode != 2
    dr = crand(rng, n) + 3.0
    if div:
        ref = ref / (dr[:, None] + dr.conj()[None, :])
    At = T(A)
    drt, dct = T(dr), T(dr.conj())
    Ct = T(np.zeros((n, n)))
    rc = lib().lindx_p4_test(P(At), P(At), n, n, K, nb, 0, 2, mode + 4, P(drt) if div else None,
                             P(dct) if div else None, P(Ct), None)
    assert rc == 0
    got = Ct.cpu().numpy()
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 3e-4
    if mode == 2:
        assert np.array_equal(got, got.conj().T)


@pytest.mark.parametrize("n,K,nb", [(37, 29, 1), (130, 70, 1), (300, 72, 8), (1024, 64, 4), (257, 33, 3)])
@pytest.mark.parametrize("beta", [0, 1])
def test_gemm_fp64_hermitian(n, K, nb, beta):
    """FP64 product with a Hermitian result (sum_b A_b A_b^H, real alpha, Hermitian C for beta) from
    the upper tiles only, against NumPy; exactly Hermitian when beta = 0"""
    print(f"[case] gemm64 hermitian n={n} K={K} nb={nb} beta={beta}", flush=True)
    rng = np.random.default_rng(n + K + nb)
    A = crand(rng, nb, n, K)
    C0 = crand(rng, n, n)
    C0 = C0 + C0.conj().T
    alpha = -0.75
    ref = alpha * sum(A[b] @ A[b].conj().T for b in range(nb)) + (C0 if beta else 0)
    At, Ct = T(A), T(C0)
    rc = lib().lindx_gemm(0, n, n, K, nb, P(At), K, n * K, 0, P(At), K, n * K, 2, P(Ct), n, alpha, 0.0, beta, 0, 1,
                          None)
    assert rc == 0
    got = Ct.cpu().numpy()
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-13
    if not beta:
        assert np.max(np.abs(got - got.conj().T)) <= 1e-14 * np.max(np.abs(got))


@pytest.mark.parametrize("n", [3, 37, 130, 257])
def test_hessenberg_and_schur(n):
    print(f"[case] schur n={n}", flush=True)
    rng = np.random.default_rng(n)
    G = crand(rng, n, n) / np.sqrt(n)
    for stop in (1, 0):
        A = T(G)
        Z = T(np.zeros((n, n)))
        rc = lib().lindx_schur(P(A), P(Z), n, stop, None)
        assert rc == 0
        torch.cuda.synchronize()
        An, Zn = A.cpu().numpy(), Z.cpu().numpy()
        assert np.max(np.abs(Zn.conj().T @ Zn - np.eye(n))) < 1e-12
        assert np.max(np.abs(Zn @ An @ Zn.conj().T - G)) < 1e-12
        if stop:
            assert np.max(np.abs(np.tril(An, -2))) < 1e-13
        else:
            assert np.max(np.abs(np.tril(An, -1))) == 0


@pytest.mark.parametrize("n", [40, 96])
def test_hessenberg_and_schur_small_tail(n):
    """Columns whose entries below the subdiagonal are tiny against the subdiagonal (1e-10 against
    O(1)): the reflector must still annihilate them (a norm formed as ||x||^2 - |x0|^2 cancels to
    zero there, and the entries would be dropped later)."""
    print(f"[case] schur small tail n={n}", flush=True)
    rng = np.random.default_rng(n + 11)
    G = np.triu(crand(rng, n, n)) / np.sqrt(n)
    i = np.arange(1, n)
    G[i, i - 1] = crand(rng, n - 1)
    G = G + 1e-10 * np.tril(crand(rng, n, n), -2)
    for stop in (1, 0):
        A = T(G)
        Z = T(np.zeros((n, n)))
        assert lib().lindx_schur(P(A), P(Z), n, stop, None) == 0
        torch.cuda.synchronize()
        An, Zn = A.cpu().numpy(), Z.cpu().numpy()
        assert np.max(np.abs(Zn.conj().T @ Zn - np.eye(n))) < 1e-12
        assert np.max(np.abs(Zn @ An @ Zn.conj().T - G)) < 1e-12
        assert np.max(np.abs(np.tril(An, -2 if stop else -1))) == 0.0


@pytest.mark.parametrize("m", [1, 2, 7, 30, 64])
def test_small_eig(m):
    rng = np.random.default_rng(m)
    A = crand(rng, m, m)
    w = T(np.zeros(m))
    Y = T(np.zeros((m, m)))
    rc = lib().lindx_small_eig(P(T(A)), m, P(w), P(Y), None)
    assert rc == 0
    wn, Yn = w.cpu().numpy(), Y.cpu().numpy()
    assert np.max(np.abs(A @ Yn - Yn * wn[None, :])) < 1e-10 * max(1, np.abs(wn).max())
    assert np.allclose(np.linalg.norm(Yn, axis=0), 1.0, atol=1e-12)
    for z in np.linalg.eigvals(A):
        assert np.min(np.abs(wn - z)) < 1e-10


@pytest.mark.parametrize("n", [1, 5, 17, 64, 130, 600])
def test_trevec_triinv(n):
    rng = np.random.default_rng(n + 1)
    Tm = np.triu(crand(rng, n, n)) + np.diag(np.arange(n) * 0.5)
    Y = T(np.zeros((n, n)))
    assert lib().lindx_trevec(P(T(Tm)), P(Y), n, None) == 0
    Yn = Y.cpu().numpy()
    d = np.diag(Tm)
    assert np.allclose(np.diag(Yn), 1.0)
    assert np.max(np.abs(Tm @ Yn - Yn * d[None, :])) < 1e-9 * np.abs(Yn).max()
    Yi = T(np.zeros((n, n)))
    assert lib().lindx_triinv(P(Y), P(Yi), n, None) == 0
    assert np.max(np.abs(Yi.cpu().numpy() @ Yn - np.eye(n))) < 1e-9 * np.abs(Yn).max()


@pytest.mark.parametrize("n", [1, 17, 32, 100, 700])
@pytest.mark.parametrize("shift", [0.0, -0.3 + 0.2j])
def test_trisylv(n, shift):
    rng = np.random.default_rng(n + 2)
    Tm = np.triu(crand(rng, n, n)) / np.sqrt(n) - 2.0 * np.eye(n)
    C = crand(rng, n, n)
    X = T(C)
    Tt = T(Tm)
    assert lib().lindx_trisylv(P(Tt), P(X), n, shift.real, shift.imag, None) == 0
    Xn = X.cpu().numpy()
    res = Tm @ Xn + Xn @ Tm.conj().T + shift * Xn - C
    assert np.max(np.abs(res)) < 1e-12 * np.abs(C).max() * n


@pytest.mark.parametrize("k", [1, 3, 16, 30, 64])
@pytest.mark.parametrize("kind", ["real", "complex", "exact1"])
def test_ritz_near(k, kind):
    """The Ritz pair nearest 1 of an upper Hessenberg matrix by inverse iteration, against
    numpy.linalg.eig: the eigenvalue to 1e-12 (relative to ||H||), the eigenvector up to phase to
    1e-9 (its condition number grows with 1 / gap), the in-space residual it reports against one
    recomputed on the host.  'real' is a real Hessenberg matrix (the steady-state iteration's, whose
    Krylov vectors are Hermitian) with an eigenvalue close to 1; 'exact1' has 1 as an exact
    eigenvalue (a converged iteration), where H - I is singular."""
    rng = np.random.default_rng(17 * k + len(kind))
    # spectrum: one eigenvalue at 0.97 (or exactly 1), the rest within 0.3 of the origin; a random
    # similarity, then the Hessenberg form (real throughout for the real kinds)
    cplx_kind = kind == "complex"
    w = 0.3 * (rng.random(k) * 2 - 1) + (0.3j * (rng.random(k) * 2 - 1) if cplx_kind else 0)
    w[0] = 1.0 if kind == "exact1" else 0.97
    Q = rng.standard_normal((k, k)) + (1j * rng.standard_normal((k, k)) if cplx_kind else 0)
    A = Q @ np.diag(w) @ np.linalg.inv(Q)
    import scipy.linalg as sl
    Hm = np.asarray(sl.hessenberg(A if cplx_kind else A.real), dtype=np.complex128)
    out = T(np.zeros(k + 2))
    its = ctypes.c_int(0)
    Ht = T(Hm)
    assert lib().lindx_ritz_near(P(Ht), k, 1.0, 0.0, P(out), ctypes.byref(its), None) == 0
    o = out.cpu().numpy()
    theta, y, rin = o[0], o[1:k + 1], o[k + 1].real
    w, V = np.linalg.eig(Hm)
    i = int(np.argmin(np.abs(w - 1)))
    scale = max(1.0, np.linalg.norm(Hm))
    print(f"[case] ritz k={k} {kind}: theta {theta:.15g} ref {w[i]:.15g}, {its.value} iterations, rin {rin:.2e}",
          flush=True)
    assert abs(theta - w[i]) <= 1e-12 * scale
    v = V[:, i] / np.linalg.norm(V[:, i])
    ph = np.vdot(v, y)
    assert np.linalg.norm(y - v * ph / abs(ph)) <= 1e-9
    assert abs(np.linalg.norm(y) - 1) < 1e-13
    j = int(np.argmax(np.abs(y)))
    assert abs(y[j].imag) <= 1e-14 and y[j].real > 0
    r_host = np.linalg.norm(Hm @ y - theta * y)
    assert abs(rin - r_host) <= 1e-12 * scale + 1e-3 * r_host


@pytest.mark.parametrize("n", [37, 130, 300])
@pytest.mark.parametrize("shift", [0.0, -0.3 + 0.2j])
@pytest.mark.parametrize("case", ["spread-1e4", "spread-median", "spread-none", "clustered-1e4", "repeated-1e4"])
def test_trisylv_block_eigenbases(n, shift, case):
    """The triangular Sylvester solve with 32 x 32 diagonal block pairs taken through their
    eigenvector matrices (the low-precision maps of the Schur route).  'spread': diagonal entries
    spread over the left half-plane as a generator's eigenvalues are (moderate block condition
    numbers), with the library's threshold 1e4, with the median condition number as threshold
    (a mix of both ways) and with threshold 0 (every pair swept: equal to the sweep bit for bit).
    'clustered': the near-equal diagonal of the sweep test (block condition numbers up to 1e13):
    pairs above the threshold must fall back to the sweep.  'repeated': two equal diagonal entries
    in the first block (infinite condition number).  Residual against T, C on the host: the
    block-eigenbasis products round at about u 32 kappa_I kappa_J of the largest entry (four
    products of length 32 with matrices of those condition numbers), bounded by
    1e-14 kappa_max^2 n max|C| with kappa_max the largest condition number of a block taken that way."""
    rng = np.random.default_rng(n + 7)
    kind, how = case.split("-")
    if kind == "spread":
        d = -(0.2 + rng.random(n)) + 1j * rng.standard_normal(n)
        Tm = 0.3 * np.triu(crand(rng, n, n), 1) / np.sqrt(n) + np.diag(d)
    else:
        Tm = np.triu(crand(rng, n, n)) / np.sqrt(n) - 2.0 * np.eye(n)
    if kind == "repeated":
        Tm[5, 5] = Tm[9, 9]
    C = crand(rng, n, n)
    nb = (n + 31) // 32
    kap = (ctypes.c_double * nb)()
    Tt = T(Tm)
    if how == "median":
        Xp = T(C)
        assert lib().lindx_trisylv_blk(P(Tt), P(Xp), n, shift.real, shift.imag, 0.0, kap, None) == 0
        thr = float(np.median(np.array(kap[:])))
    else:
        thr = {"1e4": 1e4, "none": 0.0}[how]
    X = T(C)
    assert lib().lindx_trisylv_blk(P(Tt), P(X), n, shift.real, shift.imag, thr, kap, None) == 0
    kv = np.array(kap[:])
    used = kv[np.isfinite(kv) & (kv <= thr)]
    kmax = max(1.0, float(used.max())) if used.size else 1.0
    Xn = X.cpu().numpy()
    res = np.max(np.abs(Tm @ Xn + Xn @ Tm.conj().T + shift * Xn - C))
    print(f"[case] {case} n={n}: kappa min {kv.min():.3g} median {np.median(kv):.3g} max {kv.max():.3g}, "
          f"{used.size} of {nb} blocks below the threshold, residual {res:.3g}", flush=True)
    if kind == "repeated":
        assert not np.isfinite(kv[0])
    if kind == "spread" and how == "1e4":
        assert used.size == nb  # the eigenbasis way is the one under test here
    assert res < (1e-14 * kmax ** 2 + 1e-12) * n * np.abs(C).max()
    if how == "none":
        Xs = T(C)
        assert lib().lindx_trisylv(P(Tt), P(Xs), n, shift.real, shift.imag, None) == 0
        assert torch.equal(X, Xs)


@pytest.mark.parametrize("k,length,pad", [(1, 1, 0), (9, 5000, 3), (64, 4096, 0), (65, 3001, 7), (200, 20000, 16),
                                          (31, 2048 * 2048, 0)])
def test_cgs2_step(k, length, pad):
    """One classical Gram-Schmidt step with re-orthogonalisation (the Arnoldi/GMRES kernels: 2-D dot
    kernel, multi-vector update, norm) against NumPy on an orthonormal random basis: both coefficient
    passes, the updated vector and its norm (FP64).  Ragged lengths, padded strides, chunked k."""
    rng = np.random.default_rng(k + length)
    ld = length + pad
    Vh = crand(rng, k, length)
    if k <= length:
        Q, _ = np.linalg.qr(Vh.T)  # orthonormal columns
        Vh = Q.T.copy()
    Vst = np.zeros((k, ld), dtype=np.complex128)
    Vst[:, :length] = Vh
    w0 = crand(rng, length)
    V_d, w_d = T(Vst), T(w0)
    h_d = torch.zeros(2 * k, dtype=torch.complex128, device="cuda:0")
    nrm_d = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    rc = lib().lindx_cgs2(P(V_d), ld, k, P(w_d), length, P(h_d), P(nrm_d), 1, None)
    assert rc == 0
    h1 = Vh.conj() @ w0
    w1 = w0 - Vh.T @ h1
    h2 = Vh.conj() @ w1
    w2 = w1 - Vh.T @ h2
    h = h_d.cpu().numpy()
    scale = np.linalg.norm(w0)
    assert np.max(np.abs(h[:k] - h1)) <= 1e-13 * scale
    assert np.max(np.abs(h[k:] - h2)) <= 1e-13 * scale
    assert np.max(np.abs(w_d.cpu().numpy() - w2)) <= 1e-13 * scale
    assert abs(float(nrm_d.cpu()[0]) - np.linalg.norm(w2)) <= 1e-12 * scale


@pytest.mark.parametrize("k,length,pad", [(1, 1024, 0), (7, 1024, 0), (30, 1024, 0), (64, 4096, 0), (17, 1000, 24),
                                          (5, 9, 3), (40, 4096, 0)])
def test_cgs2_small_step(k, length, pad):
    """The one-workgroup Gram-Schmidt step of small systems against NumPy and against the
    multi-kernel step: the Hessenberg column h1 + h2 and ||w2||, the normalised vector.  Ragged
    lengths, padded strides, k from 1 to the largest Krylov dimension."""
    print(f"[case] cgs2_small k={k} len={length} pad={pad}", flush=True)
    rng = np.random.default_rng(3 * k + length + pad)
    ld = length + pad
    Vh = crand(rng, k, length)
    if k <= length:
        Q, _ = np.linalg.qr(Vh.T)
        Vh = Q.T.copy()
    Vst = np.zeros((k, ld), dtype=np.complex128)
    Vst[:, :length] = Vh
    w0 = crand(rng, length)
    V_d, w_d = T(Vst), T(w0)
    hcol = torch.zeros(k + 1, dtype=torch.complex128, device="cuda:0")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    assert lib().lindx_cgs2_small(P(V_d), ld, k, P(w_d), length, P(hcol), P(nrm), None) == 0
    h1 = Vh.conj() @ w0
    w1 = w0 - Vh.T @ h1
    h2 = Vh.conj() @ w1
    w2 = w1 - Vh.T @ h2
    nw = np.linalg.norm(w2)
    scale = np.linalg.norm(w0)
    hc = hcol.cpu().numpy()
    assert np.max(np.abs(hc[:k] - (h1 + h2))) <= 1e-13 * scale
    assert abs(hc[k] - nw) <= 1e-12 * scale and hc[k].imag == 0
    assert float(nrm.cpu()[0]) == hc[k].real
    assert np.max(np.abs(w_d.cpu().numpy() - w2 / nw)) <= 1e-12 * scale / nw
    # the multi-kernel step on the same input
    w_m = T(w0)
    h_m = torch.zeros(2 * k, dtype=torch.complex128, device="cuda:0")
    n_m = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    assert lib().lindx_cgs2(P(V_d), ld, k, P(w_m), length, P(h_m), P(n_m), 1, None) == 0
    hm = h_m.cpu().numpy()
    assert np.max(np.abs(hc[:k] - (hm[:k] + hm[k:]))) <= 1e-13 * scale
    assert abs(hc[k].real - float(n_m.cpu()[0])) <= 1e-13 * scale


def test_cgs2_small_zero_norm():
    """w exactly in the span of the basis (a breakdown; standard basis vectors keep every operation
    exact): the column is the coefficients, the norm is exactly zero and w is left as the zero
    vector instead of being divided by it."""
    Vh = np.zeros((3, 64), dtype=np.complex128)
    Vh[0, 0] = Vh[1, 5] = Vh[2, 9] = 1.0
    w0 = Vh.T @ np.array([1.0, 0.5j, 0.25])
    V_d, w_d = T(Vh), T(w0)
    hcol = torch.zeros(4, dtype=torch.complex128, device="cuda:0")
    nrm = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    assert lib().lindx_cgs2_small(P(V_d), 64, 3, P(w_d), 64, P(hcol), P(nrm), None) == 0
    hc = hcol.cpu().numpy()
    assert np.array_equal(hc, [1.0, 0.5j, 0.25, 0.0])
    assert float(nrm.cpu()[0]) == 0.0
    assert np.array_equal(w_d.cpu().numpy(), np.zeros(64))


@pytest.mark.parametrize("n,d", [(200, 3), (256, 2), (1024, 4)])
def test_lindbladian_bf16x3(n, d):
    """L(X) with BF16x3 products (one stacked product, one batched reduction that also carries
    G X and X G^H) against the oracle's term-by-term FP64 L on a random non-Hermitian X, to the
    accuracy of the two-term BF16 split with FP32 accumulation (relative to the largest entry)."""
    import lind_inputs as li
    from oracle import lindblad as ol
    from paper_2608_30860_amd import Lindblad
    H, Ls = li.random_dense(n, d, 4)
    m = Lindblad(T(H), T(np.stack(Ls)), prec="bf16x3", route="eig")
    X = li.random_state(n, seed=9, hermitian=False)
    out = torch.empty((n, n), dtype=torch.complex128, device="cuda:0")
    L = lib()
    L.lindx_apply_bf16.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    Xd = T(X)
    assert L.lindx_apply_bf16(m.h, P(Xd), P(out)) == 0
    ref = ol.lindblad_apply(H, Ls, X)
    err = np.max(np.abs(out.cpu().numpy() - ref)) / np.max(np.abs(ref))
    print("bf16x3 L rel err", err)
    assert err < 1e-4
    m.close()
