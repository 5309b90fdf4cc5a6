/*
 * lind.h -- C ABI of lindx: steady states, low-lying spectra and steady-state gradients of
 * Lindblad master equations on one AMD Instinct MI355X (gfx950), following arXiv 2608.30860,
 * "Well-conditioned iterative methods for large open quantum systems".
 *
 * Problem (eq. lindblad_def): L(rho) = -i[H, rho] + sum_j (L_j rho L_j^+ - 1/2 {L_j^+ L_j, rho}),
 * split (eq. lindblad_decomposition, eq. G) as L = S + K with
 *   S(X) = G X + X G^+,  K(X) = sum_j L_j X L_j^+,  G = -iH - 1/2 sum_j L_j^+ L_j.
 * The hot path is repeated application of the completely positive trace-preserving map
 *   Phi = -K S^{-1}                                   (Section 2.2, Theorem 1)
 * inside Arnoldi, with S^{-1} built on a one-time FP64 factorisation of G.
 *
 * Conventions for every entry point
 *   - Matrices are DEVICE pointers to contiguous row-major n x n complex128 arrays (interleaved
 *     re, im; i.e. double _Complex / std::complex<double>), leading dimension n.
 *   - Jump operators: one device buffer of d stacked n x n matrices, L_j at offset j*n*n.
 *   - The caller owns every buffer it passes.  lind_create COPIES H and the L_j; later writes by
 *     the caller do not affect the context.  The context owns its factorisation and workspaces.
 *   - Calls are enqueued on opts.stream (NULL = the default stream) and synchronise only where
 *     a host scalar is returned or a host-side iteration decision is needed.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Return codes: LIND_OK on success, a negative LIND_E* code otherwise.  LIND_EINVAL leaves
 *     every output untouched.  LIND_ENOCONV still writes the best iterate and fills info.
 *     lind_last_error(ctx) returns a message for the last failure on that context.
 *   - This library never falls back to a CPU implementation: without a usable gfx950 device
 *     lind_create returns LIND_EDEVICE.
 */
#ifndef LINDX_LIND_H
#define LINDX_LIND_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lind_ctx lind_ctx;

/* largest n accepted by lind_create (the triangular eigenvector solves hold one column's
   right-hand sides, n complex128 values, in a workgroup's 160 KB of LDS) */
#define LIND_NMAX 10240

enum {
  LIND_OK = 0,
  LIND_EINVAL = -1,     /* invalid argument (NULL pointer, n < 1, d < 0, non-finite input, ...) */
  LIND_ESINGULAR = -2,  /* S not invertible: spec(G) meets iR (Theorem 1, first case), a
                           vanishing divisor mu - s_i - conj(s_j), or 1 - eta Tr W = 0 (eq. ShermanMorr) */
  LIND_ENOCONV = -3,    /* iteration cap or time limit reached; best iterate returned */
  LIND_EDEVICE = -4,    /* HIP runtime / kernel launch error, or no gfx950 device */
  LIND_ENOMEM = -5      /* device allocation failed */
};

/* arithmetic of the products inside Phi (the FP64 residual, Arnoldi orthogonalisation and the
   projected eigenproblems are always FP64) */
enum { LIND_PREC_FP64 = 0, LIND_PREC_FP32 = 1, LIND_PREC_BF16X3 = 2 };
/* Lyapunov backend (Section A.1): eigenbasis transform + elementwise divide, or Schur form +
   triangular Sylvester (Bartels-Stewart).  AUTO picks EIG when kappa_2(U) <= kappa_max. */
enum { LIND_ROUTE_AUTO = 0, LIND_ROUTE_EIG = 1, LIND_ROUTE_SCHUR = 2 };
/* steady-state method: Algorithm "Steady state as the fixed point of Phi" (Arnoldi on Phi, then
   FP64 refinement) or Algorithm "Steady state via preconditioned GMRES" (the deflated system
   L~_eta rho = eta I, eq. steady_state_linear_problem, right-preconditioned by Precond(., 0, eta)) */
enum { LIND_METHOD_PHI_ARNOLDI = 0, LIND_METHOD_GMRES = 1 };

typedef struct {
  int prec;             /* LIND_PREC_*                                    default FP64        */
  int route;            /* LIND_ROUTE_*                                   default AUTO        */
  double kappa_max;     /* AUTO threshold on kappa_2 of the eigenvector matrix, default 1e3  */
  int m;                /* Krylov dimension (<= 64)                       default 30          */
  int p;                /* Ritz pairs kept at a thick restart (eigs)      default 0 = auto    */
  int max_restarts;     /* Arnoldi / GMRES restarts                       default 200         */
  int refine_max;       /* FP64 refinement steps                          default 8           */
  double eta;           /* deflation constant (eq. steady_state_linear_problem), default 1.0 */
  double time_limit_s;  /* wall-clock cap per solver call, <= 0: none     default 0; checked
                           between Krylov steps (lind_eigs: between thick restarts)             */
  void* stream;         /* hipStream_t, NULL = default stream                                 */
  int method;           /* LIND_METHOD_* for lind_steady_state (and the state of steady_grad), default PHI_ARNOLDI */
  const double* gauge;  /* HOST, NULL or 2d doubles (re, im) of c_j: the split uses L_j + c_j I and
                           H + (1/2i) sum_j (conj(c_j)(L_j + c_j) - c_j (L_j + c_j)^+) (Remark
                           "Non-uniqueness of the decomposition", eq. lindblad_gauge); L itself is
                           unchanged.  Read by lind_create only.               default NULL        */
} lind_opts;

typedef struct {
  double resid_trace;   /* trace-norm bound sum_j ||col_j(L rho)||_2 >= ||L rho||_1 (FP64)   */
  double resid_max;     /* ||L rho||_max (the paper's stopping norm)                          */
  double err_est;       /* estimated error of the returned object (solver specific)          */
  double kappa_U;       /* 2-norm condition number of the unit-column eigenvector matrix     */
  double t_factor_s;    /* wall time of the factorisation of G (lind_create)                 */
  double t_solve_s;     /* wall time of the solver call                                      */
  int n_phi;            /* applications of Phi (or of the preconditioned operator)           */
  int n_restarts;       /* Arnoldi cycles / GMRES cycles                                     */
  int n_refine;         /* FP64 refinement steps                                             */
  int n_inner;          /* inner iterations (GMRES steps inside eigs / refinement / adjoint) */
  int route_used;       /* LIND_ROUTE_EIG or LIND_ROUTE_SCHUR                                */
} lind_info;

/* Fill opts with the defaults listed above. */
void lind_default_opts(lind_opts* opts);

/* Build a context for L defined by H (n x n, Hermitian) and d jump operators L_stacked (d x n x n),
   both device pointers (complex128).  Computes G (eq. G) and its FP64 factorisation on the GPU:
   Householder Hessenberg reduction, multishift QR to the Schur form G = Z T Z^+, and for the
   eigenbasis route the eigenvectors U = Z Y with V = U^{-+} = Z Y^{-+} (Algorithm "No-jump
   resolvent via eigendecomposition").  opts may be NULL (defaults).
   Errors: EINVAL (NULL pointers, n < 1, n > LIND_NMAX, d < 0, d > 64), ESINGULAR (min |Re s_i|
   too small: Theorem 1, first case), ENOMEM, EDEVICE. */
int lind_create(lind_ctx** out, const void* H, const void* L_stacked, int n, int d, const lind_opts* opts);

/* Release every device buffer of the context.  NULL is a no-op. */
void lind_destroy(lind_ctx* ctx);

/* out = L(rho) (eq. lindblad_def) for any complex n x n rho, always FP64.  rho and out may not
   alias. */
int lind_apply(lind_ctx* ctx, const void* rho, void* out);

/* out = L*(X), the Hilbert-Schmidt adjoint i[H, X] + sum_j (L_j^+ X L_j - 1/2 {L_j^+ L_j, X}),
   always FP64. */
int lind_apply_adjoint(lind_ctx* ctx, const void* X, void* out);

/* X = (S - mu)^{-1} Y, i.e. the solution of (G - mu/2) X + X (G - mu/2)^+ = Y
   (eq. lyapunov; eq. G-lambda).  mu = 0 gives S^{-1}; the paper's resolvent is
   R^S_mu = (mu - S)^{-1} = -(this).  FP64, via the context's route.  Y and X may alias.
   Errors: ESINGULAR if mu - s_i - conj(s_j) vanishes for some i, j. */
int lind_sinv(lind_ctx* ctx, const void* Y, void* X, double mu_re, double mu_im);

/* out = Phi(xi) = -K(S^{-1} xi) (Section 2.2) in the context's precision (opts.prec); input and
   output complex128.  xi and out may not alias. */
int lind_phi(lind_ctx* ctx, const void* xi, void* out);

/* Steady state rho_inf (L rho = 0, Tr rho = 1, rho Hermitian) by Algorithm "Steady state as the
   fixed point of Phi": restarted Arnoldi(m) on Phi, Ritz value nearest 1, rho = -S^{-1} xi,
   hermitise, normalise; followed, until the FP64 residual bound resid_trace <= tol, by FP64
   iterative refinement: r = L rho (FP64), solve (I - Phi) zeta = r by GMRES on Phi in the
   context's precision, rho <- normalise(herm(rho - S^{-1} zeta)).
   rho0: device n x n start state (NULL -> I/n); the Arnoldi start vector is xi0 = -S(rho0).
   A Krylov space that becomes invariant (an exactly zero Arnoldi norm) ends the cycle with the
   Ritz pair of the space built so far.
   rho_out: device n x n.  info may be NULL.  Returns ENOCONV (best iterate written) when the
   restart/refinement caps or the time limit are hit. */
int lind_steady_state(lind_ctx* ctx, double tol, const void* rho0, void* rho_out, lind_info* info);

/* k smallest-magnitude nonzero eigenvalues of L near the shift mu by Algorithm "Low-lying
   spectrum via shift-invert Arnoldi": Krylov-Schur Arnoldi on (mu - L~_eta)^{-1}, each
   application one right-preconditioned GMRES solve with P_mu = Precond(., mu, eta) (Algorithm
   "Precond", eq. ShermanMorr); lambda = mu - 1/nu.  Converged when
   max_k ||L v_k - lambda_k v_k||_max <= tol * max(1, |lambda_k|).
   evals_out: HOST array of k complex128, sorted by |lambda| ascending (ties: Im ascending).
   evecs_out: DEVICE k x n x n (unit Frobenius norm, largest entry real positive) or NULL.
   Errors: EINVAL (k < 1, k > m - 2), ESINGULAR (1 - eta Tr W = 0), ENOCONV. */
int lind_eigs(lind_ctx* ctx, int k, double mu_re, double mu_im, double tol, void* evals_out, void* evecs_out,
              lind_info* info);

/* Gradient of J = Re Tr(O rho_inf) (Remark "Differentiating the steady state"): solves the
   steady state to tol, then the adjoint system L~_eta^* w = O - <O> I by GMRES right-
   preconditioned with the adjoint deflated no-jump resolvent, and contracts
     grad_H = i [rho, w],   grad_L_j = L_j {rho, w} - 2 w L_j rho,
   with the convention dJ = Re Tr(g^+ dZ) (g = dJ/dRe Z + i dJ/dIm Z).
   O: device n x n (Hermitian); expval: HOST double; grad_H: device n x n or NULL;
   grad_L: device d x n x n or NULL; rho_out: device n x n or NULL (the steady state used). */
int lind_steady_grad(lind_ctx* ctx, const void* O, double tol, double* expval, void* grad_H, void* grad_L,
                     void* rho_out, lind_info* info);

/* X = (lambda - L)^{-1} B for Re(lambda) > 0 (Corollary "Resolvent of the Lindbladian") by
   GMRES right-preconditioned with the no-jump resolvent R^S_lambda = (lambda - S)^{-1}
   (eq. right-precond-identity; the contraction theorem bounds ||K R^S_lambda|| < 1), with a
   recycled subspace kept across restarts.  The operator lambda - L is applied in FP64, the
   preconditioner in the context's precision.  Stops when ||B - (lambda - L) X||_F <= tol ||B||_F.
   B, X: device n x n complex128 (may not alias).  info (may be NULL): n_inner = GMRES steps,
   n_phi = preconditioner applications, n_restarts = cycles, err_est = final relative residual,
   resid_max = its max-norm.  Errors: EINVAL (Re(lambda) <= 0, tol <= 0), ENOCONV (X holds the
   last iterate). */
int lind_resolve(lind_ctx* ctx, double lambda_re, double lambda_im, const void* B, void* X, double tol,
                 lind_info* info);

/* Implicit Euler (eq. resolvent of the implicit-solver section): rho_{k+1} = (I - dt L)^{-1} rho_k
   = (1/dt) R^L_{1/dt} rho_k for k < steps, each step a lind_resolve-type solve at lambda = 1/dt to
   relative residual tol, warm-started from rho_k; the recycled GMRES subspace is carried across
   steps.  rho0, rho_out: device n x n complex128 (may alias: in-place stepping).  info:
   n_restarts = steps done, n_inner = total GMRES steps, err_est = worst relative residual.
   Errors: EINVAL (dt <= 0, steps < 0, tol <= 0), ENOCONV (a step missed tol or the time limit
   was hit; rho_out holds the last completed state). */
int lind_ie(lind_ctx* ctx, double dt, int steps, const void* rho0, void* rho_out, double tol, lind_info* info);

/* Size of the fixed device array behind lind_apply_noalloc (64 MiB, one copy per GPU the library
   runs on, held until the process ends). */
#define LIND_NOALLOC_SCRATCH_BYTES (64LL << 20)

/* For callers that cannot allocate device memory while they run (code under stream capture,
   tight serving loops, harnesses that forbid hipMalloc): out = L(rho) exactly as lind_apply
   computes it (same kernels, FP64), but every intermediate -- the stacked products L_j rho and the
   split-K partials of the sum over j -- lives in a fixed device array of
   LIND_NOALLOC_SCRATCH_BYTES instead of the context's workspaces.  The call makes no hipMalloc,
   hipFree or other allocating call; the context (created beforehand by lind_create) and the
   device buffers rho, out (n x n complex128, may not alias) are the caller's.
   Limit: lind_apply_noalloc_bytes(n, d) <= LIND_NOALLOC_SCRATCH_BYTES (about d n^2 16 bytes plus
   the partials; e.g. n = 512 with d <= 8, n = 1024 with d <= 3), else LIND_EINVAL with a message.  The context's device
   must be the current device.  The array is shared by every call on that GPU and keeps the last
   call's contents (each call overwrites what it reads); calls that overlap on one GPU (other
   threads, other streams) race on it.  Synchronises the context's stream before returning. */
int lind_apply_noalloc(lind_ctx* ctx, const void* rho, void* out);
/* Scratch bytes lind_apply_noalloc needs for an n x n system with d jump operators (-1 if n < 1
   or d < 0). */
long long lind_apply_noalloc_bytes(int n, int d);

/* Factorisation data (device pointers owned by the context, valid until lind_destroy):
   which: 0 = G, 1 = T (Schur factor), 2 = Z (Schur vectors), 3 = U (unit-column eigenvectors),
   4 = V = U^{-+}, 5 = s (n eigenvalues of G).  Returns NULL if not available. */
const void* lind_factor_ptr(const lind_ctx* ctx, int which);

/* Message describing the last failure on ctx (or of lind_create when ctx is NULL). */
const char* lind_last_error(const lind_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* LINDX_LIND_H */
