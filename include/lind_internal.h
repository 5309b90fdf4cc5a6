/*
 * lind_internal.h -- kernel-level entry points of liblindx, exported for unit tests and for
 * the benchmark's per-kernel timing.  Not part of the stable API in lind.h.
 * All pointers are device pointers to complex128 (or complex64 where stated) row-major data;
 * stream is a hipStream_t (NULL = default).  Return 0 on success, a negative LIND_E* code on error.
 */
#ifndef LINDX_LIND_INTERNAL_H
#define LINDX_LIND_INTERNAL_H
#ifdef __cplusplus
extern "C" {
#endif

/* C = alpha * sum_{b < nbatch} op(A_b) op(B_b) (+ C if beta), op: 0 = as stored, 2 = conjugate
   transpose; A_b = A + b*sA, B_b = B + b*sB (element strides).  prec 0: complex128 operands;
   prec 1 (FP32 MFMA) / 2 (BF16 split, FP32 accumulate): complex64 operands, complex64 output
   unless out64 != 0 (complex128 output).  flags bit 0 (prec 0, M == N, real alpha): the result is
   Hermitian; only the tiles on and above the diagonal are computed and the rest is written as their
   conjugate transpose.  Asynchronous on stream. */
int lindx_gemm(int prec, int M, int N, int K, int nbatch, const void* A, long long lda, long long sA, int opA,
               const void* B, long long ldb, long long sB, int opB, void* C, long long ldc, double alpha_re,
               double alpha_im, int beta, int out64, int flags, void* stream);

/* Schur form in place: on entry A = G (n x n), on exit A = T (upper triangular), Z unitary with
   G = Z T Z^H.  mode bit 0 set returns the Hessenberg form instead of T; mode bits 8..15 choose
   the early-deflation window of the QR iteration (0: the library default, 1: none, 16..64: that
   many rows; anything else returns -1). */
int lindx_schur(void* A, void* Z, int n, int mode, void* stream);

/* eigenvalues w (m) and unit-norm right eigenvectors Y (m x m, column j for w[j]) of a dense
   m x m matrix A (m <= 64), one workgroup */
int lindx_small_eig(const void* A, int m, void* w, void* Y, void* stream);

/* eigenvectors Y of upper-triangular T (unit diagonal) and the inverse of a unit upper-triangular Y
   (n x n; only the upper triangle of the input is read, the output's lower triangle is zero).
   Each call allocates an n x n workspace for the transposed input and frees it before returning
   (synchronous).  n = 0 does nothing; n < 0 or n > 10240 (the column's right-hand sides must fit
   in 160 KB of LDS) returns -1, -5 if the workspace cannot be allocated. */
int lindx_trevec(const void* T, void* Y, int n, void* stream);

/* Ritz pair of the steady-state Arnoldi driver: for an upper Hessenberg H (k x k, k <= 64,
   complex128 row-major, device), the eigenvalue nearest sigma and its eigenvector by inverse
   iteration with the fixed shift sigma.  out (device, k + 2 complex128): out[0] = theta = y^H H y,
   out[1 .. k] = y (unit 2-norm, largest-modulus entry real positive), out[k + 1] = (||H y - theta
   y||_2, 0).  *iters (host, may be NULL) receives the iteration count.  Synchronous; 0, -1 on bad
   arguments, -4 on a device error, -5 when a workspace cannot be allocated. */
int lindx_ritz_near(const void* H, int k, double sigma_re, double sigma_im, void* out, int* iters, void* stream);
int lindx_triinv(const void* Y, void* Yinv, int n, void* stream);

/* T X + X T^H + shift X = C in place (X holds C on entry), T upper triangular */
int lindx_trisylv(const void* T, void* X, int n, double shift_re, double shift_im, void* stream);

/* The same solve (synchronous) as the low-precision maps of the Schur route run it: the 32 x 32
   diagonal blocks of T are diagonalised by their unit upper triangular eigenvector matrices Y_I,
   and a block pair (I, J) with kappa_inf(Y_I) and kappa_inf(Y_J) both <= thr is solved as
   Y_I [(Y_I^{-1} C Y_J^{-H}) / (t_a + conj t_b + shift)] Y_J^H, the others by the sweep.
   kap: host array of ceil(n / 32) doubles receiving the condition numbers (may be NULL;
   infinite where two diagonal entries of a block coincide).  0, -1 on bad arguments, -5 when a
   workspace cannot be allocated, -4 on a device error. */
int lindx_trisylv_blk(const void* T, void* X, int n, double shift_re, double shift_im, double thr, double* kap,
                      void* stream);

/* Event timing of the kernels inside a context, recorded on the context's stream.
   lindx_profile(ctx, 1) resets the counters and starts recording, (ctx, 0) stops.
   lindx_profile_read returns the number of timed launches and their summed duration for a kind:
   0 = stacked jump product [Lt_1; ..; Lt_d] X (one launch, M = d n),
   1 = jump reduction product sum_j Y_j Lt_j^H (one launch),
   2 = basis change V^H xi V with the fused divide (two launches),
   3 = one whole application of Phi. */
typedef struct lind_ctx lind_ctx;
int lindx_profile(lind_ctx* ctx, int enable);
int lindx_profile_read(lind_ctx* ctx, int kind, long long* count, double* total_ms);

/* C = sum_b op(A_b) op(B_b) through the pre-split BF16 product used by the BF16x3 map Phi
   (complex128 device arrays in and out, synchronous).  op(A) = A_b (M x K) or A_b^H (A_b stored
   K x M); op(B) = B_b (K x N) or B_b^H (B_b stored N x K); the nbatch blocks are consecutive.
   out_mode 0: planes, 1: transposed planes (both read back as complex128), 2: FP32 split-K
   partials reduced to complex128 (the only mode that takes nbatch > 1).  dr, dc (device
   complex128 of length M and N, or null; modes 0 and 1): entry (m, n) is divided by dr_m + dc_n.
   out_mode + 4: the result is Hermitian (M == N): only the tiles on and above the diagonal are
   computed and the rest is their conjugate transpose.
   Returns 0, or -1 for invalid arguments, -4 for a device error, -5 out of memory. */
int lindx_p4_test(const void* A, const void* B, int M, int N, int K, int nbatch, int opA, int opB, int out_mode,
                  const void* dr, const void* dc, void* C, void* stream);

/* Host only (no device work; usable without a GPU): the number of split-K runs the pre-split BF16
   product uses for `tiles` output tiles of 128 x 128, nbatch products of k_len each summed, on
   `cus` compute units: the run count s <= 64 (and <= the 32-deep stages available) that minimises
   rounds(s) x stages per run, the work of the longest workgroup chain, plus the partial-sum traffic
   s x tiles.  -1 for a negative argument. */
int lindx_p4_pick_split(long long tiles, int nbatch, int k_len, int cus);

/* Host only (no device work; usable without a GPU): the number of K chunks (1, 2, 4 or 8) into
   which lindx_gemm and the library's products split a single product of prec (0 FP64, 1 FP32,
   2 BF16x3) and shape M x N x K when ws_bytes of split-K workspace are available.  -1 for an
   invalid precision. */
int lindx_gemm_ksplit(int prec, int M, int N, int K, long long ws_bytes);

/* One classical Gram-Schmidt step with re-orthogonalisation, as in the Arnoldi and GMRES drivers:
   h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2, nrm = ||w||_2 (FP64).  V: k basis vectors of len
   complex128 entries at stride ld (>= len); h: 2k complex128 (h1, then h2); nrm: one double (all
   device).  reps > 1 repeats the step on the updated w (timing).  Synchronous; allocates a
   partial-sum workspace.  Returns 0, -1 for invalid arguments, -4, -5. */
int lindx_cgs2(const void* V, long long ld, int k, void* w, long long len, void* h, void* nrm, int reps,
               void* stream);

/* The same step in one workgroup, as the steady-state Arnoldi driver runs it for systems of at most
   4096 entries: afterwards w holds w2 / ||w2|| (w2 unchanged when ||w2|| = 0), hcol (device, k + 1
   complex128) the Hessenberg column [h1 + h2; ||w2||] and nrm (device double) ||w2||.  k <= 64,
   len <= 4096.  Synchronous; allocates the column workspace.  Returns 0, -1 for invalid arguments,
   -4, -5. */
int lindx_cgs2_small(const void* V, long long ld, int k, void* w, long long len, void* hcol, void* nrm, void* stream);

/* out = L(X) for the context's Lindbladian with BF16x3 products on pre-split planes (the operator
   of the inner shift-invert solves of lind_eigs in BF16x3 contexts); X, out: device n x n
   complex128, may not alias.  The planes of G and the L_j are split on the first call (eigenbasis
   route, d >= 1; LIND_EINVAL otherwise).  Synchronous. */
int lindx_apply_bf16(lind_ctx* ctx, const void* X, void* out);

/* dst = src (nbytes, a multiple of 16) with a plain vector copy kernel; used to calibrate the
   HBM byte counters of the profiler.  Asynchronous on stream. */
int lindx_copy(void* dst, const void* src, long long nbytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif
