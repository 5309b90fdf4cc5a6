// Launch wrappers of the lindx device kernels.  Host-callable, all asynchronous on `st`.
#pragma once
#include "common.hpp"

namespace lindx {

// ---------------------------------------------------------------------------
// complex matrix products  C = alpha * sum_b op(A_b) op(B_b)  (+ C)  with epilogues
// ---------------------------------------------------------------------------
enum { EPI_NONE = 0, EPI_DIV = 1, EPI_HERM_ADD = 2 };
enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16X3 = 2 };

struct GemmDesc {
  int M = 0, N = 0, K = 0, nbatch = 1;       // per-batch sizes (complex entries)
  const void* A = nullptr; long long lda = 0, sA = 0; int opA = OP_N;
  const void* B = nullptr; long long ldb = 0, sB = 0; int opB = OP_N;
  void* C = nullptr; long long ldc = 0;
  double ar = 1.0, ai = 0.0;                  // alpha
  int beta = 0;                               // 1: accumulate into C
  int epi = EPI_NONE;
  const zd* dr = nullptr; const zd* dc = nullptr; double dzr = 0.0, dzi = 0.0;  // EPI_DIV
  const void* E = nullptr; long long lde = 0;                                   // EPI_HERM_ADD
  int out64 = 0;                              // float kernels: write complex128 output
  // split-K over the batch dimension: nsplit blocks per output tile each reduce nbatch/nsplit
  // batches into ws (FP32 or FP64 complex partials), a second kernel sums them and applies the
  // epilogue.  nsplit = 1: single pass.  ws must hold nsplit * M * N complex accumulators.
  int nsplit = 1;
  void* ws = nullptr;
  long long ws_bytes = 0;  // capacity of ws (0: what gemm_ws_bytes gives for this shape)
  // Hermitian result (M == N, real alpha, Hermitian epilogue data): only tiles on and above the
  // diagonal are computed, the rest is written as their conjugate transpose (FP64 products)
  int tri = 0;
};
// workspace bytes gemm() needs for a split-K launch of this shape (0 if it would not split)
long long gemm_ws_bytes(int prec, int M, int N, int nbatch);
// chunks of K (1, 2, 4 or 8) that gemm() splits a single small product into, given ws_avail bytes of
// workspace: only where its 32 x 32 (FP64: or 64 x 64) tiles fill at most half the chip; each chunk
// at least 32 deep and K divisible by the count.  Host only.
int gemm_small_ksplit(int prec, int M, int N, int K, long long ws_avail);
// Phi(xi) = -sum_j Lt_j [(V^H xi V) / (s_a + conj s_b)] Lt_j^H for n <= 32 in one workgroup (FP64;
// all operands complex128 row-major on the device, Lt stacked d x n x n)
int phi_small(const zd* xi, const zd* V, const zd* Lt, const zd* s, const zd* sbar, int n, int d, zd* out,
              hipStream_t st);

// prec = PREC_F64: A, B, C, E are complex128.
// prec = PREC_F32 / PREC_BF16X3: A, B are complex64; C (and E) complex64 unless out64.
int gemm(int prec, const GemmDesc& g, hipStream_t st);

// ---------------------------------------------------------------------------
// complex products on pre-split BF16 operands (BF16x3 mode): four bf16 planes
// [re_hi, re_lo, im_hi, im_lo], each rows x ld with k contiguous, zero-padded to whole tiles
// ---------------------------------------------------------------------------
struct P4 {
  __bf16* p = nullptr;
  long long rows = 0, ld = 0, pstride = 0;  // allocated rows, k stride, plane stride (elements)
};
enum { P4OUT_PLANES = 0, P4OUT_PLANES_T = 1, P4OUT_WS = 2 };
struct P4Desc {
  // P4OUT_WS: the nbatch * ceil(K / 32) (batch, k-chunk) steps of each output tile are cut into
  // nsplit contiguous, nearly equal runs (1 <= nsplit <= that count), one workgroup per run
  int M = 0, N = 0, K = 0, nbatch = 1, nsplit = 1;
  // op(A) row m, k at A[pl * pA + b * sA + m * lda + k]; op(B) column n, k at B[pl * pB + b * sB + n * ldb + k]
  const __bf16* A = nullptr; long long lda = 0, pA = 0, sA = 0;
  const __bf16* B = nullptr; long long ldb = 0, pB = 0, sB = 0;
  int conjA = 0, conjB = 0;
  int out = P4OUT_PLANES;
  __bf16* C = nullptr; long long ldc = 0, pC = 0;   // planes out: [m][n] or (transposed) [n][m]
  const zd* dr = nullptr; const zd* dc = nullptr;   // optional divide by dr_m + dc_n (planes out)
  float2* ws = nullptr;                             // P4OUT_WS: nsplit * M * N partials
  void* out64 = nullptr; long long ldo = 0; double alpha = 1.0;  // P4OUT_WS: complex128 result
  // Hermitian result (M == N): only the tiles on and above the diagonal are computed; the result
  // below is the conjugate transpose (P4OUT_WS: in the reduction; planes out: mirrored writes)
  int tri = 0;
};
long long p4_rows_alloc(long long rows);
long long p4_ld(long long k);
// allocate zeroed planes for a rows x k operand (rows padded to whole tiles plus one spare tile)
int p4_alloc(P4& p, long long rows, long long k);
// planes of X (rows x cols, complex128 if is64 else complex64), transposed and/or conjugated
int p4_split(const void* X, int is64, long long ldx, int rows, int cols, int trans, int conj, const P4& out,
             hipStream_t st);
int p4_gemm(const P4Desc& g, hipStream_t st);
// split-K count for a P4OUT_WS product of `tiles` output tiles and nbatch * k_len reduction
// length, on a device with `cus` compute units (one workgroup per unit at a time)
int p4_pick_split(long long tiles, int nbatch, int k_len, int cus);
// compute units of device dev (256 on MI355X if the query fails: only a tuning input)
int device_cus(int dev);
// complex128 X (rows x cols) from planes, reading P[r][c] (or P[c][r] when trans)
int p4_join(const P4& P, int rows, int cols, int trans, zd* X, long long ldx, hipStream_t st);

// ---------------------------------------------------------------------------
// level-1 / elementwise kernels on complex128 vectors of length len (= n*n)
// ---------------------------------------------------------------------------
// h[j] = <V_j, w> = sum_i conj(V[j*ld + i]) w[i], j < k.  Result left on device (h) in FP64.
int multi_dot(const zd* V, long long ld, int k, const zd* w, long long len, zd* h, zd* scratch,
              hipStream_t st);
// w -= sum_j h[j] V_j   (coeff = -1)  or  out = sum_j h[j] V_j (accumulate = 0, coeff = +1)
int multi_axpy(const zd* V, long long ld, int k, const zd* h, zd* w, long long len, int accumulate,
               double coeff, hipStream_t st);
// ||w||_2 into out (device double); scratch >= 1024 doubles
int nrm2(const zd* w, long long len, double* out, double* scratch, hipStream_t st);
// w *= 1/s where s is a device double (scalar produced by nrm2)
int scale_by_inv(zd* w, long long len, const double* s, hipStream_t st);
// as scale_by_inv (no scaling when s <= 0), and column j of the device Hessenberg matrix Hd (row stride
// ld): Hd[i][j] = h1[i] + h2[i] for i <= j, Hd[j+1][j] = s, sub[j] = s
int scale_by_inv_hcol(zd* w, long long len, const double* s, const zd* h1, const zd* h2, zd* Hd, int ld, int j,
                      double* sub, hipStream_t st);
// the two CGS2 passes of Arnoldi step j = k - 1 against V_0 .. V_{k-1}, the norm, the scaling of w and
// its Hessenberg column (as above) in one workgroup, for len <= 4096 entries and k <= 64; -1 otherwise
int cgs2_small(const zd* V, long long ld, int k, zd* w, long long len, zd* Hd, int ldh, double* sub, hipStream_t st);
// y = a*x + b*y with host scalars
int axpby(zd a, const zd* x, zd b, zd* y, long long len, hipStream_t st);
int copy(const zd* x, zd* y, long long len, hipStream_t st);
int fill_zero(void* p, long long bytes, hipStream_t st);
// complex128 <-> complex64
int to_c64(const zd* x, zf* y, long long len, hipStream_t st);
int to_c128(const zf* x, zd* y, long long len, hipStream_t st);
// X <- scale * (X + X^H)/2 (n x n, in place); optional: divide by the real part of the trace
// (trace taken after hermitisation).  trace_out (device zd) receives the trace before scaling.
int hermitize(zd* X, int n, int normalize_trace, zd* trace_out, double* scratch, hipStream_t st);
// trace of n x n X into out (device zd)
int trace(const zd* X, int n, zd* out, double* scratch, hipStream_t st);
// norms of an n x n matrix: out[0] = Frobenius, out[1] = max |x_ij|, out[2] = sum_j ||col_j||_2
// (an upper bound on the trace norm), out[3] = max_i |Im x_ii|.  scratch >= 4*1024 doubles.
int mat_norms(const zd* X, int n, double* out, double* scratch, hipStream_t st);
// X += c * I
int add_identity(zd* X, int n, zd c, hipStream_t st);
// Sherman-Morrison step: Z += coef * W where coef = c*Tr(Z)/(1 - c*trW) computed on device
// X += c Tr(Y) I with the trace taken on the device (scratch_tr: one device complex128)
int add_identity_trace(zd* X, int n, const zd* Y, zd c, zd* scratch_tr, hipStream_t st);
int sherman_morrison(zd* Z, const zd* W, int n, zd c, zd trW, zd* scratch_tr, double* scratch,
                     hipStream_t st);
// D = G X (n x n) elementwise helpers for the generator: G = -iH - 1/2 W
int make_generator(const zd* H, const zd* W, zd* G, int n, hipStream_t st);
// scale columns: U[:, j] *= s[j], V[:, j] /= conj?  (s real) -- U and V both n x n
int scale_cols(zd* X, int n, const double* s, int invert, hipStream_t st);
int col_norms(const zd* X, int n, double* out, hipStream_t st);
// y = A x for n x n A (opA = N or C), vectors of length n
// y = op(A) x (n x n A); A^H x for n > 256 runs in two passes through scratch, which holds
// gemv_scratch_elems(n) entries (nullptr: one pass)
int gemv(const zd* A, int n, int opA, const zd* x, zd* y, zd* scratch, hipStream_t st);
long long gemv_scratch_elems(int n);
// out[i] = conj(x[i]) for complex arrays (used for sigma-bar)
int conj_copy(const zd* x, zd* y, long long len, hipStream_t st);
// X <- J X^T J etc: reverse both indices and transpose-conjugate (adjoint triangular form)
int flip_conj_transpose(const zd* X, zd* Y, int n, hipStream_t st);
// Y[i][j] = X[n-1-i][n-1-j]
int flip_rev(const zd* X, zd* Y, int n, hipStream_t st);

// ---------------------------------------------------------------------------
// factorisation of G (FP64): Hessenberg reduction, Schur form by QR iteration,
// eigenvectors of the triangular factor and the inverse of the eigenvector matrix.
// ---------------------------------------------------------------------------
struct SchurWork;
// In: A (n x n, overwritten by T, upper triangular), Z (n x n) out: Schur vectors, A = Z T Z^H
// on entry A holds G.  Returns 0 on success, -3 if the QR iteration failed to converge.
int schur_factor(zd* A, zd* Z, int n, hipStream_t st, double* t_hess, double* t_qr);
int schur_factor_ex(zd* A, zd* Z, int n, hipStream_t st, double* t_hess, double* t_qr, int mode);
// Y: eigenvectors of upper-triangular T (unit diagonal), Yinv = Y^{-1} (unit upper triangular);
// ws: n x n device workspace (receives the transposed input), overwritten
int trevec(const zd* T, zd* ws, zd* Y, int n, hipStream_t st);
int triinv_unit(const zd* Y, zd* ws, zd* Yinv, int n, hipStream_t st);
// extract diagonal of T into s
int diag_extract(const zd* T, zd* s, int n, hipStream_t st);

// small dense eigenproblem on the device (one workgroup, m <= 64):
// in: A (m x m, leading dim lda) -- general complex.  out: w (m eigenvalues), Y (m x m right
// eigenvectors, column j for w[j], unit 2-norm), info (device int: 0 ok, 1 no convergence).
int small_eig(const zd* A, int lda, int m, zd* w, zd* Y, int* info, hipStream_t st);
// Ritz pair of an upper Hessenberg H (k x k, k <= 64) with the eigenvalue nearest sigma, by inverse
// iteration: out[0] = theta, out[1..k] = unit y, out[k + 1] = (||H y - theta y||, 0); info = iterations
int ritz_near(const zd* H, int ld, int k, zd sigma, zd* out, int* info, hipStream_t st);

// ---------------------------------------------------------------------------
// triangular Sylvester solve  T X + X T^H + shift*X = Y  (T upper triangular, n x n)
// ---------------------------------------------------------------------------
// T X + X T^H + shift X = C (T upper triangular, X overwrites C); ws holds trisylv_ws_elems(n)
// complex entries of scratch
// Block eigenbases of T's 32 x 32 diagonal blocks (trisylv_blk_setup): Y, Y^{-1} (each
// trisylv_blk_elems(n) entries, block after block) and kap (one per block).  A block pair whose
// two condition numbers are <= thr is solved through them; null kap: every pair is swept.
struct TsBlk {
  const zd* Y = nullptr;
  const zd* Yi = nullptr;
  const double* kap = nullptr;
  double thr = 0.0;
};
int trisylv(const zd* T, zd* X, int n, zd shift, zd* ws, hipStream_t st, const TsBlk* blk = nullptr);
long long trisylv_ws_elems(int n);
long long trisylv_blk_elems(int n);
int trisylv_blk_setup(const zd* T, int n, zd* Y, zd* Yi, double* kap, hipStream_t st);

}  // namespace lindx
