// One-time FP64 factorisation of the no-jump generator G on the GPU.
//
//   G = Z T Z^H    (complex Schur form, Z unitary, T upper triangular)
//
// 1. Householder reduction to upper Hessenberg form: per column, one workgroup builds the
//    reflector and two bandwidth-bound passes apply it to both sides of A (A u is formed before
//    the left update, so one read-write pass does both); the reflectors reach Z in blocks of 64
//    in compact WY form, by three FP64 products.
// 2. Multishift QR iteration (complex single-shift bulges, up to 19 per sweep, shifts from the
//    eigenvalues of the trailing block).  A chain of bulges is chased down the diagonal in
//    64 x 64 windows that advance by 24 rows: each window is chased in LDS by one workgroup that
//    accumulates the window's unitary U_w; the launch of the next window first applies U_w^H to
//    the rest of the window's rows inside the active block (the columns the next window adds in
//    its own prologue, the columns beyond it on extra workgroups), while the updates of the rows
//    above the windows, of the columns right of the active block, and of Z are deferred to the
//    end of the sweep and applied window after window by row/column-parallel kernels (those of Z
//    on a second stream, since the iteration never reads Z).  Active blocks of at most 64 rows
//    are finished in LDS by one wave.  Before each sweep, aggressive early deflation (Braman,
//    Byers and Mathias, SIAM J. Matrix Anal. Appl. 23, 2002) brings the trailing 24 x 24 window
//    to Schur form in LDS, splits off the eigenvalues whose coupling to the rest of the matrix is
//    below machine precision, and hands the window's remaining eigenvalues to the sweep as
//    shifts; when many deflate the sweep is skipped.
// 3. Eigenvectors of T by back substitution (one wave per column) and the inverse of the unit
//    upper-triangular eigenvector matrix, giving the eigenbasis route G = U diag(s) U^{-1}.
#include <vector>
#include <chrono>
#include "kernels.hpp"
#include "lds_qr.hpp"

namespace lindx {

static constexpr int WIN = 64;    // window rows
static constexpr int STEP = 24;   // default window advance
static constexpr int NSMAX = 19;  // default bulges per sweep (WIN >= step + 2 * bulges + 1)
static constexpr int NSCAP = 23;  // most bulges one chase kernel holds
static constexpr int CHASE_T = 512;  // threads of the chase kernel (8 waves, two per SIMD)
static constexpr int MAXWIN = 256;
static constexpr int AEDW = 24;   // default early-deflation window rows (<= WIN)
static constexpr int WYB = 64;    // Householder reflectors applied to Z per block

struct WinList {
  int nwin;
  int r[MAXWIN];
  int bw[MAXWIN];
};

// ------------------------------------------------------------------ Hessenberg reduction -----
// Reflector for column k: P = I - gam u u^H with u = x + ph*||x|| e_{k+1}, P x = -ph*||x|| e_{k+1}.
// Each column costs two launches.  Column k of A is kept contiguously in `col` (written by the
// update of column k - 1; column 0 by k_hh_col0), and every workgroup of pass 1 derives the
// reflector's scalars from it in the same order, so all obtain the same bits without a launch of
// their own.
struct HHScal {
  zd x0, ph;
  double nrm, ax0;
  bool skip;
};
// Called by all 256 threads of a workgroup.  The part below x0 is summed on its own: ||x||^2 -
// |x0|^2 cancels to zero when that part is small against x0, and the column would be left
// unreduced.
__device__ inline HHScal hh_scalars(const zd* col, int n, int k) {
  __shared__ double sh[4];
  double s = 0;
  for (int i = k + 2 + threadIdx.x; i < n; i += 256) s += zabs2(col[i]);
  for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  const double tail = sh[0] + sh[1] + sh[2] + sh[3];
  HHScal r;
  r.x0 = col[k + 1];
  r.nrm = sqrt(zabs2(r.x0) + tail);
  r.ax0 = sqrt(zabs2(r.x0));
  r.ph = r.ax0 > 0 ? zscale(r.x0, 1.0 / r.ax0) : zmk(1, 0);
  r.skip = !(tail > 0.0);
  return r;
}
__device__ inline zd hh_u(const zd* col, const HHScal& r, int k, int i) {
  if (r.skip || i <= k) return zmk(0, 0);
  return i == k + 1 ? zadd(r.x0, zscale(r.ph, r.nrm)) : col[i];
}
__global__ void k_hh_col0(const zd* A, int n, zd* col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) col[i] = A[(long long)i * n];
}

// The two one-sided updates of column k are applied in one pass.  With w = gam u^H A (left) and
// A' = A - u w, the right update needs A' u = A u - u (w u), so A u can be formed from the matrix
// before the left update, together with u^H A:
//   A <- A - u w - y u^H,  y = gam (A u - u (w u)),  w u = gam u^H (A u);   Z <- Z - gam (Z u) u^H.
// Z is updated by blocks of reflectors (k_wy_t and three products, see hessenberg()).
// Pass 1 (k_hh_pass1): workgroups [0, ncb * nrc) form partial sums of u^H A over row chunks
// (rows > k; workgroup (cb, rc) = (b % ncb, b / ncb), 64 columns each); the others form the raw
// row sums (A u)_i, one row per wave, and store, for their rows, u, column c of the reflector
// block and the reduced column k of A (which no workgroup of this pass reads).
__global__ __launch_bounds__(256) void k_hh_pass1(zd* A, int n, int k, const zd* col, int rchunk, int ncb, int nrc,
                                                  zd* part, zd* y, zd* u, double* gam, zd* vb, int c,
                                                  double* gb) {
  __shared__ zd ss[4][64];
  const HHScal r = hh_scalars(col, n, k);
  const int nlp = ncb * nrc;
  if ((int)blockIdx.x < nlp) {
    const int cb = blockIdx.x % ncb, rc = blockIdx.x / ncb;
    const int j = k + 1 + cb * 64 + (threadIdx.x & 63);
    const int rg = threadIdx.x >> 6;
    const int r0 = k + 1 + rc * rchunk;
    const int r1 = r0 + rchunk < n ? r0 + rchunk : n;
    zd s = zmk(0, 0);
    if (j < n)
      for (int i = r0 + rg; i < r1; i += 4) s = zadd(s, zcmul(hh_u(col, r, k, i), A[(long long)i * n + j]));
    ss[rg][threadIdx.x & 63] = s;
    __syncthreads();
    if (rg == 0 && j < n) {
      const zd t = zadd(zadd(ss[0][threadIdx.x], ss[1][threadIdx.x]), zadd(ss[2][threadIdx.x], ss[3][threadIdx.x]));
      part[(long long)rc * n + j] = t;
    }
    return;
  }
  if ((int)blockIdx.x == nlp && threadIdx.x == 0) {
    const double g = r.skip ? 0.0 : 1.0 / (r.nrm * (r.nrm + r.ax0));  // u^H u = 2 ||x|| (||x|| + |x0|)
    gam[0] = g;
    gb[c] = g;
  }
  const int row = (blockIdx.x - nlp) * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  zd s = zmk(0, 0);
  for (int j = k + 1 + lane; j < n; j += 64) s = zadd(s, zmul(A[(long long)row * n + j], hh_u(col, r, k, j)));
  double a = s.x, b = s.y;
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  if (lane == 0) {
    y[row] = zmk(a, b);
    const zd ur = hh_u(col, r, k, row);
    u[row] = ur;
    vb[(long long)row * WYB + c] = ur;
    if (!r.skip && row > k) A[(long long)row * n + k] = (row == k + 1) ? zscale(r.ph, -r.nrm) : zmk(0, 0);
  }
}
// A <- A - u w - y u^H on a tile of 64 columns (> k) and HU_R rows.  Each workgroup forms w_j for
// its columns from the row-chunk partial sums, and w u = gam sum_i conj(u_i) (A u)_i from the row
// sums (the same bits in every workgroup); the new column k + 1 also goes to `col`.
constexpr int HU_R = 128;
__global__ __launch_bounds__(256) void k_hh_update(zd* A, int n, int k, const zd* u, const double* gam,
                                                   const zd* y, const zd* part, int nrc, zd* col) {
  __shared__ double sh[2][4];
  __shared__ zd ws[64];
  const int t = threadIdx.x, lane = t & 63, rg = t >> 6;
  const double g = gam[0];
  double a = 0, b = 0;
  for (int i = k + 1 + t; i < n; i += 256) {
    const zd p = zcmul(u[i], y[i]);
    a += p.x;
    b += p.y;
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_down(a, o, 64);
    b += __shfl_down(b, o, 64);
  }
  if (lane == 0) {
    sh[0][rg] = a;
    sh[1][rg] = b;
  }
  const int j = k + 1 + blockIdx.x * 64 + lane;
  if (rg == 0) {
    zd s = zmk(0, 0);
    if (j < n)
      for (int q = 0; q < nrc; ++q) s = zadd(s, part[(long long)q * n + j]);
    ws[lane] = zscale(s, g);
  }
  __syncthreads();
  const zd wu = zscale(zmk(sh[0][0] + sh[0][1] + sh[0][2] + sh[0][3], sh[1][0] + sh[1][1] + sh[1][2] + sh[1][3]), g);
  if (j >= n) return;
  const zd wj = ws[lane], cu = zconj(u[j]);
  const int i0 = blockIdx.y * HU_R, i1 = i0 + HU_R < n ? i0 + HU_R : n;
  for (int i = i0 + rg; i < i1; i += 4) {
    const zd ui = u[i];
    const zd yi = zscale(zsub(y[i], zmul(ui, wu)), g);
    const long long e = (long long)i * n + j;
    const zd v = zsub(zsub(A[e], zmul(ui, wj)), zmul(yi, cu));
    A[e] = v;
    if (j == k + 1) col[i] = v;
  }
}

// Compact WY form of a block of nb reflectors (Schreiber and Van Loan): H_0 H_1 ... H_{nb-1} =
// I - V T V^H with T upper triangular, T_ii = gam_i and T[0:i, i] = -gam_i T[0:i, 0:i] (V^H v_i).
// gr holds V^H V (row stride WYB), staged in LDS; one wave (lane j: row j of T), column i of T
// after column i - 1.
__global__ __launch_bounds__(64) void k_wy_t(const zd* gr, const double* gb, int nb, zd* tb) {
  __shared__ zd Ts[WYB * (WYB + 1)];
  __shared__ zd Gs[WYB * (WYB + 1)];
  const int j = threadIdx.x;
  for (int e = j; e < WYB * WYB; e += 64) {
    const int r = e / WYB, c = e % WYB;
    Ts[r * (WYB + 1) + c] = zmk(0, 0);
    Gs[r * (WYB + 1) + c] = (r < nb && c < nb) ? gr[e] : zmk(0, 0);
  }
  __syncthreads();
  for (int i = 0; i < nb; ++i) {
    const double gi = gb[i];
    if (j < i) {
      zd acc = zmk(0, 0);
      for (int l = j; l < i; ++l) acc = zadd(acc, zmul(Ts[j * (WYB + 1) + l], Gs[l * (WYB + 1) + i]));
      Ts[j * (WYB + 1) + i] = zscale(acc, -gi);
    }
    if (j == i) Ts[i * (WYB + 1) + i] = zmk(gi, 0);
    __syncthreads();
  }
  for (int e = j; e < WYB * WYB; e += 64) tb[e] = Ts[(e / WYB) * (WYB + 1) + e % WYB];
}

static int gridN(long long len) {
  long long nb = (len + 255) / 256;
  if (nb > 16384) nb = 16384;
  return (int)(nb < 1 ? 1 : nb);
}

// y holds the n row sums.  The reflectors reach Z in blocks of WYB: with V (n x nb, row stride WYB; rows
// <= k0 are zero) and T from k_wy_t, Z <- Z - ((Z V) T) V^H.  The products over the rows of V are
// split into NBK row chunks (batches summed through the workspace) so that they fill the chip.
struct WyBufs {
  zd* vb;    // n x WYB
  double* gb;  // WYB
  zd* gr;    // WYB x WYB
  zd* tb;    // WYB x WYB
  zd* w1;    // n x WYB
  zd* w2;    // n x WYB
  zd* ws;    // split-K partials
  long long ws_bytes;
};
static constexpr int WY_NBK = 8;
static long long wy_ws_bytes(int n) {
  const long long a = gemm_ws_bytes(PREC_F64, n, WYB, WY_NBK), b = gemm_ws_bytes(PREC_F64, WYB, WYB, WY_NBK);
  return a > b ? a : b;
}
static int wy_flush(zd* Z, int n, int k0, int nb, const WyBufs& wy, hipStream_t st) {
  // rows s0 .. n-1 of V: from k0 + 1, extended downwards over zero rows to a multiple of WY_NBK
  int nbk = WY_NBK;
  int kr = n - (k0 + 1);
  int s0 = n - ((kr + nbk - 1) / nbk) * nbk;
  if (s0 < 0) {
    nbk = 1;
    s0 = k0 + 1;
  }
  const int kt = n - s0, kc = kt / nbk;
  const zd* V = wy.vb + (long long)s0 * WYB;
  GemmDesc g;  // V^H V
  g.M = nb; g.N = nb; g.K = kc; g.nbatch = nbk;
  g.A = V; g.lda = WYB; g.sA = (long long)kc * WYB; g.opA = OP_C;
  g.B = V; g.ldb = WYB; g.sB = (long long)kc * WYB; g.opB = OP_N;
  g.C = wy.gr; g.ldc = WYB; g.ws = wy.ws; g.ws_bytes = wy.ws_bytes;
  if (gemm(PREC_F64, g, st)) return -4;
  hipLaunchKernelGGL(k_wy_t, dim3(1), dim3(64), 0, st, (const zd*)wy.gr, (const double*)wy.gb, nb, wy.tb);
  GemmDesc h;  // W1 = Z[:, s0:] V
  h.M = n; h.N = nb; h.K = kc; h.nbatch = nbk;
  h.A = Z + s0; h.lda = n; h.sA = kc; h.opA = OP_N;
  h.B = V; h.ldb = WYB; h.sB = (long long)kc * WYB; h.opB = OP_N;
  h.C = wy.w1; h.ldc = WYB; h.ws = wy.ws; h.ws_bytes = wy.ws_bytes;
  if (gemm(PREC_F64, h, st)) return -4;
  GemmDesc q;  // W2 = W1 T
  q.M = n; q.N = nb; q.K = nb;
  q.A = wy.w1; q.lda = WYB; q.opA = OP_N;
  q.B = wy.tb; q.ldb = WYB; q.opB = OP_N;
  q.C = wy.w2; q.ldc = WYB;
  if (gemm(PREC_F64, q, st)) return -4;
  GemmDesc z;  // Z[:, s0:] -= W2 V^H
  z.M = n; z.N = kt; z.K = nb;
  z.A = wy.w2; z.lda = WYB; z.opA = OP_N;
  z.B = V; z.ldb = WYB; z.opB = OP_C;
  z.C = Z + s0; z.ldc = n; z.ar = -1.0; z.beta = 1;
  return gemm(PREC_F64, z, st) ? -4 : 0;
}

static int hessenberg(zd* A, zd* Z, int n, zd* u, double* gam, zd* part, zd* col, zd* y, const WyBufs& wy,
                      hipStream_t st) {
  const int nrc = 16;
  int k0 = 0;
  hipLaunchKernelGGL(k_hh_col0, dim3((n + 255) / 256), dim3(256), 0, st, (const zd*)A, n, col);
  for (int k = 0; k + 2 < n; ++k) {
    const int rows = n - k - 1;
    const int rchunk = (rows + nrc - 1) / nrc;
    const int ncb = (rows + 63) / 64;
    hipLaunchKernelGGL(k_hh_pass1, dim3(ncb * nrc + (n + 3) / 4), dim3(256), 0, st, A, n, k, (const zd*)col, rchunk,
                       ncb, nrc, part, y, u, gam, wy.vb, k - k0, wy.gb);
    hipLaunchKernelGGL(k_hh_update, dim3(ncb, (n + HU_R - 1) / HU_R), dim3(256), 0, st, A, n, k, (const zd*)u,
                       (const double*)gam, (const zd*)y, (const zd*)part, nrc, col);
    if (k - k0 + 1 == WYB || k + 3 >= n) {
      if (wy_flush(Z, n, k0, k - k0 + 1, wy, st)) return -4;
      k0 = k + 1;
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ------------------------------------------------------------------ QR iteration -------------
__global__ void k_identity(zd* Z, int n) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    long long i = t / n, j = t % n;
    Z[t] = (i == j) ? zmk(1, 0) : zmk(0, 0);
  }
}
__global__ void k_extract_diag_sub(const zd* A, int n, zd* out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    out[i] = A[(long long)i * n + i];
    out[n + i] = (i + 1 < n) ? A[(long long)(i + 1) * n + i] : zmk(0, 0);
  }
}
__global__ void k_set_zero(zd* A, long long idx) { A[idx] = zmk(0, 0); }
__global__ void k_zero_lower(zd* A, int n) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    long long i = t / n, j = t % n;
    if (i > j) A[t] = zmk(0, 0);
  }
}
__global__ void k_zero_int(int* p, int cnt) {
  int i = threadIdx.x;
  if (i < cnt) p[i] = 0;
}

// Shifts for a sweep: eigenvalues of the trailing ns x ns block (rows/cols [lo, lo+ns)).
// exceptional != 0: ad hoc shifts around the last diagonal entry.
__global__ __launch_bounds__(64) void k_shifts(const zd* A, int n, int lo, int ns, int exceptional,
                                                zd* shifts) {
  __shared__ zd Hs[64 * LDM];
  const int t = threadIdx.x;
  for (int i = 0; i < ns; ++i)
    for (int j = t; j < ns; j += 64) Hs[i * LDM + j] = A[(long long)(lo + i) * n + lo + j];
  __syncthreads();
  if (exceptional) {
    zd d = Hs[(ns - 1) * LDM + ns - 1];
    double sc = cabs1(A[(long long)(lo + ns - 1) * n + lo + ns - 2]) + cabs1(Hs[(ns - 1) * LDM + ns - 2]);
    if (t < ns) {
      double th = 6.283185307179586 * (t + 0.5) / ns;
      shifts[t] = zadd(d, zmk(0.75 * sc * cos(th), 0.75 * sc * sin(th)));
    }
    return;
  }
  int rc = qr_lds(Hs, nullptr, ns, 0);
  if (t < ns) shifts[t] = Hs[t * LDM + t];
  (void)rc;
}

// Broadcast lane l's value of a double to the whole wave (l uniform): v_readlane into scalars.
__device__ inline double bcast(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane((int)v, l);
  const int hi = __builtin_amdgcn_readlane((int)(v >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

typedef double v4d_t __attribute__((ext_vector_type(4)));

// One wave accumulates a 16 x 16 complex tile C = sum_k A(i, k) B(k, j) over k < K (K padded
// to a multiple of 4 with zeros by the caller) with FP64 MFMA; A(i, k) and B(k, j) are read from
// LDS through the accessors.  Accumulator layout: lane l, register r holds row 4r + l/16,
// column l % 16.
template <typename FA, typename FB>
__device__ inline void tile16_mfma(FA getA, FB getB, int K, v4d_t& cr, v4d_t& ci) {
  const int lane = threadIdx.x & 63;
  const int i = lane & 15, kk = lane >> 4;
  for (int k0 = 0; k0 < K; k0 += 4) {
    zd a = getA(i, k0 + kk);
    zd b = getB(k0 + kk, i);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, ci, 0, 0, 0);
  }
}

// rows [rp, rp+bwp) x columns [c0, c1] of A <- U^H (those rows), 64 columns at a time, by a
// workgroup of CHASE_T threads: U in Ul (row stride LDM), the columns in Xs (row stride LDM);
// wave w computes output rows 16 (w & 3) .. +15 and columns 16 (w >> 2) .. +15 of each 32-column
// half.  Ends with a barrier, so the caller may reuse Ul and Xs.
__device__ inline void left_update_block(zd* A, int n, int rp, int bwp, int c0, int c1, const zd* U, zd* Ul,
                                         zd* Xs) {
  const int t = threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  for (int e = t; e < WIN * WIN; e += CHASE_T) {
    const int i = e >> 6, j = e & 63;
    Ul[i * LDM + j] = (i < bwp && j < bwp) ? U[i * WIN + j] : zmk(0, 0);
  }
  for (int cb = c0; cb <= c1; cb += 64) {
    for (int e = t; e < WIN * 64; e += CHASE_T) {
      const int i = e >> 6, c = e & 63;
      Xs[i * LDM + c] = (i < bwp && cb + c <= c1) ? A[(long long)(rp + i) * n + cb + c] : zmk(0, 0);
    }
    __syncthreads();
    const int ro = 16 * (w & 3);
    if (ro < bwp) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int co = 32 * h + 16 * (w >> 2);
        if (cb + co > c1) continue;
        v4d_t cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
        const int Kp = (bwp + 3) & ~3;
        tile16_mfma([&](int i, int k) { return zconj(Ul[k * LDM + ro + i]); },
                    [&](int k, int j) { return Xs[k * LDM + co + j]; }, Kp, cr, ci);
        for (int q = 0; q < 4; ++q) {
          const int row = ro + 4 * q + (lane >> 4), col = cb + co + (lane & 15);
          if (row < bwp && col <= c1) A[(long long)(rp + row) * n + col] = zmk(cr[q], ci[q]);
        }
      }
    }
    __syncthreads();
  }
}

// Chase the bulge chain through window rows/cols [r, r+bw).  All bulges move in lockstep: at
// step t bulge b rotates at pair P0 + t - 2b (front bulge first in the equivalent sequential
// order).  Rotations of one step act on disjoint row pairs and disjoint column pairs, and a
// bulge's parameters only read entries that the other bulges of the same step do not touch.
//
// Bulge b belongs to wave b % 8 for the whole chase: lane b / 8 of that wave computes the
// rotation, v_readlane hands it to the wave in scalar registers, and the same wave applies the
// row rotation (lane = column) and then the column rotation of the window and of the window
// unitary (lane = row).  The parameters of a bulge read rows q, q+1, which no other bulge's row
// rotation of the same step writes, so one step needs a barrier only between the row and the
// column rotations (other bulges' rows meet this bulge's columns) and at its end.
//
// The launch also finishes the left update of the previous window of the sweep (unitary Up, rows
// [rp, rp+bwp); none if Up is null): workgroup 0 applies it to the columns this window adds,
// [rp+bwp, r+bw), before loading the window; workgroups 1 .. apply it to 64 columns each from
// r+bw up to ihi, which this window does not touch.
__global__ __launch_bounds__(CHASE_T) void k_chase(zd* A, int n, int ilo, int ihi, int r, int bw,
                                                const zd* shifts, int ns, int* cnt, zd* Uout, const zd* Up,
                                                int rp, int bwp) {
  __shared__ zd Hs[WIN * LDM];
  __shared__ zd Us[WIN * LDM];
  constexpr int NWV = CHASE_T / 64;                // waves
  constexpr int BPW = (NSCAP + NWV - 1) / NWV;  // bulges per wave
  const int t = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = t & 63;
  if (blockIdx.x > 0) {
    const int c0 = r + bw + 64 * (blockIdx.x - 1);
    const int c1 = c0 + 63 < ihi ? c0 + 63 : ihi;
    if (Up && c0 <= c1) left_update_block(A, n, rp, bwp, c0, c1, Up, Us, Hs);
    return;
  }
  {
    // The window and the operands of the prologue (the previous window's unitary and the columns
    // [c0p, c1p] this window adds, rows [rp, rp+bwp)) are loaded together.  The prologue's
    // results land in Hs for the rows inside the window and in A for the rows above it; the
    // window entries they replace are not stored from v.
    const int c1p = r + bw - 1;
    const int c0p = Up ? rp + bwp : c1p + 1;  // empty range without a previous window
    zd v[WIN * WIN / CHASE_T];
#pragma unroll
    for (int k = 0; k < WIN * WIN / CHASE_T; ++k) {
      const int e = t + CHASE_T * k, i = e >> 6, j = e & 63;
      v[k] = (i < bw && j < bw) ? A[(long long)(r + i) * n + r + j] : zmk(0, 0);
    }
    v4d_t pr[2], pi[2];
    const int ro = 16 * (w & 3);
    if (c0p <= c1p) {
      for (int e = t; e < WIN * WIN; e += CHASE_T) {
        const int i = e >> 6, j = e & 63;
        Us[i * LDM + j] = (i < bwp && j < bwp) ? Up[i * WIN + j] : zmk(0, 0);
        Hs[i * LDM + j] = (i < bwp && c0p + j <= c1p) ? A[(long long)(rp + i) * n + c0p + j] : zmk(0, 0);
      }
      __syncthreads();
      const int Kp = (bwp + 3) & ~3;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        pr[h] = v4d_t{0, 0, 0, 0};
        pi[h] = v4d_t{0, 0, 0, 0};
        const int co = 32 * h + 16 * (w >> 2);
        if (ro < bwp && c0p + co <= c1p)
          tile16_mfma([&](int i, int k) { return zconj(Us[k * LDM + ro + i]); },
                      [&](int k, int j) { return Hs[k * LDM + co + j]; }, Kp, pr[h], pi[h]);
      }
      __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < WIN * WIN / CHASE_T; ++k) {
      const int e = t + CHASE_T * k, i = e >> 6, j = e & 63;
      const bool repl = (r + i < rp + bwp) && (r + j >= c0p);
      if (!repl) Hs[i * LDM + j] = v[k];
      Us[i * LDM + j] = (i == j) ? zmk(1, 0) : zmk(0, 0);
    }
    if (c0p <= c1p && ro < bwp) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int co = 32 * h + 16 * (w >> 2);
        if (c0p + co > c1p) continue;
        for (int q = 0; q < 4; ++q) {
          const int row = rp + ro + 4 * q + (lane >> 4), col = c0p + co + (lane & 15);
          if (row >= rp + bwp || col > c1p) continue;
          const zd val = zmk(pr[h][q], pi[h][q]);
          if (row >= r)
            Hs[(row - r) * LDM + (col - r)] = val;
          else
            A[(long long)row * n + col] = val;
        }
      }
    }
  }
  // lane u < BPW of wave w owns bulge b = w + NWV u: its shift and its next pair
  const int myb = w + NWV * lane;
  const bool own = lane < BPW && myb < ns;
  zd sh = zmk(0, 0);
  int nxt = 0;
  if (own) {
    sh = shifts[myb];
    nxt = ilo + cnt[myb];
  }
  const int P0 = ilo + cnt[0];
  __syncthreads();
  const bool at_end = (r + bw - 1 >= ihi);
  const int pmax = at_end ? ihi - 1 : r + bw - 3;
  const int pmin = (r == ilo) ? ilo : r + 1;
  const int plim = pmax < ihi - 1 ? pmax : ihi - 1;
  const int t_end = at_end ? (ihi - 1 - (P0 - 2 * (ns - 1))) : (pmax - P0);
  for (int step = 0; step <= t_end; ++step) {
    // parameters of this wave's bulges (lane u: bulge w + 4u)
    double cs = 1.0;
    zd sn = zmk(0, 0);
    int q = -1;
    if (own) {
      const int p = P0 + step - 2 * myb;
      if (p >= ilo && p >= pmin && p <= plim) {
        q = p - r;
        zd f, g, rr;
        if (p == ilo) {
          f = zsub(Hs[q * LDM + q], sh);
          g = Hs[(q + 1) * LDM + q];
        } else {
          f = Hs[q * LDM + q - 1];
          g = Hs[(q + 1) * LDM + q - 1];
        }
        zlartg(f, g, cs, sn, rr);
        nxt = p + 1;
      }
    }
    double bc[BPW], bsr[BPW], bsi[BPW];
    int bq[BPW];
#pragma unroll
    for (int u = 0; u < BPW; ++u) {
      bq[u] = __builtin_amdgcn_readlane(q, u);
      bc[u] = bcast(cs, u);
      bsr[u] = bcast(sn.x, u);
      bsi[u] = bcast(sn.y, u);
    }
    // row rotations: rows q, q+1 from column c0 (q, or q-1 with the chased entry zeroed)
    {
      zd x[BPW], y[BPW];
#pragma unroll
      for (int u = 0; u < BPW; ++u) {
        const int qq = bq[u];
        const int c0 = (qq >= 0 && r + qq == ilo) ? qq : qq - 1;
        if (qq >= 0 && lane >= c0 && lane < bw) {
          x[u] = Hs[qq * LDM + lane];
          y[u] = Hs[(qq + 1) * LDM + lane];
        }
      }
#pragma unroll
      for (int u = 0; u < BPW; ++u) {
        const int qq = bq[u];
        const bool first = (qq >= 0 && r + qq == ilo);
        const int c0 = first ? qq : qq - 1;
        if (qq >= 0 && lane >= c0 && lane < bw) {
          const zd sv = zmk(bsr[u], bsi[u]);
          Hs[qq * LDM + lane] = zadd(zscale(x[u], bc[u]), zmul(sv, y[u]));
          Hs[(qq + 1) * LDM + lane] =
              (!first && lane == qq - 1) ? zmk(0, 0) : zsub(zscale(y[u], bc[u]), zmul(zconj(sv), x[u]));
        }
      }
    }
    __syncthreads();
    // column rotations: columns q, q+1 of the window (rows <= q+2) and of the window unitary
    {
      zd hx[BPW], hy[BPW], ux[BPW], uy[BPW];
#pragma unroll
      for (int u = 0; u < BPW; ++u) {
        const int qq = bq[u];
        if (qq >= 0) {
          if (lane <= qq + 2 && lane < bw) {
            hx[u] = Hs[lane * LDM + qq];
            hy[u] = Hs[lane * LDM + qq + 1];
          }
          if (lane < bw) {
            ux[u] = Us[lane * LDM + qq];
            uy[u] = Us[lane * LDM + qq + 1];
          }
        }
      }
#pragma unroll
      for (int u = 0; u < BPW; ++u) {
        const int qq = bq[u];
        if (qq >= 0) {
          const zd sv = zmk(bsr[u], bsi[u]);
          const double c = bc[u];
          if (lane <= qq + 2 && lane < bw) {
            Hs[lane * LDM + qq] = zadd(zscale(hx[u], c), zmul(zconj(sv), hy[u]));
            Hs[lane * LDM + qq + 1] = zsub(zscale(hy[u], c), zmul(sv, hx[u]));
          }
          if (lane < bw) {
            Us[lane * LDM + qq] = zadd(zscale(ux[u], c), zmul(zconj(sv), uy[u]));
            Us[lane * LDM + qq + 1] = zsub(zscale(uy[u], c), zmul(sv, ux[u]));
          }
        }
      }
    }
    __syncthreads();
  }
  if (own) cnt[myb] = nxt - ilo;
#pragma unroll
  for (int k = 0; k < WIN * WIN / CHASE_T; ++k) {
    const int e = t + CHASE_T * k, i = e >> 6, j = e & 63;
    if (i < bw && j < bw) {
      A[(long long)(r + i) * n + r + j] = Hs[i * LDM + j];
      Uout[i * WIN + j] = Us[i * LDM + j];
    }
  }
}

// One wave loads the m x m diagonal block of A at (r0, r0) into Hs (row stride LDM) and sets Us
// to the identity; loads are issued 16 rows at a time before their LDS stores.
__device__ inline void load_window(const zd* A, int n, int r0, int m, zd* Hs, zd* Us) {
  const int t = threadIdx.x & 63;
  for (int i0 = 0; i0 < m; i0 += 16) {
    zd v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = i0 + k;
      v[k] = (i < m && t < m) ? A[(long long)(r0 + i) * n + r0 + t] : zmk(0, 0);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int i = i0 + k;
      if (i < m && t < m) {
        Hs[i * LDM + t] = v[k];
        Us[i * LDM + t] = (i == t) ? zmk(1, 0) : zmk(0, 0);
      }
    }
  }
  __syncthreads();
}

// Aggressive early deflation on the trailing window [kw, ihi] (jw = ihi - kw + 1 <= 64 rows, kw
// above the first row of the active block, s = A[kw, kw-1] the entry that couples the window to
// the rest).  The window is brought to Schur form T = V^H W V in LDS; the coupling column then
// reads s V^H e_1, so the eigenvalue in position k of T decouples when |s| |V[0, k]| is below
// machine precision relative to |T[k, k]|.  Deflations are counted from the bottom of T up to the
// first one that fails the test (no reordering).  If none deflate, A is left unchanged.  Otherwise
// the undeflated leading part is returned to Hessenberg form: a reflector P maps s conj(V[0, :nu])
// to a multiple of e_1 (applied as P T P and V P), then Householder reduction of T[:nu, :nu]
// (applied to the rows' full width and accumulated into V); the window, the coupling column and V
// (into Uout, for the deferred updates outside the window) are written back.
// res[0] = deflated count, res[1] = 1 if A was changed, res[2] = status of the window QR.
// ritz[0 .. jw) = diagonal of T; its first jw - res[0] entries are the undeflated eigenvalues.
__global__ __launch_bounds__(64) void k_aed(zd* A, int n, int kw, int ihi, zd* Uout, zd* ritz, int* res) {
  __shared__ zd Hs[WIN * LDM];
  __shared__ zd Us[WIN * LDM];
  __shared__ zd hv[WIN];
  __shared__ double red[2];
  __shared__ int nd_s;
  const double ulp = 2.220446049250313e-16;
  const int jw = ihi - kw + 1;
  const int t = threadIdx.x;
  const zd s = A[(long long)kw * n + kw - 1];
  load_window(A, n, kw, jw, Hs, Us);
  const int rc = qr_lds(Hs, Us, jw, 1);
  for (int i = 0; i < jw; ++i)
    for (int j = t; j < i; j += 64) Hs[i * LDM + j] = zmk(0, 0);
  __syncthreads();
  if (t == 0) {
    int nd = 0;
    if (rc == 0) {
      const double as = cabs1(s);
      for (int k = jw - 1; k >= 0; --k) {
        double foo = cabs1(Hs[k * LDM + k]);
        if (foo == 0.0) foo = as;
        if (as * cabs1(Us[k]) <= fmax(1e-300, ulp * foo)) ++nd;
        else break;
      }
    }
    nd_s = nd;
    res[0] = nd;
    res[1] = nd > 0 ? 1 : 0;
    res[2] = rc;
  }
  for (int i = t; i < jw; i += 64) ritz[i] = Hs[i * LDM + i];
  __syncthreads();
  const int nd = nd_s, nu = jw - nd;
  if (nd == 0) return;
  if (nu > 1) {
    // reflector P = I - 2 h h^H with P x = -ph |x| e_1, x = s conj(V[0, :nu])
    if (t == 0) {
      double nx2 = 0;
      for (int i = 0; i < nu; ++i) nx2 += zabs2(Us[i]);
      const double nx = sqrt(nx2) * sqrt(zabs2(s));
      const zd x0 = zmul(s, zconj(Us[0]));
      const double ax0 = sqrt(zabs2(x0));
      const zd ph = ax0 > 0 ? zscale(x0, 1.0 / ax0) : zmk(1, 0);
      red[0] = nx;
      // |v|^2 = |x|^2 + 2 |x0| |x| + |x|^2
      red[1] = 1.0 / sqrt(2.0 * nx * (nx + ax0));
      hv[0] = zadd(x0, zscale(ph, nx));
    }
    __syncthreads();
    for (int i = t + 1; i < nu; i += 64) hv[i] = zmul(s, zconj(Us[i]));
    __syncthreads();
    for (int i = t; i < nu; i += 64) hv[i] = zscale(hv[i], red[1]);
    __syncthreads();
    // T[:nu, :] = P T[:nu, :]   (lane = column)
    for (int j = t; j < jw; j += 64) {
      zd w = zmk(0, 0);
      for (int i = 0; i < nu; ++i) w = zadd(w, zcmul(hv[i], Hs[i * LDM + j]));
      w = zscale(w, 2.0);
      for (int i = 0; i < nu; ++i) Hs[i * LDM + j] = zsub(Hs[i * LDM + j], zmul(hv[i], w));
    }
    __syncthreads();
    // T[:nu, :nu] = T[:nu, :nu] P and V[:, :nu] = V[:, :nu] P   (lane = row)
    for (int i = t; i < jw; i += 64) {
      zd y = zmk(0, 0), yv = zmk(0, 0);
      for (int j = 0; j < nu; ++j) {
        if (i < nu) y = zadd(y, zmul(Hs[i * LDM + j], hv[j]));
        yv = zadd(yv, zmul(Us[i * LDM + j], hv[j]));
      }
      y = zscale(y, 2.0);
      yv = zscale(yv, 2.0);
      for (int j = 0; j < nu; ++j) {
        if (i < nu) Hs[i * LDM + j] = zsub(Hs[i * LDM + j], zmul(y, zconj(hv[j])));
        Us[i * LDM + j] = zsub(Us[i * LDM + j], zmul(yv, zconj(hv[j])));
      }
    }
    __syncthreads();
    // Householder reduction of T[:nu, :nu] to Hessenberg form.  The column norm is a wave
    // reduction (every lane holds the result); the sums of the two updates run on four
    // independent accumulators to shorten their dependency chains.
    for (int k = 0; k + 2 < nu; ++k) {
      __syncthreads();
      // the part below x0 on its own (see hh_scalars)
      double tail = (t > k + 1 && t < nu) ? zabs2(Hs[t * LDM + k]) : 0.0;
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) tail += __shfl_xor(tail, o, 64);
      tail = __shfl(tail, 0, 64);  // one value for the whole wave: the branch below is uniform
      const zd x0 = Hs[(k + 1) * LDM + k];
      const double ax0 = sqrt(zabs2(x0));
      const double nrm2 = zabs2(x0) + tail;
      const double gam = tail > 0 ? 1.0 / (sqrt(nrm2) * (sqrt(nrm2) + ax0)) : 0.0;  // I - gam u u^H
      if (gam != 0.0) {
        const double nrm = sqrt(nrm2);
        const zd ph = ax0 > 0 ? zscale(x0, 1.0 / ax0) : zmk(1, 0);
        if (t == 0) {
          hv[k + 1] = zadd(x0, zscale(ph, nrm));
          red[1] = -nrm;
          hv[0] = ph;
        }
        for (int i = k + 2 + t; i < nu; i += 64) hv[i] = Hs[i * LDM + k];
        __syncthreads();
        // rows k+1 .. nu-1, columns k+1 .. jw-1 from the left
        for (int j = k + 1 + t; j < jw; j += 64) {
          zd w0 = zmk(0, 0), w1 = zmk(0, 0), w2 = zmk(0, 0), w3 = zmk(0, 0);
          int i = k + 1;
          for (; i + 3 < nu; i += 4) {
            w0 = zadd(w0, zcmul(hv[i], Hs[i * LDM + j]));
            w1 = zadd(w1, zcmul(hv[i + 1], Hs[(i + 1) * LDM + j]));
            w2 = zadd(w2, zcmul(hv[i + 2], Hs[(i + 2) * LDM + j]));
            w3 = zadd(w3, zcmul(hv[i + 3], Hs[(i + 3) * LDM + j]));
          }
          for (; i < nu; ++i) w0 = zadd(w0, zcmul(hv[i], Hs[i * LDM + j]));
          const zd w = zscale(zadd(zadd(w0, w1), zadd(w2, w3)), gam);
          for (i = k + 1; i < nu; ++i) Hs[i * LDM + j] = zsub(Hs[i * LDM + j], zmul(hv[i], w));
        }
        __syncthreads();
        // columns k+1 .. nu-1 from the right: rows 0 .. nu-1 of T, all rows of V
        for (int i = t; i < jw; i += 64) {
          zd y0 = zmk(0, 0), y1 = zmk(0, 0), v0 = zmk(0, 0), v1 = zmk(0, 0);
          int j = k + 1;
          for (; j + 1 < nu; j += 2) {
            if (i < nu) {
              y0 = zadd(y0, zmul(Hs[i * LDM + j], hv[j]));
              y1 = zadd(y1, zmul(Hs[i * LDM + j + 1], hv[j + 1]));
            }
            v0 = zadd(v0, zmul(Us[i * LDM + j], hv[j]));
            v1 = zadd(v1, zmul(Us[i * LDM + j + 1], hv[j + 1]));
          }
          if (j < nu) {
            if (i < nu) y0 = zadd(y0, zmul(Hs[i * LDM + j], hv[j]));
            v0 = zadd(v0, zmul(Us[i * LDM + j], hv[j]));
          }
          const zd y = zscale(zadd(y0, y1), gam);
          const zd yv = zscale(zadd(v0, v1), gam);
          for (j = k + 1; j < nu; ++j) {
            if (i < nu) Hs[i * LDM + j] = zsub(Hs[i * LDM + j], zmul(y, zconj(hv[j])));
            Us[i * LDM + j] = zsub(Us[i * LDM + j], zmul(yv, zconj(hv[j])));
          }
        }
        __syncthreads();
        if (t == 0) Hs[(k + 1) * LDM + k] = zscale(hv[0], red[1]);
        for (int i = k + 2 + t; i < nu; i += 64) Hs[i * LDM + k] = zmk(0, 0);
        __syncthreads();
      }
    }
  }
  // write back: Hessenberg part T[:nu, :nu], triangular rest, the coupling column
  for (int i = 0; i < jw; ++i)
    for (int j = t; j < jw; j += 64) {
      const bool keep = (j >= i) || (j == i - 1 && i < nu);
      A[(long long)(kw + i) * n + kw + j] = keep ? Hs[i * LDM + j] : zmk(0, 0);
      Uout[i * WIN + j] = Us[i * LDM + j];
    }
  for (int i = t; i < jw; i += 64)
    A[(long long)(kw + i) * n + kw - 1] = (i == 0 && nu > 0) ? zmul(s, zconj(Us[0])) : zmk(0, 0);
}

// Finish an active block [lo, hi] (size <= 64) in LDS: Schur form of the block, unitary to Uout.
__global__ __launch_bounds__(64) void k_small_block(zd* A, int n, int lo, int hi, zd* Uout, int* info) {
  __shared__ zd Hs[WIN * LDM];
  __shared__ zd Us[WIN * LDM];
  const int m = hi - lo + 1;
  const int t = threadIdx.x;
  load_window(A, n, lo, m, Hs, Us);
  int rc = qr_lds(Hs, Us, m, 1);
  if (t == 0) info[0] = rc;
  for (int i = 0; i < m; ++i)
    for (int j = t; j < m; j += 64) {
      A[(long long)(lo + i) * n + lo + j] = (i > j) ? zmk(0, 0) : Hs[i * LDM + j];
      Uout[i * WIN + j] = Us[i * LDM + j];
    }
}

// Window unitary `win` of a list (bw x bw, zero-padded to WIN x WIN) through registers: thread t
// holds entries t + 256 k, k < 16.
__device__ inline void load_unitary(const zd* Ubuf, const WinList& wl, int win, int t, zd ru[16]) {
  const zd* U = Ubuf + (long long)win * WIN * WIN;
  const int bw = wl.bw[win];
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = t + 256 * k;
    const int i = e >> 6, j = e & 63;
    ru[k] = (i < bw && j < bw) ? U[i * WIN + j] : zmk(0, 0);
  }
}
__device__ inline void store_unitary(zd* Ul, int t, const zd ru[16]) {
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    const int e = t + 256 * k;
    Ul[(e >> 6) * LDM + (e & 63)] = ru[k];
  }
}

// Deferred right updates: for each window w in order, rows i of X (i < limit_w) get
// X[i, r_w : r_w+bw_w] <- X[i, r_w : r_w+bw_w] U_w.  limit_w = r_w (mode 1) or nrows (mode 0).
// One workgroup per 16 rows (first row rb); wave w owns output columns 16w .. 16w+15.
__device__ inline void right_apply_rows(zd* X, int ldx, int nrows, const WinList& wl, const zd* Ubuf, int mode,
                                        int rb, zd* Ul, zd* Xs) {
  const int t = threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  // the windows a block takes part in form a suffix of the list (the window origins increase)
  int win0 = 0;
  if (mode)
    while (win0 < wl.nwin && rb >= wl.r[win0]) ++win0;
  if (win0 >= wl.nwin) return;  // uniform over the block
  // the next window's unitary is loaded into registers while the current one is applied
  zd ru[16];
  load_unitary(Ubuf, wl, win0, t, ru);
  for (int win = win0; win < wl.nwin; ++win) {
    const int r = wl.r[win], bw = wl.bw[win];
    const int lim = mode ? r : nrows;
    __syncthreads();
    store_unitary(Ul, t, ru);
    for (int e = t; e < 16 * WIN; e += 256) {
      int i = e >> 6, j = e & 63;
      int row = rb + i;
      Xs[i * LDM + j] = (row < lim && j < bw) ? X[(long long)row * ldx + r + j] : zmk(0, 0);
    }
    __syncthreads();
    if (win + 1 < wl.nwin) load_unitary(Ubuf, wl, win + 1, t, ru);
    if (16 * w < bw) {
      v4d_t cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
      const int Kp = (bw + 3) & ~3;
      tile16_mfma([&](int i, int k) { return Xs[i * LDM + k]; },
                  [&](int k, int j) { return Ul[k * LDM + 16 * w + j]; }, Kp, cr, ci);
      for (int q = 0; q < 4; ++q) {
        const int row = rb + 4 * q + (lane >> 4), col = 16 * w + (lane & 15);
        if (row < lim && col < bw) X[(long long)row * ldx + r + col] = zmk(cr[q], ci[q]);
      }
    }
  }
}

// Deferred left updates of the columns right of the active block: columns (hi, n), 16 per
// workgroup from column cb; wave w owns output rows 16w .. 16w+15 of each window.
__device__ inline void left_apply_cols(zd* A, int n, const WinList& wl, const zd* Ubuf, int cb, zd* Ul, zd* Xs) {
  const int t = threadIdx.x;
  const int w = t >> 6, lane = t & 63;
  if (wl.nwin <= 0) return;
  zd ru[16];
  load_unitary(Ubuf, wl, 0, t, ru);
  for (int win = 0; win < wl.nwin; ++win) {
    const int r = wl.r[win], bw = wl.bw[win];
    __syncthreads();
    store_unitary(Ul, t, ru);
    for (int e = t; e < WIN * 16; e += 256) {
      int i = e >> 4, c = e & 15;
      int col = cb + c;
      Xs[i * 17 + c] = (i < bw && col < n) ? A[(long long)(r + i) * n + col] : zmk(0, 0);
    }
    __syncthreads();
    if (win + 1 < wl.nwin) load_unitary(Ubuf, wl, win + 1, t, ru);
    if (16 * w < bw) {
      v4d_t cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
      const int Kp = (bw + 3) & ~3;
      tile16_mfma([&](int i, int k) { return zconj(Ul[k * LDM + 16 * w + i]); },
                  [&](int k, int j) { return Xs[k * 17 + j]; }, Kp, cr, ci);
      for (int q = 0; q < 4; ++q) {
        const int row = 16 * w + 4 * q + (lane >> 4), col = cb + (lane & 15);
        if (row < bw && col < n) A[(long long)(r + row) * n + col] = zmk(cr[q], ci[q]);
      }
    }
  }
}

static constexpr int XS_ELEMS = (16 * LDM > WIN * 17) ? 16 * LDM : WIN * 17;

__global__ __launch_bounds__(256) void k_right_apply_seq(zd* X, int ldx, int nrows, WinList wl, const zd* Ubuf,
                                                         int mode) {
  __shared__ zd Ul[WIN * LDM];
  __shared__ zd Xs[XS_ELEMS];
  right_apply_rows(X, ldx, nrows, wl, Ubuf, mode, blockIdx.x * 16, Ul, Xs);
}

// The two deferred updates of A in one launch (they touch disjoint parts of A): workgroups
// [0, nrb) update the rows above the windows, the others the columns right of the active block.
__global__ __launch_bounds__(256) void k_apply_seq_a(zd* A, int n, int nrb, int c0, WinList wl, const zd* Ubuf) {
  __shared__ zd Ul[WIN * LDM];
  __shared__ zd Xs[XS_ELEMS];
  if ((int)blockIdx.x < nrb)
    right_apply_rows(A, n, n, wl, Ubuf, 1, blockIdx.x * 16, Ul, Xs);
  else
    left_apply_cols(A, n, wl, Ubuf, c0 + (blockIdx.x - nrb) * 16, Ul, Xs);
}

// Deferred updates of one sweep (or one early deflation / small block).  Z is never read by the
// QR iteration, so its update runs on the side stream zs (ordered after the producers of the
// window unitaries by `ready`; `done` tells the next user of this Ubuf half that it may be
// overwritten); the updates of A stay on st.
static void apply_deferred(zd* A, zd* Z, int n, int hi, const WinList& wl, const zd* Ubuf, hipStream_t st,
                           hipStream_t zs, hipEvent_t ready, hipEvent_t done) {
  hipEventRecord(ready, st);
  hipStreamWaitEvent(zs, ready, 0);
  hipLaunchKernelGGL(k_right_apply_seq, dim3((n + 15) / 16), dim3(256), 0, zs, Z, n, n, wl, Ubuf, 0);
  hipEventRecord(done, zs);
  // A: rows above each window
  int maxr = 0;
  for (int w = 0; w < wl.nwin; ++w) maxr = wl.r[w] > maxr ? wl.r[w] : maxr;
  // and columns right of the active block, in one launch
  const int nrb = maxr > 0 ? (maxr + 15) / 16 : 0;
  const int ncb = hi + 1 < n ? (n - hi - 1 + 15) / 16 : 0;
  if (nrb + ncb > 0)
    hipLaunchKernelGGL(k_apply_seq_a, dim3(nrb + ncb), dim3(256), 0, st, A, n, nrb, hi + 1, wl, Ubuf);
}

static inline double h_cabs1(zd a) { return fabs(a.x) + fabs(a.y); }

int schur_factor(zd* A, zd* Z, int n, hipStream_t st, double* t_hess, double* t_qr) {
  return schur_factor_ex(A, Z, n, st, t_hess, t_qr, 0);
}

// mode bit 0: stop after the Hessenberg reduction; bits 8..15: early-deflation window (0: default,
// 1: none, otherwise 16 .. 64 rows); bits 16..23: window advance (0: default, else 8 .. 48);
// bits 24..30: most bulges per sweep (0: default, else 2 .. 23, and at most (63 - advance) / 2)
int schur_factor_ex(zd* A, zd* Z, int n, hipStream_t st, double* t_hess, double* t_qr, int mode) {
  const int stop_after_hessenberg = mode & 1;
  int aedw = (mode >> 8) & 255;
  if (aedw == 0) aedw = AEDW;
  if (aedw != 1 && (aedw < 16 || aedw > WIN)) return -1;
  int step = (mode >> 16) & 255;
  if (step == 0) step = STEP;
  int nsmax = (mode >> 24) & 127;
  if (nsmax == 0) nsmax = NSMAX;
  if (step < 8 || step > 48 || nsmax < 2 || nsmax > NSCAP || WIN < step + 2 * nsmax + 1) return -1;
  // at most MAXWIN windows per sweep
  while ((n + step - 1) / step + 2 > MAXWIN) ++step;
  if (WIN < step + 2 * nsmax + 1) nsmax = (WIN - 1 - step) / 2;
  if (nsmax < 2) return -1;
  if (n < 1) return -1;
  zd *u = nullptr, *part = nullptr, *w = nullptr, *y = nullptr, *Ubuf = nullptr, *shifts = nullptr, *ds = nullptr;
  hipStream_t zs = nullptr;
  hipEvent_t ev_ready[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
  double* gam = nullptr;
  int *cnt = nullptr, *info = nullptr;
  WyBufs wy{};
  const int nrc = 16;
  auto cleanup = [&]() {
    if (zs) hipStreamSynchronize(zs);
    for (int b = 0; b < 2; ++b) {
      if (ev_ready[b]) hipEventDestroy(ev_ready[b]);
      if (ev_done[b]) hipEventDestroy(ev_done[b]);
    }
    if (zs) hipStreamDestroy(zs);
    hipFree(u); hipFree(part); hipFree(w); hipFree(y); hipFree(Ubuf); hipFree(shifts); hipFree(ds);
    hipFree(gam); hipFree(cnt); hipFree(info);
    hipFree(wy.vb); hipFree(wy.gb); hipFree(wy.gr); hipFree(wy.tb); hipFree(wy.w1); hipFree(wy.w2); hipFree(wy.ws);
  };
  if (hipMalloc(&u, sizeof(zd) * n) != hipSuccess || hipMalloc(&part, sizeof(zd) * (size_t)nrc * n) != hipSuccess ||
      hipMalloc(&w, sizeof(zd) * n) != hipSuccess || hipMalloc(&y, sizeof(zd) * (2 * (size_t)n + (n + 255) / 256 + 1)) != hipSuccess ||
      hipMalloc(&Ubuf, sizeof(zd) * 2 * (size_t)MAXWIN * WIN * WIN) != hipSuccess ||
      hipMalloc(&shifts, sizeof(zd) * 2 * WIN) != hipSuccess || hipMalloc(&ds, sizeof(zd) * 2 * n) != hipSuccess ||
      hipMalloc(&gam, sizeof(double) * 4) != hipSuccess || hipMalloc(&cnt, sizeof(int) * 64) != hipSuccess ||
      hipMalloc(&info, sizeof(int) * 4) != hipSuccess || hipMalloc(&wy.vb, sizeof(zd) * (size_t)n * WYB) != hipSuccess ||
      hipMalloc(&wy.gb, sizeof(double) * WYB) != hipSuccess || hipMalloc(&wy.gr, sizeof(zd) * WYB * WYB) != hipSuccess ||
      hipMalloc(&wy.tb, sizeof(zd) * WYB * WYB) != hipSuccess || hipMalloc(&wy.w1, sizeof(zd) * (size_t)n * WYB) != hipSuccess ||
      hipMalloc(&wy.w2, sizeof(zd) * (size_t)n * WYB) != hipSuccess ||
      hipMalloc(&wy.ws, (size_t)(wy.ws_bytes = wy_ws_bytes(n) > 16 ? wy_ws_bytes(n) : 16)) != hipSuccess) {
    cleanup();
    return -5;
  }
  if (hipStreamCreateWithFlags(&zs, hipStreamNonBlocking) != hipSuccess) {
    zs = nullptr;
    cleanup();
    return -4;
  }
  for (int b = 0; b < 2; ++b) {
    if (hipEventCreateWithFlags(&ev_ready[b], hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ev_done[b], hipEventDisableTiming) != hipSuccess) {
      cleanup();
      return -4;
    }
    hipEventRecord(ev_done[b], zs);
  }
  // the window unitaries of consecutive deferred updates alternate between two halves of Ubuf,
  // so the side stream can still read one half while the next windows are written to the other
  int ub = 0;
  auto ubuf = [&]() {
    hipStreamWaitEvent(st, ev_done[ub], 0);
    return Ubuf + (long long)ub * MAXWIN * WIN * WIN;
  };
  auto deferred = [&](int hi, const WinList& wl, const zd* U) {
    apply_deferred(A, Z, n, hi, wl, U, st, zs, ev_ready[ub], ev_done[ub]);
    ub ^= 1;
  };
  auto t0 = std::chrono::steady_clock::now();
  hipLaunchKernelGGL(k_identity, dim3(gridN((long long)n * n)), dim3(256), 0, st, Z, n);
  const int hrc = n > 2 ? hessenberg(A, Z, n, u, gam, part, w, y, wy, st) : 0;
  hipStreamSynchronize(st);
  auto t1 = std::chrono::steady_clock::now();
  if (t_hess) *t_hess = std::chrono::duration<double>(t1 - t0).count();
  if (hrc || stop_after_hessenberg) {
    cleanup();
    return (hrc == 0 && hipGetLastError() == hipSuccess) ? 0 : -4;
  }

  const double ulp = 2.220446049250313e-16;
  std::vector<zd> hds(2 * (size_t)n);
  int ihi = n - 1;
  int stall = 0, sweeps = 0, last_ihi = -1, last_ilo = -1;
  int status = 0;
  const long long max_sweeps = 20LL * n / nsmax + 400;
  int hres[4] = {0, 0, 0, 0};
  while (ihi > 0) {
    hipLaunchKernelGGL(k_extract_diag_sub, dim3((n + 255) / 256), dim3(256), 0, st, A, n, ds);
    if (hipMemcpyAsync(hds.data(), ds, sizeof(zd) * 2 * n, hipMemcpyDeviceToHost, st) != hipSuccess) { status = -4; break; }
    if (hipStreamSynchronize(st) != hipSuccess) { status = -4; break; }
    auto negligible = [&](int i) {  // subdiagonal entry (i+1, i)
      double tst = h_cabs1(hds[i]) + h_cabs1(hds[i + 1]);
      return h_cabs1(hds[n + i]) <= fmax(ulp * tst, 1e-300);
    };
    while (ihi > 0 && negligible(ihi - 1)) {
      hipLaunchKernelGGL(k_set_zero, dim3(1), dim3(1), 0, st, A, (long long)ihi * n + ihi - 1);
      --ihi;
    }
    if (ihi <= 0) break;
    int ilo = ihi - 1;
    while (ilo > 0 && !negligible(ilo - 1)) --ilo;
    if (ilo > 0) hipLaunchKernelGGL(k_set_zero, dim3(1), dim3(1), 0, st, A, (long long)ilo * n + ilo - 1);
    if (ihi == last_ihi && ilo == last_ilo) ++stall; else stall = 0;
    last_ihi = ihi;
    last_ilo = ilo;
    int size = ihi - ilo + 1;
    WinList wl;
    if (size <= WIN) {
      zd* U = ubuf();
      hipLaunchKernelGGL(k_small_block, dim3(1), dim3(64), 0, st, A, n, ilo, ihi, U, info);
      wl.nwin = 1;
      wl.r[0] = ilo;
      wl.bw[0] = size;
      deferred(ihi, wl, U);
      int hinfo = 0;
      hipMemcpyAsync(&hinfo, info, sizeof(int), hipMemcpyDeviceToHost, st);
      hipStreamSynchronize(st);
      if (hinfo != 0) { status = -3; break; }
      ihi = ilo - 1;
      continue;
    }
    if (++sweeps > max_sweeps) { status = -3; break; }
    // aggressive early deflation on the trailing window; its undeflated eigenvalues are the
    // next sweep's shifts
    int ns = size / 8;
    if (ns > nsmax) ns = nsmax;
    if (ns < 2) ns = 2;
    const zd* sh = shifts + WIN;
    bool need_shifts = true;
    if (aedw > 1) {
      const int jw = aedw;
      const int kw = ihi - jw + 1;
      zd* U = ubuf();
      hipLaunchKernelGGL(k_aed, dim3(1), dim3(64), 0, st, A, n, kw, ihi, U, shifts, info + 1);
      if (hipMemcpyAsync(hres, info + 1, sizeof(int) * 3, hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) { status = -4; break; }
      const int nd = hres[0];
      if (hres[1]) {
        wl.nwin = 1;
        wl.r[0] = kw;
        wl.bw[0] = jw;
        deferred(ihi, wl, U);
      }
      if (nd > 0) stall = 0;
      // many deflations: look again before sweeping
      if (100 * nd > 20 * jw) continue;
      ihi -= nd;
      size = ihi - ilo + 1;
      if (size <= WIN) continue;
      ns = size / 8;
      if (ns > nsmax) ns = nsmax;
      if (ns < 2) ns = 2;
      const int nu = jw - nd;
      if (hres[2] == 0 && nu >= ns) {
        sh = shifts + (nu - ns);
        need_shifts = false;
      }
    }
    const int exceptional = (stall > 0 && stall % 8 == 0) ? 1 : 0;
    if (exceptional || need_shifts) {
      hipLaunchKernelGGL(k_shifts, dim3(1), dim3(64), 0, st, A, n, ihi - ns + 1, ns, exceptional, shifts + WIN);
      sh = shifts + WIN;
    }
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, st, cnt, 64);
    zd* U = ubuf();
    wl.nwin = 0;
    for (int r = ilo;; r += step) {
      int bw = ihi + 1 - r < WIN ? ihi + 1 - r : WIN;
      zd* Uw = U + (long long)wl.nwin * WIN * WIN;
      // the previous window's left update rides along (its right part on extra workgroups)
      const zd* Up = wl.nwin > 0 ? Uw - (long long)WIN * WIN : nullptr;
      const int rp = wl.nwin > 0 ? wl.r[wl.nwin - 1] : 0, bwp = wl.nwin > 0 ? wl.bw[wl.nwin - 1] : 0;
      const int nright = (Up && r + bw <= ihi) ? (ihi - (r + bw) + 1 + 63) / 64 : 0;
      hipLaunchKernelGGL(k_chase, dim3(1 + nright), dim3(CHASE_T), 0, st, A, n, ilo, ihi, r, bw, sh, ns, cnt, Uw, Up,
                         rp, bwp);
      wl.r[wl.nwin] = r;
      wl.bw[wl.nwin] = bw;
      ++wl.nwin;
      if (r + bw - 1 >= ihi) break;
    }
    deferred(ihi, wl, U);
  }
  if (status == 0) hipLaunchKernelGGL(k_zero_lower, dim3(gridN((long long)n * n)), dim3(256), 0, st, A, n);
  // Z is complete once the side stream's updates are
  hipStreamWaitEvent(st, ev_done[0], 0);
  hipStreamWaitEvent(st, ev_done[1], 0);
  hipStreamSynchronize(st);
  auto t2 = std::chrono::steady_clock::now();
  if (t_qr) *t_qr = std::chrono::duration<double>(t2 - t1).count();
  if (hipGetLastError() != hipSuccess && status == 0) status = -4;
  cleanup();
  return status;
}

// ------------------------------------------------------------------ triangular solves --------
// mode 0 (eigenvectors of T): column j solves (T - T_jj I) y = 0 with y_j = 1.
// mode 1 (inverse of a unit upper-triangular M): column j solves M x = e_j.
// Both are back substitutions x_i = -(sum_{k=i+1..j} M_ik x_k) / d_i, d_i = M_ii - M_jj (tiny
// values lifted to ulp |M_jj|) or 1.  The kernel reads Mt = M^T (plain transpose, upper triangle
// of M only), so that lanes running down a column of M read consecutive addresses.  One
// work-group per column; the right-hand sides of the rows not yet solved live in LDS.  Rows go in
// blocks of BS_B aligned to multiples of BS_B (x_j = 1 enters through the first block like a
// solved value): the diagonal block sits in the registers of wave 0 (lane r owns row kb + r, each
// solved value is broadcast with v_readlane), then the block's contribution to every row above is
// one rank-BS_B update over the work-group, so no step waits on a global load or a reduction.
// Work-groups are dispatched to the 8 XCDs in turn; the column map gives each XCD runs of BS_R
// neighbouring columns, longest first, which sweep the same row blocks at about the same time and
// so share them in that XCD's L2.
constexpr int BS_T = 256, BS_B = 16, BS_R = 16;
static int backsolve_grid(int n) { return ((n + 8 * BS_R - 1) / (8 * BS_R)) * 8 * BS_R; }
#define MT(i, k) Mt[(long long)(k) * n + (i)]  // M[i][k]

// ys[i] -= sum_c M[i][kb + c] x[kb + c] for i < kb; FIRST: the block holding x_j = 1, whose
// columns beyond j are not read.
template <bool FIRST>
__device__ inline void backsolve_bulk(const zd* Mt, zd* ys, int n, int j, int kb, int t) {
  zd xv[BS_B];
#pragma unroll
  for (int c = 0; c < BS_B; ++c) xv[c] = (!FIRST || kb + c <= j) ? ys[kb + c] : zmk(0, 0);
  for (int i = t; i < kb; i += BS_T) {
    double ar = ys[i].x, ai = ys[i].y;
#pragma unroll
    for (int c = 0; c < BS_B; ++c) {
      if (!FIRST || kb + c <= j) {
        const zd mv = MT(i, kb + c);
        ar = fma(-mv.x, xv[c].x, ar);
        ar = fma(mv.y, xv[c].y, ar);
        ai = fma(-mv.x, xv[c].y, ai);
        ai = fma(-mv.y, xv[c].x, ai);
      }
    }
    ys[i] = zmk(ar, ai);
  }
}

__global__ __launch_bounds__(BS_T) void k_upper_backsolve(const zd* Mt, zd* X, int n, int mode) {
  extern __shared__ zd ys[];
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int j = n - 1 - ((slot / BS_R) * 8 * BS_R + xcd * BS_R + slot % BS_R);
  if (j < 0) return;  // padding of the grid to whole rounds (uniform over the work-group)
  const int t = threadIdx.x, lane = t & 63;
  const double ulp = 2.220446049250313e-16;
  const zd mjj = MT(j, j);
  const double smin = fmax(ulp * cabs1(mjj), 1e-290);
  for (int i = t; i <= j; i += BS_T) ys[i] = zmk(i == j ? 1.0 : 0.0, 0);
  __syncthreads();
  for (int kb = (j / BS_B) * BS_B; kb >= 0; kb -= BS_B) {
    if (t < 64) {
      const bool own = lane < BS_B && kb + lane < j;
      const int r = kb + (own ? lane : 0);
      zd m[BS_B];
#pragma unroll
      for (int c = 0; c < BS_B; ++c) m[c] = (own && kb + c <= j) ? MT(r, kb + c) : zmk(0, 0);
      zd acc = own ? ys[r] : zmk(0, 0);
      zd rd = zmk(1, 0);
      if (mode == 0 && own) {
        zd den = zsub(MT(r, r), mjj);
        if (cabs1(den) < smin) den = zmk(smin, 0);
        rd = zdiv(zmk(1, 0), den);
      }
#pragma unroll
      for (int c = BS_B - 1; c >= 0; --c) {
        if (kb + c <= j) {
          zd x = zmk(1, 0);
          if (kb + c < j) {
            const zd xl = mode == 0 ? zmul(acc, rd) : acc;
            x = zmk(bcast(xl.x, c), bcast(xl.y, c));
          }
          if (lane < c) acc = zsub(acc, zmul(m[c], x));
          if (lane == c) acc = x;
        }
      }
      if (own) ys[r] = acc;
    }
    __syncthreads();
    if (kb > 0) {
      if (kb + BS_B > j)
        backsolve_bulk<true>(Mt, ys, n, j, kb, t);
      else
        backsolve_bulk<false>(Mt, ys, n, j, kb, t);
      __syncthreads();
    }
  }
  for (int i = t; i < n; i += BS_T) X[(long long)i * n + j] = (i <= j) ? ys[i] : zmk(0, 0);
}
#undef MT

// Y = X^T (plain transpose) on the tiles of an n x n matrix that meet its upper triangle, 32 x 32
// tiles through LDS; tiles wholly below the diagonal are skipped (the back substitutions never
// read them).
__global__ __launch_bounds__(256) void k_transpose_upper(const zd* X, zd* Y, int n) {
  __shared__ zd tile[32][33];
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = bi * 32 + r, k = bj * 32 + tx;
    if (i < n && k < n) tile[r][tx] = X[(long long)i * n + k];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int k = bj * 32 + r, i = bi * 32 + tx;
    if (i < n && k < n) Y[(long long)k * n + i] = tile[tx][r];
  }
}

static int backsolve(const zd* M, zd* Mt, zd* X, int n, int mode, hipStream_t st) {
  if (n < 1) return n == 0 ? 0 : -1;
  const size_t lds = sizeof(zd) * (size_t)n;
  if (lds > 160 * 1024) return -1;
  if (lds > 64 * 1024 &&
      hipFuncSetAttribute((const void*)k_upper_backsolve, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) !=
          hipSuccess)
    return -1;
  const int nt = (n + 31) / 32;
  hipLaunchKernelGGL(k_transpose_upper, dim3(nt, nt), dim3(256), 0, st, M, Mt, n);
  hipLaunchKernelGGL(k_upper_backsolve, dim3(backsolve_grid(n)), dim3(BS_T), lds, st, (const zd*)Mt, X, n, mode);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
int trevec(const zd* T, zd* ws, zd* Y, int n, hipStream_t st) { return backsolve(T, ws, Y, n, 0, st); }
int triinv_unit(const zd* Y, zd* ws, zd* Yinv, int n, hipStream_t st) { return backsolve(Y, ws, Yinv, n, 1, st); }
__global__ void k_diag(const zd* T, zd* s, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) s[i] = T[(long long)i * n + i];
}
int diag_extract(const zd* T, zd* s, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_diag, dim3((n + 255) / 256), dim3(256), 0, st, T, s, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
