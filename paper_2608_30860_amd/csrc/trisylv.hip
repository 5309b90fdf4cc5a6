// Triangular Sylvester solve of the Schur route (Bartels-Stewart, Section A.1):
//   T X + X T^H + sigma X = C,   T upper triangular (n x n), X overwrites C.
// Entrywise, (T_ii + conj(T_jj) + sigma) X_ij = C_ij - sum_{k>i} T_ik X_kj - sum_{k>j} X_ik conj(T_jk),
// so block (I, J) of 32 x 32 blocks depends on the blocks below it in its column and right of it
// in its row, and the blocks of one anti-diagonal I + J = S are independent.  Of the block products
// a block of anti-diagonal S needs, only two (K = I + 1 and K = J + 1) involve blocks of
// anti-diagonal S + 1; the others involve blocks solved at least two anti-diagonals earlier.  So one
// launch per anti-diagonal S (k_trisylv_level) holds two kinds of workgroups:
//  - solve: one per block of S.  It subtracts the partial sums left by the previous launch and
//    the two products with anti-diagonal S + 1 from C_IJ, then solves
//    T_II X + X T_JJ^H + sigma X = C in LDS by an anti-diagonal sweep: at each step every pending
//    entry takes its products with the two entries solved at the step before (one in its column,
//    one in its row), so a step costs two products per entry and one barrier.
//  - update: the remaining block products of the blocks of anti-diagonal S - 1, spread over up to
//    PMAX workgroups per block (FP64 MFMA, operands through LDS); each writes its partial sum to
//    the workspace half that the next launch reads.
// The critical path is then one launch per anti-diagonal, with the long product sums beside it.
//
// Block eigenbases (optional, for the low-precision modes of the map Phi): a diagonal block has
// T_II = Y_I D_I Y_I^{-1} with Y_I unit upper triangular (its eigenvectors), so the block equation
// T_II X + X T_JJ^H + sigma X = C has the solution
//   X = Y_I [ (Y_I^{-1} C Y_J^{-H})_ab / (t_a + conj(t_b) + sigma) ] Y_J^H,
// four 32 x 32 products on the matrix cores in place of the 63-step sweep.  Its rounding error
// grows with kappa(Y_I) kappa(Y_J), so it is taken only for block pairs whose condition numbers
// (computed once per factorisation, infinity norm) are both within a threshold; every other pair is
// swept.  Both ways are FP64 throughout.
#include "kernels.hpp"

namespace lindx {

static constexpr int TB = 32;
static constexpr int TP = TB + 1;  // row stride of the product tiles
// Row stride of the solve tiles: the sweep reads C down an anti-diagonal (k = c - q across the
// lanes), a lane stride of SP - 1 = 33 entries = 528 bytes, which falls on distinct LDS banks
// (32 entries = 512 bytes would put every lane on the same ones).
static constexpr int SP = TB + 2;
// partial sums per block: a block has up to 2 n / 32 far products (100 at n = 1600), taken by up to
// 16 update workgroups in runs of at most 7, so that they finish beside the solve of the block
// pairs of the next anti-diagonal; the solve reads the partial sums four slots at a time
static constexpr int PMAX = 16;

typedef double v4d_s __attribute__((ext_vector_type(4)));

long long trisylv_ws_elems(int n) {
  const long long nb = (n + TB - 1) / TB;
  return 2 * nb * PMAX * TB * TB;  // two halves: one read, one written by each launch
}

// block products outside the critical pair: block (I, J) has max(0, nb-2-I) terms T_IK X_KJ
// (K = I+2 ...) and then max(0, nb-2-J) terms X_IK T_JK^H (K = J+2 ...)
__device__ __forceinline__ int far_terms_a(int nb, int I) { return max(0, nb - 2 - I); }
__device__ __forceinline__ int far_terms(int nb, int I, int J) { return far_terms_a(nb, I) + max(0, nb - 2 - J); }

// operand tiles of one block product into registers: first kind A = T_IK, B = X_KJ; second kind
// A = X_IK, B = T_JK^H (kept as conj(T_JK), transposed when stored)
__device__ __forceinline__ void term_load(const zd* __restrict__ T, const zd* __restrict__ X, int n, int i0, int j0,
                                          int bi, int bj, int K, bool first, int t, zd ra[4], zd rb[4]) {
  const int k0 = K * TB;
  const int bk = min(TB, n - k0);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = t + 256 * u;
    const int r = e >> 5, q = e & 31;
    if (first) {
      ra[u] = (r < bi && q < bk) ? T[(long long)(i0 + r) * n + k0 + q] : zmk(0, 0);
      rb[u] = (r < bk && q < bj) ? X[(long long)(k0 + r) * n + j0 + q] : zmk(0, 0);
    } else {
      ra[u] = (r < bi && q < bk) ? X[(long long)(i0 + r) * n + k0 + q] : zmk(0, 0);
      rb[u] = (r < bj && q < bk) ? zconj(T[(long long)(j0 + r) * n + k0 + q]) : zmk(0, 0);
    }
  }
}
__device__ __forceinline__ void term_store(zd* As, zd* Bs, bool first, int t, const zd ra[4], const zd rb[4]) {
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = t + 256 * u;
    const int r = e >> 5, q = e & 31;
    As[r * TP + q] = ra[u];
    if (first)
      Bs[r * TP + q] = rb[u];
    else
      Bs[q * TP + r] = rb[u];
  }
}
// wave w accumulates the 16 x 16 quadrant (w >> 1, w & 1) of As Bs; register r of lane l holds
// row 4 r + l / 16, column l % 16 of the quadrant
__device__ __forceinline__ void term_mfma(const zd* As, const zd* Bs, int lane, int qi, int qj, v4d_s& cr,
                                          v4d_s& ci) {
  const int i = lane & 15, kk = lane >> 4;
#pragma unroll
  for (int k0l = 0; k0l < TB; k0l += 4) {
    const zd a = As[(qi + i) * TP + k0l + kk];
    const zd bb = Bs[(k0l + kk) * TP + qj + i];
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bb.x, cr, 0, 0, 0);
    cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bb.y, cr, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bb.y, ci, 0, 0, 0);
    ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bb.x, ci, 0, 0, 0);
  }
}

// Sweep order of the 1024 entries of a 32 x 32 block: by the step at which an entry is solved
// (lev = 62 - r - q), then by the first step at which it takes a product (min(32 - r, 32 - q)),
// taken from both ends of the anti-diagonal inwards.  Thread t holds the entries 256 u + t, so
// the 64 entries a wave holds in one slot are active over a short window of steps.
struct SweepOrder {
  unsigned short rq[TB * TB];
};
constexpr SweepOrder make_sweep_order() {
  SweepOrder o{};
  int k = 0;
  for (int lev = 0; lev <= 2 * (TB - 1); ++lev) {
    int lo = (TB - 1 - lev) > 0 ? TB - 1 - lev : 0;
    int hi = (2 * (TB - 1) - lev) < TB - 1 ? 2 * (TB - 1) - lev : TB - 1;
    while (lo <= hi) {
      // first product step of row r on this anti-diagonal: min(TB - r, TB - q)
      const int ql = 2 * (TB - 1) - lev - lo, qh = 2 * (TB - 1) - lev - hi;
      const int sl = (TB - lo) < (TB - ql) ? TB - lo : TB - ql;
      const int sh = (TB - hi) < (TB - qh) ? TB - hi : TB - qh;
      if (sl <= sh) {
        o.rq[k++] = (unsigned short)(lo * TB + ql);
        ++lo;
      } else {
        o.rq[k++] = (unsigned short)(hi * TB + qh);
        --hi;
      }
    }
  }
  return o;
}
__constant__ SweepOrder c_sweep = make_sweep_order();

// Eigenvectors of diagonal block I of T: Y (unit upper triangular, column k solves
// (T_II - t_kk) y = 0 by back substitution), its inverse, and kap = ||Y||_inf ||Y^{-1}||_inf (infinite
// or NaN when two diagonal entries coincide).  A last block of b < 32 rows is padded with the identity.
__global__ __launch_bounds__(64) void k_blk_eig(const zd* __restrict__ T, int n, zd* __restrict__ Y,
                                                zd* __restrict__ Yi, double* __restrict__ kap) {
  __shared__ zd Ts[TB][TB + 1];
  __shared__ zd Ys[TB][TB + 1];
  __shared__ zd Zs[TB][TB + 1];
  __shared__ double rs[2][TB];
  const int I = blockIdx.x, t = threadIdx.x;
  const int i0 = I * TB, b = min(TB, n - i0);
  for (int e = t; e < TB * TB; e += 64) {
    const int r = e / TB, q = e % TB;
    Ts[r][q] = (r < b && q < b) ? T[(long long)(i0 + r) * n + i0 + q] : zmk(0, 0);
  }
  __syncthreads();
  if (t < TB) {
    const int k = t;
    for (int i = 0; i < TB; ++i) Ys[i][k] = zmk(i == k ? 1.0 : 0.0, 0.0);
    if (k < b)
      for (int i = k - 1; i >= 0; --i) {
        zd acc = zmk(0, 0);
        for (int m = i + 1; m <= k; ++m) acc = zadd(acc, zmul(Ts[i][m], Ys[m][k]));
        Ys[i][k] = zdiv(zmk(-acc.x, -acc.y), zsub(Ts[i][i], Ts[k][k]));
      }
  }
  __syncthreads();
  if (t < TB) {
    const int k = t;
    for (int i = 0; i < TB; ++i) Zs[i][k] = zmk(i == k ? 1.0 : 0.0, 0.0);
    for (int i = k - 1; i >= 0; --i) {
      zd acc = zmk(0, 0);
      for (int m = i + 1; m <= k; ++m) acc = zadd(acc, zmul(Ys[i][m], Zs[m][k]));
      Zs[i][k] = zmk(-acc.x, -acc.y);
    }
  }
  __syncthreads();
  if (t < TB) {
    double sy = 0, sz = 0;
    for (int q = 0; q < TB; ++q) {
      sy += sqrt(zabs2(Ys[t][q]));
      sz += sqrt(zabs2(Zs[t][q]));
    }
    rs[0][t] = sy;
    rs[1][t] = sz;
  }
  __syncthreads();
  if (t == 0) {
    double my = 0, mz = 0;
    bool finite = true;
    for (int r = 0; r < TB; ++r) {
      finite = finite && isfinite(rs[0][r]) && isfinite(rs[1][r]);
      my = fmax(my, rs[0][r]);
      mz = fmax(mz, rs[1][r]);
    }
    kap[I] = finite ? my * mz : INFINITY;
  }
  for (int e = t; e < TB * TB; e += 64) {
    const int r = e / TB, q = e % TB;
    Y[(long long)I * TB * TB + e] = Ys[r][q];
    Yi[(long long)I * TB * TB + e] = Zs[r][q];
  }
}

// One launch per anti-diagonal S: workgroups [0, cnt) solve the blocks I = Imin + b of S; the
// next cntu * py workgroups compute partial sums of the far products of the blocks of S - 1
// (block Iu = Iminu + b', slot p; terms p, p + PMAX, ...).  wsr holds the partial sums of S
// (written by the previous launch), wsw receives those of S - 1.
__global__ __launch_bounds__(256) void k_trisylv_level(const zd* __restrict__ T, zd* __restrict__ X, int n, int nb,
                                                       int S, int Imin, int cnt, int Iminu, int py, zd sigma,
                                                       const zd* __restrict__ wsr, zd* __restrict__ wsw,
                                                       int pyr, TsBlk blk) {
  __shared__ zd sm[3 * TB * SP];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int qi = 16 * (w >> 1), qj = 16 * (w & 1);
  zd ra[4], rb[4];
  if ((int)blockIdx.x >= cnt) {
    // ---- far products of anti-diagonal S - 1
    zd* As = sm;
    zd* Bs = sm + TB * TP;
    const int idx = blockIdx.x - cnt;
    const int bu = idx / py, p = idx % py;
    const int I = Iminu + bu, J = S - 1 - I;
    const int nA = far_terms_a(nb, I);
    const int terms = far_terms(nb, I, J);
    if (p >= terms) return;  // uniform over the workgroup
    const int i0 = I * TB, j0 = J * TB;
    const int bi = min(TB, n - i0), bj = min(TB, n - j0);
    v4d_s cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    // the tiles of the next term are loaded while the current one is multiplied
    term_load(T, X, n, i0, j0, bi, bj, p < nA ? I + 2 + p : J + 2 + (p - nA), p < nA, t, ra, rb);
    for (int term = p; term < terms; term += py) {
      __syncthreads();
      term_store(As, Bs, term < nA, t, ra, rb);
      __syncthreads();
      const int nx = term + py;
      if (nx < terms) term_load(T, X, n, i0, j0, bi, bj, nx < nA ? I + 2 + nx : J + 2 + (nx - nA), nx < nA, t, ra, rb);
      term_mfma(As, Bs, lane, qi, qj, cr, ci);
    }
    zd* out = wsw + ((long long)bu * PMAX + p) * TB * TB;
#pragma unroll
    for (int r = 0; r < 4; ++r) out[(qi + 4 * r + (lane >> 4)) * TB + qj + (lane & 15)] = zmk(cr[r], ci[r]);
    return;
  }
  // ---- solve of block (I, J) of anti-diagonal S
  zd* As = sm;               // T_II (row stride SP); product tile A before that
  zd* Bh = sm + TB * SP;     // Bh[m][q] = conj(T_JJ[q][m]); product tile B before that
  zd* Cs = sm + 2 * TB * SP; // solved entries; the near products before that
  const int b = blockIdx.x;
  const int I = Imin + b, J = S - I;
  const int i0 = I * TB, j0 = J * TB;
  const int bi = min(TB, n - i0), bj = min(TB, n - j0);
  const int np = min(pyr, far_terms(nb, I, J));  // slots the previous launch wrote for this block
  const bool nearA = I + 1 < nb, nearB = J + 1 < nb;
  if (nearA) term_load(T, X, n, i0, j0, bi, bj, I + 1, true, t, ra, rb);
  // thread t owns the entries 256 u + t of the sweep order and keeps them in registers until
  // they are solved
  int er[4], eq[4];
  bool ok[4];
  zd v[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int rq = c_sweep.rq[256 * u + t];
    er[u] = rq >> 5;
    eq[u] = rq & 31;
    ok[u] = er[u] < bi && eq[u] < bj;
    v[u] = ok[u] ? X[(long long)(i0 + er[u]) * n + j0 + eq[u]] : zmk(0, 0);
  }
  // block eigenbases for this pair (uniform over the workgroup)?
  const double kapI = blk.kap ? blk.kap[I] : INFINITY, kapJ = blk.kap ? blk.kap[J] : INFINITY;
  const bool eig = kapI < INFINITY && kapJ < INFINITY && kapI <= blk.thr && kapJ <= blk.thr;
  // T_II and T_JJ^H (sweep), or Y_I^{-1} and Y_J^{-1} (eigenbases), pass through registers while
  // LDS holds the product tiles
  zd ta[4], tb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = t + 256 * k;
    const int r = e >> 5, q = e & 31;
    if (eig) {
      ta[k] = blk.Yi[(long long)I * TB * TB + e];
      tb[k] = blk.Yi[(long long)J * TB * TB + e];
    } else {
      ta[k] = (r < bi && q < bi) ? T[(long long)(i0 + r) * n + i0 + q] : zmk(0, 0);
      tb[k] = (r < bj && q < bj) ? zconj(T[(long long)(j0 + r) * n + j0 + q]) : zmk(0, 0);
    }
  }
  // partial sums in groups of four slots, all loads of a group in flight together
  for (int p0 = 0; p0 < np; p0 += 4) {
    zd part[4][4];
#pragma unroll
    for (int pp = 0; pp < 4; ++pp)
#pragma unroll
      for (int u = 0; u < 4; ++u)
        part[pp][u] = p0 + pp < np ? wsr[((long long)b * PMAX + p0 + pp) * TB * TB + er[u] * TB + eq[u]] : zmk(0, 0);
#pragma unroll
    for (int pp = 0; pp < 4; ++pp)
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = zsub(v[u], part[pp][u]);
  }
  if (nearA || nearB) {
    v4d_s cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    if (nearA) {
      term_store(As, Bh, true, t, ra, rb);
      __syncthreads();
      if (nearB) term_load(T, X, n, i0, j0, bi, bj, J + 1, false, t, ra, rb);
      term_mfma(As, Bh, lane, qi, qj, cr, ci);
    } else {
      term_load(T, X, n, i0, j0, bi, bj, J + 1, false, t, ra, rb);
    }
    if (nearB) {
      __syncthreads();
      term_store(As, Bh, false, t, ra, rb);
      __syncthreads();
      term_mfma(As, Bh, lane, qi, qj, cr, ci);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) Cs[(qi + 4 * r + (lane >> 4)) * SP + qj + (lane & 15)] = zmk(cr[r], ci[r]);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) v[u] = zsub(v[u], Cs[er[u] * SP + eq[u]]);
    __syncthreads();
  }
  if (eig) {
    // block eigenbases: X = Y_I [(Y_I^{-1} C Y_J^{-H}) / (t_a + conj t_b + sigma)] Y_J^H, four
    // products of 32 x 32 tiles in LDS (row stride TP), each wave one 16 x 16 quadrant; the
    // inverses came in with the right-hand side, the eigenvector tiles and the diagonal entries
    // are loaded while the first two products run
    zd* Ap = sm;
    zd* Bp = sm + TB * SP;
    zd* Cp = sm + 2 * TB * SP;
    const int ra0 = qi + (lane >> 4), cb = qj + (lane & 15);
    zd yi[4], yj[4], da[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = t + 256 * k;
      yi[k] = blk.Y[(long long)I * TB * TB + e];
      yj[k] = blk.Y[(long long)J * TB * TB + e];
      const int a = ra0 + 4 * k;
      da[k] = a < bi ? T[(long long)(i0 + a) * n + i0 + a] : zmk(1, 0);
    }
    const zd tbd = cb < bj ? zconj(T[(long long)(j0 + cb) * n + j0 + cb]) : zmk(0, 0);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) Cp[er[u] * TP + eq[u]] = v[u];  // zero outside the block
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = t + 256 * k;
      Ap[(e >> 5) * TP + (e & 31)] = ta[k];
    }
    __syncthreads();
    v4d_s cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
    term_mfma(Ap, Cp, lane, qi, qj, cr, ci);  // Y_I^{-1} C
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) Ap[(ra0 + 4 * r) * TP + cb] = zmk(cr[r], ci[r]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = t + 256 * k;
      Bp[(e & 31) * TP + (e >> 5)] = zconj(tb[k]);  // Bp[k][c] = conj(Y_J^{-1}[c][k])
    }
    __syncthreads();
    cr = v4d_s{0, 0, 0, 0};
    ci = v4d_s{0, 0, 0, 0};
    term_mfma(Ap, Bp, lane, qi, qj, cr, ci);  // (Y_I^{-1} C) Y_J^{-H}
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = ra0 + 4 * r;
      zd w = zmk(0, 0);
      if (a < bi && cb < bj) w = zdiv(zmk(cr[r], ci[r]), zadd(zadd(da[r], tbd), sigma));
      Cp[a * TP + cb] = w;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = t + 256 * k;
      Ap[(e >> 5) * TP + (e & 31)] = yi[k];
    }
    __syncthreads();
    cr = v4d_s{0, 0, 0, 0};
    ci = v4d_s{0, 0, 0, 0};
    term_mfma(Ap, Cp, lane, qi, qj, cr, ci);  // Y_I W
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) Ap[(ra0 + 4 * r) * TP + cb] = zmk(cr[r], ci[r]);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int e = t + 256 * k;
      Bp[(e & 31) * TP + (e >> 5)] = zconj(yj[k]);  // Bp[k][c] = conj(Y_J[c][k])
    }
    __syncthreads();
    cr = v4d_s{0, 0, 0, 0};
    ci = v4d_s{0, 0, 0, 0};
    term_mfma(Ap, Bp, lane, qi, qj, cr, ci);  // (Y_I W) Y_J^H
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int a = ra0 + 4 * r;
      if (a < bi && cb < bj) X[(long long)(i0 + a) * n + j0 + cb] = zmk(cr[r], ci[r]);
    }
    return;
  }
  // the zero slot (padding column of row 0 of As) stands in for both operands of a product that
  // does not apply
  const int ZS = TB;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int e = t + 256 * k;
    const int r = e >> 5, q = e & 31;
    As[r * SP + q] = ta[k];
    Bh[q * SP + r] = tb[k];
  }
  if (t == 0) As[ZS] = zmk(0, 0);
  __syncthreads();
  // Entry (r, q) is solved at step lev = (bi-1-r) + (bj-1-q).  At step L it takes the product
  // with the entry of its column solved at step L - 1, row k = kb - L (kb = bi + bj - 1 - q),
  // for bj - q <= L <= lev, and the product with the entry of its row solved at step L - 1,
  // column m = mb - L (mb = bi + bj - 1 - r), for bi - r <= L <= lev.  A wave skips a slot
  // outside the union of its entries' windows.
  zd rinv[4];
  int lev[4], lo1[4], lo2[4], n1[4], n2[4], pA1[4], pC1[4], pC2[4], pB2[4], wlo[4], whi[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = er[u], q = eq[u];
    rinv[u] = ok[u] ? zdiv(zmk(1, 0), zadd(zadd(As[r * SP + r], Bh[q * SP + q]), sigma)) : zmk(0, 0);
    const int kb = bi + bj - 1 - q, mb = bi + bj - 1 - r;
    lev[u] = ok[u] ? kb - 1 - r : -1;
    // product windows [lo, lo + len): empty for an entry outside the block
    lo1[u] = bj - q;
    lo2[u] = bi - r;
    n1[u] = ok[u] ? max(0, lev[u] - lo1[u] + 1) : 0;
    n2[u] = ok[u] ? max(0, lev[u] - lo2[u] + 1) : 0;
    pA1[u] = r * SP + kb;                     // As[r][k] = pA1 - L
    pC1[u] = 2 * TB * SP + kb * SP + q;       // Cs[k][q] = pC1 - L SP
    pC2[u] = 2 * TB * SP + r * SP + mb;       // Cs[r][m] = pC2 - L
    pB2[u] = TB * SP + mb * SP + q;           // Bh[m][q] = pB2 - L SP
    int lo = ok[u] ? min(min(lo1[u], lo2[u]), lev[u]) : 1 << 20;
    int hi = lev[u];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      lo = min(lo, __shfl_xor(lo, o, 64));
      hi = max(hi, __shfl_xor(hi, o, 64));
    }
    wlo[u] = __builtin_amdgcn_readfirstlane(lo);
    whi[u] = __builtin_amdgcn_readfirstlane(hi);
  }
  // One barrier per step separates the writes of step L from the reads of step L + 1.
  const int nlev = (bi - 1) + (bj - 1);
  for (int L = 0; L <= nlev; ++L) {
    zd a1[4], c1[4], c2[4], b2[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (L < wlo[u] || L > whi[u]) continue;
      // the addresses are selected by masks, not branches, so that all reads are in flight at once
      const int m1 = -(int)((unsigned)(L - lo1[u]) < (unsigned)n1[u]);
      const int m2 = -(int)((unsigned)(L - lo2[u]) < (unsigned)n2[u]);
      a1[u] = sm[ZS + ((pA1[u] - L - ZS) & m1)];
      c1[u] = sm[ZS + ((pC1[u] - L * SP - ZS) & m1)];
      c2[u] = sm[ZS + ((pC2[u] - L - ZS) & m2)];
      b2[u] = sm[ZS + ((pB2[u] - L * SP - ZS) & m2)];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (L < wlo[u] || L > whi[u]) continue;
      zd x = v[u];
      x.x -= a1[u].x * c1[u].x - a1[u].y * c1[u].y;
      x.y -= a1[u].x * c1[u].y + a1[u].y * c1[u].x;
      x.x -= c2[u].x * b2[u].x - c2[u].y * b2[u].y;
      x.y -= c2[u].x * b2[u].y + c2[u].y * b2[u].x;
      if (L == lev[u]) {
        x = zmul(x, rinv[u]);
        Cs[er[u] * SP + eq[u]] = x;
      }
      v[u] = x;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (ok[u]) X[(long long)(i0 + er[u]) * n + j0 + eq[u]] = v[u];
}

long long trisylv_blk_elems(int n) { return (long long)((n + TB - 1) / TB) * TB * TB; }

int trisylv_blk_setup(const zd* T, int n, zd* Y, zd* Yi, double* kap, hipStream_t st) {
  if (n <= 0) return 0;
  if (!T || !Y || !Yi || !kap) return -1;
  hipLaunchKernelGGL(k_blk_eig, dim3((n + TB - 1) / TB), dim3(64), 0, st, T, n, Y, Yi, kap);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int trisylv(const zd* T, zd* X, int n, zd shift, zd* ws, hipStream_t st, const TsBlk* blkp) {
  const TsBlk blk = blkp ? *blkp : TsBlk{};
  if (n <= 0) return 0;
  if (!ws) return -1;
  const int nb = (n + TB - 1) / TB;
  const long long half = (long long)nb * PMAX * TB * TB;
  auto imin = [&](int S) { return S - (nb - 1) > 0 ? S - (nb - 1) : 0; };
  auto imax = [&](int S) { return S < nb - 1 ? S : nb - 1; };
  // workgroups the chip holds at once (two per compute unit at this kernel's register use): a
  // launch wider than that runs in two rounds, so the far products are spread no wider
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -4;
  const int resident = 2 * device_cus(dev);
  int py_prev = 0;
  for (int lev = 0; lev <= 2 * (nb - 1); ++lev) {
    const int S = 2 * (nb - 1) - lev;  // I + J
    const int Imin = imin(S), cnt = imax(S) - Imin + 1;
    // far products of anti-diagonal S - 1, spread over py workgroups per block (py = the most far
    // terms a block of S - 1 has, at most PMAX, and no more than one round of the chip allows)
    int cntu = 0, py = 1, Iminu = 0;
    if (S >= 1) {
      int terms = 0;
      for (int I = imin(S - 1); I <= imax(S - 1); ++I) {
        const int J = S - 1 - I;
        const int f = (nb - 2 - I > 0 ? nb - 2 - I : 0) + (nb - 2 - J > 0 ? nb - 2 - J : 0);
        terms = f > terms ? f : terms;
      }
      if (terms > 0) {
        Iminu = imin(S - 1);
        cntu = imax(S - 1) - Iminu + 1;
        py = terms < PMAX ? terms : PMAX;
        const int fit = (resident - cnt) / cntu;
        if (py > fit) py = fit > 1 ? fit : 1;
      }
    }
    const zd* wsr = ws + (lev & 1) * half;
    zd* wsw = ws + ((lev + 1) & 1) * half;
    hipLaunchKernelGGL(k_trisylv_level, dim3(cnt + cntu * py), dim3(256), 0, st, T, X, n, nb, S, Imin, cnt, Iminu,
                       py, shift, wsr, wsw, py_prev, blk);
    py_prev = cntu ? py : 0;
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
