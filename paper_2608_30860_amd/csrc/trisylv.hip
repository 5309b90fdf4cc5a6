// Triangular Sylvester solve of the Schur route (Bartels-Stewart, Section A.1):
//   T X + X T^H + sigma X = C,   T upper triangular (n x n), X overwrites C.
// Entrywise, (T_ii + conj(T_jj) + sigma) X_ij = C_ij - sum_{k>i} T_ik X_kj - sum_{k>j} X_ik conj(T_jk),
// so block (I, J) of 32 x 32 blocks depends on the blocks below it in its column and right of it
// in its row, and the blocks of one anti-diagonal I + J = S are independent.  Per anti-diagonal:
//  1. k_trisylv_upd: the block products T_IK X_KJ (K > I) and X_IK T_JK^H (K > J) of every block
//     of the anti-diagonal, spread over up to PMAX workgroups per block (FP64 MFMA, operands
//     through LDS); each workgroup writes its partial sum to the workspace.
//  2. k_trisylv_solve: one workgroup per block subtracts the partial sums from C_IJ and solves
//     T_II X + X T_JJ^H + sigma X = C in LDS by an anti-diagonal sweep: at each step every
//     pending entry takes its products with the two entries solved at the step before (one in its
//     column, one in its row), so a step costs two products per entry and one barrier.
#include "kernels.hpp"

namespace lindx {

static constexpr int TB = 32;
static constexpr int TP = TB + 1;
static constexpr int PMAX = 16;  // partial sums per block

typedef double v4d_s __attribute__((ext_vector_type(4)));

long long trisylv_ws_elems(int n) {
  const long long nb = (n + TB - 1) / TB;
  return nb * PMAX * TB * TB;
}

// partial sums of the block products of anti-diagonal S: workgroup (b, p) takes the terms
// t = p, p + PMAX, ... of block I = Imin + b (terms 0 .. nb-2-I: T_IK X_KJ with K = I+1+t; the
// rest: X_IK T_JK^H with K = J+1+(t - (nb-1-I))).  Wave w computes the 16 x 16 quadrant
// (w >> 1, w & 1) of the 32 x 32 result.
__global__ __launch_bounds__(256) void k_trisylv_upd(const zd* __restrict__ T, const zd* __restrict__ X, int n,
                                                     int nb, int S, int Imin, zd* __restrict__ ws) {
  __shared__ zd As[TB * TP];
  __shared__ zd Bs[TB * TP];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int b = blockIdx.x, p = blockIdx.y;
  const int I = Imin + b;
  const int J = S - I;
  const int nA = nb - 1 - I, nBt = nb - 1 - J;
  const int terms = nA + nBt;
  if (p >= terms) return;  // uniform over the workgroup
  const int i0 = I * TB, j0 = J * TB;
  const int bi = min(TB, n - i0), bj = min(TB, n - j0);
  const int qi = 16 * (w >> 1), qj = 16 * (w & 1);
  v4d_s cr = {0, 0, 0, 0}, ci = {0, 0, 0, 0};
  for (int term = p; term < terms; term += PMAX) {
    const bool first = term < nA;
    const int K = first ? I + 1 + term : J + 1 + (term - nA);
    const int k0 = K * TB;
    const int bk = min(TB, n - k0);
    __syncthreads();
    for (int e = t; e < TB * TB; e += 256) {
      const int r = e >> 5, q = e & 31;
      if (first) {
        // A = T_IK (rows i, cols k), B = X_KJ (rows k, cols j)
        As[r * TP + q] = (r < bi && q < bk) ? T[(long long)(i0 + r) * n + k0 + q] : zmk(0, 0);
        Bs[r * TP + q] = (r < bk && q < bj) ? X[(long long)(k0 + r) * n + j0 + q] : zmk(0, 0);
      } else {
        // A = X_IK (rows i, cols k), B[k][j] = conj(T[j0 + j][k0 + k])
        As[r * TP + q] = (r < bi && q < bk) ? X[(long long)(i0 + r) * n + k0 + q] : zmk(0, 0);
        Bs[q * TP + r] = (r < bj && q < bk) ? zconj(T[(long long)(j0 + r) * n + k0 + q]) : zmk(0, 0);
      }
    }
    __syncthreads();
    {
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
  }
  // accumulator: register r of lane l holds row 4 r + l / 16, column l % 16 of the quadrant
  zd* out = ws + ((long long)b * PMAX + p) * TB * TB;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = qi + 4 * r + (lane >> 4), col = qj + (lane & 15);
    out[row * TB + col] = zmk(cr[r], ci[r]);
  }
}

// C_IJ minus the partial sums, then the diagonal-block solve (see the file comment)
__global__ __launch_bounds__(256) void k_trisylv_solve(const zd* __restrict__ T, zd* __restrict__ X, int n, int nb,
                                                       int S, int Imin, zd sigma, const zd* __restrict__ ws) {
  __shared__ zd As[TB * TP];
  __shared__ zd Bs[TB * TP];
  __shared__ zd Cs[TB * TP];
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  const int I = Imin + b;
  const int J = S - I;
  const int i0 = I * TB, j0 = J * TB;
  const int bi = min(TB, n - i0), bj = min(TB, n - j0);
  const int np = min(PMAX, (nb - 1 - I) + (nb - 1 - J));
  // thread t owns entries (r0 + 8 u, q0); the partial sums are loaded 16 at a time before use
  const int q0 = t & 31, r0 = t >> 5;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = r0 + 8 * u;
    zd part[PMAX];
#pragma unroll
    for (int p = 0; p < PMAX; ++p)
      part[p] = p < np ? ws[((long long)b * PMAX + p) * TB * TB + r * TB + q0] : zmk(0, 0);
    zd v = (r < bi && q0 < bj) ? X[(long long)(i0 + r) * n + j0 + q0] : zmk(0, 0);
#pragma unroll
    for (int p = 0; p < PMAX; ++p) v = zsub(v, part[p]);
    Cs[r * TP + q0] = v;
  }
  for (int e = t; e < TB * TB; e += 256) {
    const int r = e >> 5, q = e & 31;
    As[r * TP + q] = (r < bi && q < bi) ? T[(long long)(i0 + r) * n + i0 + q] : zmk(0, 0);
    Bs[r * TP + q] = (r < bj && q < bj) ? T[(long long)(j0 + r) * n + j0 + q] : zmk(0, 0);
  }
  __syncthreads();
  // step L: every entry not solved yet takes its products with the two entries solved at step
  // L - 1 in its column (row k below) and in its row (column m to the right); the entries with
  // (bi-1-r) + (bj-1-q) = L are then complete and divided by their diagonal.  One thread owns
  // an entry throughout, so one barrier per step separates the writes of step L from the reads
  // of step L + 1.
  const int nlev = (bi - 1) + (bj - 1);
  for (int L = 0; L <= nlev; ++L) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 8 * u, q = q0;
      const int lev = (bi - 1 - r) + (bj - 1 - q);
      if (r >= bi || q >= bj || lev < L) continue;
      zd v = Cs[r * TP + q];
      if (L > 0) {
        const int k = bi - 1 - (L - 1 - (bj - 1 - q));
        if (k > r && k < bi) v = zsub(v, zmul(As[r * TP + k], Cs[k * TP + q]));
        const int m = bj - 1 - (L - 1 - (bi - 1 - r));
        if (m > q && m < bj) v = zsub(v, zmul(Cs[r * TP + m], zconj(Bs[q * TP + m])));
      }
      if (lev == L) v = zdiv(v, zadd(zadd(As[r * TP + r], zconj(Bs[q * TP + q])), sigma));
      Cs[r * TP + q] = v;
    }
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = r0 + 8 * u;
    if (r < bi && q0 < bj) X[(long long)(i0 + r) * n + j0 + q0] = Cs[r * TP + q0];
  }
}

int trisylv(const zd* T, zd* X, int n, zd shift, zd* ws, hipStream_t st) {
  if (n <= 0) return 0;
  if (!ws) return -1;
  const int nb = (n + TB - 1) / TB;
  for (int lev = 0; lev <= 2 * (nb - 1); ++lev) {
    const int S = 2 * (nb - 1) - lev;  // I + J
    const int Imin = S - (nb - 1) > 0 ? S - (nb - 1) : 0;
    const int Imax = S < nb - 1 ? S : nb - 1;
    const int cnt = Imax - Imin + 1;
    // the most terms a block of this anti-diagonal has
    const int terms = 2 * (nb - 1) - S;
    if (terms > 0) {
      const int py = terms < PMAX ? terms : PMAX;
      hipLaunchKernelGGL(k_trisylv_upd, dim3(cnt, py), dim3(256), 0, st, T, X, n, nb, S, Imin, ws);
    }
    hipLaunchKernelGGL(k_trisylv_solve, dim3(cnt), dim3(256), 0, st, T, X, n, nb, S, Imin, shift, ws);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
