// Triangular Sylvester solve of the Schur route (Bartels-Stewart, Section A.1):
//   T X + X T^H + sigma X = C,   T upper triangular (n x n), X overwrites C.
// Entrywise, (T_ii + conj(T_jj) + sigma) X_ij = C_ij - sum_{k>i} T_ik X_kj - sum_{k>j} X_ik conj(T_jk),
// so block (I, J) depends on the blocks below it in its column and right of it in its row.
// Blocks on one anti-diagonal are independent: one launch per anti-diagonal, one workgroup per
// block, which first subtracts the contributions of the solved blocks (FP64 products through LDS
// tiles) and then solves its diagonal b x b problem in LDS by an anti-diagonal sweep.
#include "kernels.hpp"

namespace lindx {

static constexpr int TB = 32;
static constexpr int TP = TB + 1;

__global__ __launch_bounds__(256) void k_trisylv_level(const zd* __restrict__ T, zd* __restrict__ X, int n, int nb,
                                                       int S, int Imin, zd sigma) {
  __shared__ zd As[TB * TP];
  __shared__ zd Bs[TB * TP];
  __shared__ zd Cs[TB * TP];
  const int t = threadIdx.x;
  const int I = Imin + blockIdx.x;
  const int J = S - I;
  const int i0 = I * TB, j0 = J * TB;
  const int bi = min(TB, n - i0), bj = min(TB, n - j0);
  // load C = X_IJ
  for (int e = t; e < TB * TB; e += 256) {
    int r = e / TB, q = e - r * TB;
    Cs[r * TP + q] = (r < bi && q < bj) ? X[(long long)(i0 + r) * n + j0 + q] : zmk(0, 0);
  }
  // accumulators: each thread owns 4 entries (rows r0 + 8*u, column q0)
  const int q0 = t & 31;
  const int r0 = t >> 5;  // 0..7
  zd acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = zmk(0, 0);
  // - sum_{K > I} T_IK X_KJ
  for (int K = I + 1; K < nb; ++K) {
    const int k0 = K * TB;
    const int bk = min(TB, n - k0);
    __syncthreads();
    for (int e = t; e < TB * TB; e += 256) {
      int r = e / TB, q = e - r * TB;
      As[r * TP + q] = (r < bi && q < bk) ? T[(long long)(i0 + r) * n + k0 + q] : zmk(0, 0);
      Bs[r * TP + q] = (r < bk && q < bj) ? X[(long long)(k0 + r) * n + j0 + q] : zmk(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 8 * u;
      zd a = acc[u];
      for (int k = 0; k < TB; ++k) a = zadd(a, zmul(As[r * TP + k], Bs[k * TP + q0]));
      acc[u] = a;
    }
  }
  // - sum_{K > J} X_IK T_JK^H
  for (int K = J + 1; K < nb; ++K) {
    const int k0 = K * TB;
    const int bk = min(TB, n - k0);
    __syncthreads();
    for (int e = t; e < TB * TB; e += 256) {
      int r = e / TB, q = e - r * TB;
      As[r * TP + q] = (r < bi && q < bk) ? X[(long long)(i0 + r) * n + k0 + q] : zmk(0, 0);
      // Bs[k][q] = conj(T[j0+q][k0+k])
      Bs[q * TP + r] = zmk(0, 0);
    }
    __syncthreads();
    for (int e = t; e < TB * TB; e += 256) {
      int r = e / TB, q = e - r * TB;  // r: row of T_JK (j index), q: column (k index)
      if (r < bj && q < bk) Bs[q * TP + r] = zconj(T[(long long)(j0 + r) * n + k0 + q]);
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = r0 + 8 * u;
      zd a = acc[u];
      for (int k = 0; k < TB; ++k) a = zadd(a, zmul(As[r * TP + k], Bs[k * TP + q0]));
      acc[u] = a;
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = r0 + 8 * u;
    Cs[r * TP + q0] = zsub(Cs[r * TP + q0], acc[u]);
  }
  // diagonal blocks T_II (As) and T_JJ (Bs)
  for (int e = t; e < TB * TB; e += 256) {
    int r = e / TB, q = e - r * TB;
    As[r * TP + q] = (r < bi && q < bi) ? T[(long long)(i0 + r) * n + i0 + q] : zmk(0, 0);
    Bs[r * TP + q] = (r < bj && q < bj) ? T[(long long)(j0 + r) * n + j0 + q] : zmk(0, 0);
  }
  __syncthreads();
  // anti-diagonal sweep from the bottom-right corner of the block
  for (int lev = 0; lev <= (bi - 1) + (bj - 1); ++lev) {
    // entries with (bi-1-r) + (bj-1-q) == lev
    for (int e = t; e < TB; e += 256) {
      int r = bi - 1 - e;
      int q = (bj - 1) - (lev - e);
      if (r < 0 || q < 0 || q >= bj) continue;
      zd v = Cs[r * TP + q];
      for (int k = r + 1; k < bi; ++k) v = zsub(v, zmul(As[r * TP + k], Cs[k * TP + q]));
      for (int k = q + 1; k < bj; ++k) v = zsub(v, zmul(Cs[r * TP + k], zconj(Bs[q * TP + k])));
      zd den = zadd(zadd(As[r * TP + r], zconj(Bs[q * TP + q])), sigma);
      Cs[r * TP + q] = zdiv(v, den);
    }
    __syncthreads();
  }
  for (int e = t; e < TB * TB; e += 256) {
    int r = e / TB, q = e - r * TB;
    if (r < bi && q < bj) X[(long long)(i0 + r) * n + j0 + q] = Cs[r * TP + q];
  }
}

int trisylv(const zd* T, zd* X, int n, zd shift, hipStream_t st) {
  const int nb = (n + TB - 1) / TB;
  for (int lev = 0; lev <= 2 * (nb - 1); ++lev) {
    const int S = 2 * (nb - 1) - lev;  // I + J
    const int Imin = S - (nb - 1) > 0 ? S - (nb - 1) : 0;
    const int Imax = S < nb - 1 ? S : nb - 1;
    const int cnt = Imax - Imin + 1;
    hipLaunchKernelGGL(k_trisylv_level, dim3(cnt), dim3(256), 0, st, T, X, n, nb, S, Imin, shift);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
