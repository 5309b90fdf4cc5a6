// Single-workgroup dense eigensolver for the small projected problems of the Krylov drivers
// (the m x m Hessenberg matrix of Arnoldi, the Krylov-Schur matrix after a thick restart):
// Householder reduction to Hessenberg form, complex single-shift QR to Schur form, right
// eigenvectors of the triangular factor, back-transformation, unit-norm columns.  FP64, LDS.
#include "kernels.hpp"
#include "lds_qr.hpp"

namespace lindx {

__global__ __launch_bounds__(64) void k_small_eig(const zd* A, int lda, int m, zd* w, zd* Yout, int* info) {
  __shared__ zd Hs[64 * LDM];
  __shared__ zd Qs[64 * LDM];
  __shared__ zd u[64];
  const int t = threadIdx.x;
  for (int i = 0; i < m; ++i)
    for (int j = t; j < m; j += 64) {
      Hs[i * LDM + j] = A[(long long)i * lda + j];
      Qs[i * LDM + j] = (i == j) ? zmk(1, 0) : zmk(0, 0);
    }
  __syncthreads();
  hessenberg_lds(Hs, Qs, m, u);
  int rc = qr_lds(Hs, Qs, m, 1);
  for (int i = t; i < m; i += 64) w[i] = Hs[i * LDM + i];
  if (t == 0) info[0] = rc;
  __syncthreads();
  if (Yout == nullptr) return;
  // eigenvectors of T into Yout (global scratch, ld = m), then X = Q Y into Hs
  // (T is no longer needed once Y is formed).
  {
    const double ulp = 2.220446049250313e-16;
    const int j = t;
    if (j < m) {
      zd tjj = Hs[j * LDM + j];
      double smin = fmax(ulp * cabs1(tjj), 1e-290);
      for (int i = 0; i < m; ++i) Yout[(long long)i * m + j] = zmk(0, 0);
      Yout[(long long)j * m + j] = zmk(1, 0);
      for (int i = j - 1; i >= 0; --i) {
        zd acc = Hs[i * LDM + j];
        for (int k = i + 1; k < j; ++k) acc = zadd(acc, zmul(Hs[i * LDM + k], Yout[(long long)k * m + j]));
        zd den = zsub(Hs[i * LDM + i], tjj);
        if (cabs1(den) < smin) den = zmk(smin, 0);
        Yout[(long long)i * m + j] = zdiv(zscale(acc, -1.0), den);
      }
    }
  }
  __syncthreads();
  if (t < m) {
    const int j = t;
    double nrm = 0;
    for (int i = 0; i < m; ++i) {
      zd acc = zmk(0, 0);
      for (int k = 0; k <= j; ++k) acc = zadd(acc, zmul(Qs[i * LDM + k], Yout[(long long)k * m + j]));
      Hs[i * LDM + j] = acc;
      nrm += zabs2(acc);
    }
    nrm = sqrt(nrm);
    // unit norm, phase: largest-modulus entry real positive
    int imax = 0;
    double amax = -1;
    for (int i = 0; i < m; ++i) {
      double a = zabs2(Hs[i * LDM + j]);
      if (a > amax) { amax = a; imax = i; }
    }
    zd ph = Hs[imax * LDM + j];
    double aph = sqrt(zabs2(ph));
    zd f = aph > 0 ? zscale(zconj(ph), 1.0 / (aph * nrm)) : zmk(1.0 / nrm, 0);
    for (int i = 0; i < m; ++i) Hs[i * LDM + j] = zmul(Hs[i * LDM + j], f);
  }
  __syncthreads();
  for (int i = 0; i < m; ++i)
    for (int j = t; j < m; j += 64) Yout[(long long)i * m + j] = Hs[i * LDM + j];
}

int small_eig(const zd* A, int lda, int m, zd* w, zd* Y, int* info, hipStream_t st) {
  if (m < 1 || m > 64) return -1;
  hipLaunchKernelGGL(k_small_eig, dim3(1), dim3(64), 0, st, A, lda, m, w, Y, info);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
