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

// The Ritz pair of an upper Hessenberg H (k x k, k <= 64) whose eigenvalue is nearest sigma, by
// inverse iteration with the fixed shift sigma: one LU factorisation of H - sigma I with partial
// pivoting (a Hessenberg matrix only ever swaps neighbouring rows), then per iteration a forward
// and a back substitution, x <- (H - sigma I)^{-1} x / ||.||, until the direction settles.  The
// iteration converges to the eigenvector of the eigenvalue nearest sigma at the rate
// |lambda_1 - sigma| / |lambda_2 - sigma|.  A zero pivot is replaced by ulp ||H||_F (H - sigma I is
// singular exactly when sigma is an eigenvalue, and then the first solve already gives the
// eigenvector).  Output out[0] = theta = y^H H y, out[1 .. k] = y with unit norm and its
// largest-modulus entry real positive, out[k + 1] = (||H y - theta y||_2, 0), info = iterations.
// One wave; lane c owns column c in the elimination and row c in the substitutions.
__global__ __launch_bounds__(64) void k_ritz_near(const zd* H, int ld, int k, zd sigma, zd* out, int* info) {
  __shared__ zd A[64 * LDM];
  __shared__ zd x[64];
  __shared__ zd lf[64];
  __shared__ int piv[64];
  const int t = threadIdx.x;
  double fro = 0;
  for (int i = 0; i < k; ++i) {
    if (t < k) {
      zd h = H[(long long)i * ld + t];
      fro += zabs2(h);
      if (i == t) h = zsub(h, sigma);
      A[i * LDM + t] = h;
    }
  }
  for (int o = 32; o > 0; o >>= 1) fro += __shfl_xor(fro, o, 64);
  const double tiny = fmax(2.220446049250313e-16 * sqrt(fro), 1e-300);
  __syncthreads();
  // LU of the Hessenberg matrix: step j pivots between rows j and j + 1 and eliminates A[j+1][j]
  for (int j = 0; j + 1 < k; ++j) {
    const zd d = A[j * LDM + j], e = A[(j + 1) * LDM + j];
    const bool sw = cabs1(e) > cabs1(d);
    if (sw && t >= j && t < k) {
      const zd u = A[j * LDM + t];
      A[j * LDM + t] = A[(j + 1) * LDM + t];
      A[(j + 1) * LDM + t] = u;
    }
    __syncthreads();
    zd p = A[j * LDM + j];
    if (cabs1(p) < tiny) p = zmk(tiny, 0);
    const zd l = zdiv(A[(j + 1) * LDM + j], p);
    if (t > j && t < k) A[(j + 1) * LDM + t] = zsub(A[(j + 1) * LDM + t], zmul(l, A[j * LDM + t]));
    if (t == 0) {
      A[j * LDM + j] = p;
      lf[j] = l;
      piv[j] = sw ? 1 : 0;
    }
    __syncthreads();
  }
  if (t == 0 && cabs1(A[(k - 1) * LDM + k - 1]) < tiny) A[(k - 1) * LDM + k - 1] = zmk(tiny, 0);
  __syncthreads();
  // per-lane operands of the substitutions: lane j holds l_j and the swap flag of elimination step
  // j and the reciprocal of U_jj, so that both substitutions pass their running value by
  // v_readlane instead of an LDS round trip per row
  const zd lj = (t + 1 < k) ? lf[t] : zmk(0, 0);
  const int pj = (t + 1 < k) ? piv[t] : 0;
  const zd rj = t < k ? zdiv(zmk(1.0, 0.0), A[t * LDM + t]) : zmk(0, 0);
  // start: all ones (a fixed vector, so the result is deterministic)
  zd xr = t < k ? zmk(1.0 / sqrt((double)k), 0) : zmk(0, 0);
  int it = 0;
  double dprev = 1e300;
  for (; it < 60; ++it) {
    // forward: the row swaps and eliminations applied to x.  Step j leaves its final entry j
    // (row j + 1's original value if the rows were swapped, else the running value) and carries
    // the updated row j + 1 on.
    zd carry = zreadlane(xr, 0);
    zd bi = zmk(0, 0);
    for (int j = 0; j + 1 < k; ++j) {
      const zd nb = zreadlane(xr, j + 1);
      const zd l = zreadlane(lj, j);
      const bool sw = __builtin_amdgcn_readlane(pj, j) != 0;
      const zd fin = sw ? nb : carry;
      const zd oth = sw ? carry : nb;
      if (t == j) bi = fin;
      carry = zsub(oth, zmul(l, fin));
    }
    if (t == k - 1) bi = carry;
    // back substitution, column oriented: x_i = b_i / U_ii, then b_r -= U_ri x_i for r < i
    zd xi = zmk(0, 0);
    for (int i = k - 1; i >= 0; --i) {
      const zd xv = zmul(zreadlane(bi, i), zreadlane(rj, i));
      if (t == i) xi = xv;
      if (t < i) bi = zsub(bi, zmul(A[t * LDM + i], xv));
    }
    // normalise; the direction has settled when the new vector, rotated onto the old one's phase,
    // differs from it by rounding only (or stops getting closer)
    double nn = t < k ? zabs2(xi) : 0.0;
    for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
    xi = zscale(xi, 1.0 / sqrt(nn));
    const zd old = xr;
    zd ov = zcmul(xi, old);  // <new, old>
    for (int o = 32; o > 0; o >>= 1) {
      ov.x += __shfl_xor(ov.x, o, 64);
      ov.y += __shfl_xor(ov.y, o, 64);
    }
    const double aov = sqrt(zabs2(ov));
    const zd rot = aov > 0 ? zscale(ov, 1.0 / aov) : zmk(1, 0);
    xi = zmul(xi, rot);  // same phase as the old vector
    double dd = t < k ? zabs2(zsub(xi, old)) : 0.0;
    for (int o = 32; o > 0; o >>= 1) dd += __shfl_xor(dd, o, 64);
    xr = t < k ? xi : zmk(0, 0);
    const double dist = sqrt(dd);
    if (dist <= 4e-15 || (it >= 8 && dist >= 0.5 * dprev)) { ++it; break; }
    dprev = dist;
  }
  if (t < k) x[t] = xr;
  __syncthreads();
  // theta = y^H H y and the residual ||H y - theta y|| (H re-read from global memory)
  zd hy = zmk(0, 0);
  if (t < k)
    for (int j = 0; j < k; ++j) hy = zadd(hy, zmul(H[(long long)t * ld + j], x[j]));
  const zd yt = t < k ? x[t] : zmk(0, 0);
  zd th = zcmul(yt, hy);
  for (int o = 32; o > 0; o >>= 1) {
    th.x += __shfl_xor(th.x, o, 64);
    th.y += __shfl_xor(th.y, o, 64);
  }
  double rr = t < k ? zabs2(zsub(hy, zmul(th, yt))) : 0.0;
  for (int o = 32; o > 0; o >>= 1) rr += __shfl_xor(rr, o, 64);
  // phase: the largest-modulus entry real positive (first one on ties)
  double a = t < k ? zabs2(yt) : -1.0;
  int am = t;
  for (int o = 32; o > 0; o >>= 1) {
    const double a2 = __shfl_xor(a, o, 64);
    const int m2 = __shfl_xor(am, o, 64);
    if (a2 > a || (a2 == a && m2 < am)) { a = a2; am = m2; }
  }
  const zd ph = zmk(__shfl(yt.x, am, 64), __shfl(yt.y, am, 64));
  const double aph = sqrt(zabs2(ph));
  const zd f = aph > 0 ? zscale(zconj(ph), 1.0 / aph) : zmk(1, 0);
  if (t < k) out[1 + t] = zmul(yt, f);
  if (t == 0) {
    out[0] = th;
    out[k + 1] = zmk(sqrt(rr), 0);
    info[0] = it;
  }
}

int ritz_near(const zd* H, int ld, int k, zd sigma, zd* out, int* info, hipStream_t st) {
  if (k < 1 || k > 64 || ld < k) return -1;
  hipLaunchKernelGGL(k_ritz_near, dim3(1), dim3(64), 0, st, H, ld, k, sigma, out, info);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int small_eig(const zd* A, int lda, int m, zd* w, zd* Y, int* info, hipStream_t st) {
  if (m < 1 || m > 64) return -1;
  hipLaunchKernelGGL(k_small_eig, dim3(1), dim3(64), 0, st, A, lda, m, w, Y, info);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
