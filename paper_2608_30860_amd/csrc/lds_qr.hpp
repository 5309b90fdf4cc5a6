// Single-wave (64-lane) dense complex eigen-kernels on matrices held in LDS (m <= 64).
// Used for the Krylov projections (m x m Hessenberg / Krylov-Schur matrices), for the shifts
// of the multishift QR on G, and for the last small active blocks of that QR.
#pragma once
#include "common.hpp"

namespace lindx {

static constexpr int LDM = 65;  // LDS row stride for the <= 64 x 64 matrices

__device__ inline double cabs1(zd a) { return fabs(a.x) + fabs(a.y); }

// 1/sqrt(x) for x in the normal range: the hardware estimate y refined by one Newton-Raphson
// step carried to second order, y (1 + e/2 + 3 e^2/8) with e = 1 - x y^2 (the series of
// (1 - e)^(-1/2)), which leaves an error of order e^3 below double rounding.
__device__ inline double rsqrt_nr(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double e = fma(-x * y, y, 1.0);
  return fma(y * e, fma(0.375, e, 0.5), y);
}

// Givens rotation G = [[c, s], [-conj(s), c]] (c real) with G [f; g] = [r; 0].  It sits on the
// serial path of every bulge step, so the common case takes two reciprocal square roots and no
// division; squares near the ends of the exponent range take the exact square roots.
__device__ inline void zlartg(zd f, zd g, double& c, zd& s, zd& r) {
  const double f2 = zabs2(f), g2 = zabs2(g);
  if (g2 == 0.0) {
    c = 1.0; s = zmk(0, 0); r = f;
    return;
  }
  if (f2 == 0.0) {
    const double ag = sqrt(g2);
    c = 0.0;
    s = zscale(zconj(g), 1.0 / ag);
    r = zmk(ag, 0);
    return;
  }
  const double h2 = f2 + g2;
  if (f2 > 1e-280 && g2 > 1e-280 && h2 < 1e280) {
    const double ia = rsqrt_nr(f2), ih = rsqrt_nr(h2);
    const zd ph = zscale(f, ia);  // f / |f|
    c = (f2 * ia) * ih;
    s = zscale(zmul(ph, zconj(g)), ih);
    r = zscale(ph, h2 * ih);
    return;
  }
  const double af = sqrt(f2);
  const double nrm = sqrt(h2);
  const double inv_af = 1.0 / af, inv_n = 1.0 / nrm;
  const zd ph = zscale(f, inv_af);
  c = af * inv_n;
  s = zscale(zmul(ph, zconj(g)), inv_n);
  r = zscale(ph, nrm);
}

// rows (p, p+1) <- G rows, columns [c0, c1]
__device__ inline void rot_rows(zd* H, int ld, int p, int c0, int c1, double c, zd s) {
  int j = c0 + (int)(threadIdx.x & 63);
  for (; j <= c1; j += 64) {
    zd a = H[p * ld + j], b = H[(p + 1) * ld + j];
    H[p * ld + j] = zadd(zscale(a, c), zmul(s, b));
    H[(p + 1) * ld + j] = zsub(zscale(b, c), zmul(zconj(s), a));
  }
}
// columns (p, p+1) <- columns G^H, rows [r0, r1]
__device__ inline void rot_cols(zd* H, int ld, int p, int r0, int r1, double c, zd s) {
  int i = r0 + (int)(threadIdx.x & 63);
  for (; i <= r1; i += 64) {
    zd a = H[i * ld + p], b = H[i * ld + p + 1];
    H[i * ld + p] = zadd(zscale(a, c), zmul(zconj(s), b));
    H[i * ld + p + 1] = zsub(zscale(b, c), zmul(s, a));
  }
}

__device__ inline void wsync() { __syncthreads(); }

// Householder reduction of a dense m x m matrix in LDS to upper Hessenberg form, A <- Q^H A Q,
// accumulating Q (initialised by the caller).  Reflector P = I - 2 u u^H / (u^H u).
__device__ inline void hessenberg_lds(zd* A, zd* Q, int m, zd* u) {
  const int t = threadIdx.x & 63;
  for (int k = 0; k + 2 < m; ++k) {
    // column below the subdiagonal
    // the part below the subdiagonal on its own: ||x||^2 - |x0|^2 cancels to zero when it is
    // small against x0, and the column would be left unreduced
    double tail = 0;
    for (int i = k + 2; i < m; ++i) tail += zabs2(A[i * LDM + k]);
    if (!(tail > 0.0)) continue;  // already reduced
    const double nrm2 = zabs2(A[(k + 1) * LDM + k]) + tail;
    double nrm = sqrt(nrm2);
    zd x0 = A[(k + 1) * LDM + k];
    double ax0 = sqrt(zabs2(x0));
    zd ph = ax0 > 0 ? zscale(x0, 1.0 / ax0) : zmk(1, 0);
    wsync();
    for (int i = t; i < m; i += 64) u[i] = (i > k) ? A[i * LDM + k] : zmk(0, 0);
    wsync();
    if (t == 0) u[k + 1] = zadd(x0, zscale(ph, nrm));
    wsync();
    double uu = 0;
    for (int i = k + 1; i < m; ++i) uu += zabs2(u[i]);
    double gam = 2.0 / uu;
    // left: A[k+1:, :] -= gam u (u^H A)
    for (int j = t; j < m; j += 64) {
      zd w = zmk(0, 0);
      for (int i = k + 1; i < m; ++i) w = zadd(w, zcmul(u[i], A[i * LDM + j]));
      w = zscale(w, gam);
      for (int i = k + 1; i < m; ++i) A[i * LDM + j] = zsub(A[i * LDM + j], zmul(u[i], w));
    }
    wsync();
    // right: A[:, k+1:] -= gam (A u) u^H ; Q likewise
    for (int i = t; i < m; i += 64) {
      zd y = zmk(0, 0), yq = zmk(0, 0);
      for (int j = k + 1; j < m; ++j) {
        y = zadd(y, zmul(A[i * LDM + j], u[j]));
        yq = zadd(yq, zmul(Q[i * LDM + j], u[j]));
      }
      y = zscale(y, gam);
      yq = zscale(yq, gam);
      for (int j = k + 1; j < m; ++j) {
        A[i * LDM + j] = zsub(A[i * LDM + j], zmul(y, zconj(u[j])));
        Q[i * LDM + j] = zsub(Q[i * LDM + j], zmul(yq, zconj(u[j])));
      }
    }
    wsync();
    for (int i = k + 2 + t; i < m; i += 64) A[i * LDM + k] = zmk(0, 0);
    wsync();
  }
}

// Broadcast of lane l's complex value to the wave (l uniform): v_readlane into scalar registers.
__device__ inline zd zreadlane(zd v, int l) {
  const long long xr = __double_as_longlong(v.x), xi = __double_as_longlong(v.y);
  const int a0 = __builtin_amdgcn_readlane((int)xr, l), a1 = __builtin_amdgcn_readlane((int)(xr >> 32), l);
  const int b0 = __builtin_amdgcn_readlane((int)xi, l), b1 = __builtin_amdgcn_readlane((int)(xi >> 32), l);
  return zmk(__longlong_as_double(((long long)a1 << 32) | (unsigned)a0),
             __longlong_as_double(((long long)b1 << 32) | (unsigned)b0));
}

// Complex single-shift QR (Wilkinson shifts, exceptional shifts every 10 stalled sweeps) on an
// m x m upper Hessenberg matrix in LDS, m <= 64, run by ONE wave of 64 lanes.  With full != 0 the
// whole rows/columns are updated so the result is the Schur form T = Q^H H Q; Q (if non-null)
// accumulates the rotations.  Returns 0 on convergence, 1 otherwise.
//
// Lane j owns column j in a row rotation and row j in a column rotation.  The next rotation's
// input (column p, rows p+1 and p+2) comes out of the current column rotation in lanes p+1 and
// p+2 and is handed on by v_readlane, so each rotation costs two LDS round trips; one wave's LDS
// operations complete in order, so no barrier is needed between the phases.  The deflation test
// looks at all subdiagonal entries at once (one lane each) and takes the lowest split point from
// a ballot.
__device__ inline int qr_lds(zd* H, zd* Q, int m, int full) {
  const double ulp = 2.220446049250313e-16;
  const double smlnum = 1e-300;
  const int lane = threadIdx.x & 63;
  int ihi = m - 1;
  int its = 0, total = 0;
  __syncthreads();
  while (ihi > 0) {
    bool negl = false;
    if (lane >= 1 && lane <= ihi) {
      const zd sub = H[lane * LDM + lane - 1];
      const double tst = cabs1(H[(lane - 1) * LDM + lane - 1]) + cabs1(H[lane * LDM + lane]);
      negl = cabs1(sub) <= fmax(ulp * tst, smlnum);
    }
    const unsigned long long bal = __ballot(negl);
    const int l = bal ? 63 - __clzll(bal) : 0;
    if (l > 0 && lane == 0) H[l * LDM + l - 1] = zmk(0, 0);
    if (l == ihi) {
      ihi -= 1;
      its = 0;
      continue;
    }
    if (++total > 60 * m + 200) {
      __syncthreads();
      return 1;
    }
    zd sigma;
    const zd a = H[(ihi - 1) * LDM + ihi - 1], b = H[(ihi - 1) * LDM + ihi];
    const zd c = H[ihi * LDM + ihi - 1], d = H[ihi * LDM + ihi];
    if (its == 10 || its == 20) {
      sigma = zadd(d, zmk(1.5 * cabs1(c), 0.0));
    } else {
      // eigenvalue of [[a, b], [c, d]] nearest d
      const zd hm = zscale(zsub(a, d), 0.5);
      const zd disc = zadd(zmul(hm, hm), zmul(b, c));
      // principal square root of disc (non-negative real part) without trigonometry
      const double ad = sqrt(zabs2(disc));
      zd sq = zmk(0, 0);
      if (ad > 0) {
        if (disc.x >= 0) {
          const double re = sqrt(0.5 * (ad + disc.x));
          sq = zmk(re, disc.y / (2.0 * re));
        } else {
          const double im = copysign(sqrt(0.5 * (ad - disc.x)), disc.y);
          sq = zmk(disc.y / (2.0 * im), im);
        }
      }
      const zd e1 = zadd(zadd(d, hm), sq), e2 = zsub(zadd(d, hm), sq);
      sigma = (zabs2(zsub(e1, d)) <= zabs2(zsub(e2, d))) ? e1 : e2;
    }
    ++its;
    const int c1 = full ? m - 1 : ihi;
    const int r0 = full ? 0 : l;
    zd f = zsub(H[l * LDM + l], sigma);
    zd g = H[(l + 1) * LDM + l];
    for (int p = l; p < ihi; ++p) {
      double cs;
      zd sn, rr;
      zlartg(f, g, cs, sn, rr);
      // rows p, p+1 from column c0; the chased entry (p+1, p-1) becomes exactly zero
      const int c0 = (p == l) ? l : p - 1;
      if (lane >= c0 && lane <= c1) {
        const zd x = H[p * LDM + lane], y = H[(p + 1) * LDM + lane];
        H[p * LDM + lane] = zadd(zscale(x, cs), zmul(sn, y));
        H[(p + 1) * LDM + lane] = (p > l && lane == p - 1) ? zmk(0, 0) : zsub(zscale(y, cs), zmul(zconj(sn), x));
      }
      // columns p, p+1 for rows r0 .. min(p+2, ihi), and of Q; for m <= 32 the rows of Q ride
      // in lanes 32 .. 63 of the same instructions
      const int r1 = p + 2 < ihi ? p + 2 : ihi;
      zd nx = zmk(0, 0);
      if (Q && m <= 32) {
        const bool qh = lane >= 32;
        const int rr = lane & 31;
        zd* M = qh ? Q : H;
        if (qh ? rr < m : (rr >= r0 && rr <= r1)) {
          const zd x = M[rr * LDM + p], y = M[rr * LDM + p + 1];
          const zd nv = zadd(zscale(x, cs), zmul(zconj(sn), y));
          M[rr * LDM + p] = nv;
          M[rr * LDM + p + 1] = zsub(zscale(y, cs), zmul(sn, x));
          if (!qh) nx = nv;
        }
      } else {
        if (lane >= r0 && lane <= r1) {
          const zd x = H[lane * LDM + p], y = H[lane * LDM + p + 1];
          nx = zadd(zscale(x, cs), zmul(zconj(sn), y));
          H[lane * LDM + p] = nx;
          H[lane * LDM + p + 1] = zsub(zscale(y, cs), zmul(sn, x));
        }
        if (Q && lane < m) {
          const zd x = Q[lane * LDM + p], y = Q[lane * LDM + p + 1];
          Q[lane * LDM + p] = zadd(zscale(x, cs), zmul(zconj(sn), y));
          Q[lane * LDM + p + 1] = zsub(zscale(y, cs), zmul(sn, x));
        }
      }
      if (p + 1 < ihi) {
        f = zreadlane(nx, p + 1);
        g = zreadlane(nx, p + 2);
      }
    }
  }
  __syncthreads();
  return 0;
}

// Right eigenvectors of an upper-triangular T (m x m in LDS): column j of Y solves
// (T - T_jj) y = 0 with y_j = 1 (back substitution, lane j owns column j).
__device__ inline void trevec_lds(const zd* T, zd* Y, int m) {
  const double ulp = 2.220446049250313e-16;
  const int j = threadIdx.x & 63;
  if (j < m) {
    zd tjj = T[j * LDM + j];
    double smin = fmax(ulp * cabs1(tjj), 1e-290);
    for (int i = m - 1; i > j; --i) Y[i * LDM + j] = zmk(0, 0);
    Y[j * LDM + j] = zmk(1, 0);
    for (int i = j - 1; i >= 0; --i) {
      zd acc = T[i * LDM + j];
      for (int k = i + 1; k < j; ++k) acc = zadd(acc, zmul(T[i * LDM + k], Y[k * LDM + j]));
      zd den = zsub(T[i * LDM + i], tjj);
      if (cabs1(den) < smin) den = zmk(smin, 0);
      Y[i * LDM + j] = zdiv(zscale(acc, -1.0), den);
    }
  }
  wsync();
}

}  // namespace lindx
