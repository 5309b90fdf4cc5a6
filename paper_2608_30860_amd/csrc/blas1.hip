// Bandwidth-bound kernels on complex128 n x n matrices and n^2-long Krylov vectors:
// Gram-Schmidt dot products and updates (FP64), norms, traces, hermitisation, conversions.
// All reductions are two-stage with a fixed order (no atomics), so results are deterministic.
#include "kernels.hpp"

namespace lindx {

static constexpr int RB = 256;      // threads per block
static constexpr int NPART = 1024;  // first-stage partial count

__device__ inline double warp_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}
__device__ inline double warp_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_down(v, o, 64));
  return v;
}
// block-wide sum of 256 threads; result valid in thread 0
__device__ inline double block_sum(double v, double* sh) {
  v = warp_sum(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return r;
}
__device__ inline double block_max(double v, double* sh) {
  v = warp_max(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = 0;
  if (threadIdx.x == 0) r = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
  __syncthreads();
  return r;
}

static int nparts(long long len) {
  long long p = (len + RB * 4 - 1) / (RB * 4);
  if (p > NPART) p = NPART;
  if (p < 1) p = 1;
  return (int)p;
}

// ---------------------------------------------------------------- multi-dot (Gram-Schmidt) ----
// stage 1 on a 2-D grid: block (x, y) takes row chunk x of every vector and the 8 basis vectors of
// group y, so a launch has (row chunks) x (k / 8) independent blocks; w's chunk is read once per
// group (it stays in L2 across the groups).  The 16 partial sums of a thread are reduced in one
// pass at the end (wave shuffles, one LDS exchange between the 4 waves).
static constexpr int MDG = 8;  // basis vectors per block
static int mdot_parts(long long len) {
  long long p = (len + 2047) / 2048;  // >= 8 rows per thread and vector
  if (p > NPART) p = NPART;
  if (p < 1) p = 1;
  return (int)p;
}
__global__ __launch_bounds__(RB) void k_mdot1(const zd* __restrict__ V, long long ld, int k,
                                              const zd* __restrict__ w, long long len,
                                              zd* __restrict__ part, int np) {
  __shared__ double sh[RB / 64][2 * MDG];
  const long long chunk = (len + np - 1) / np;
  const long long i0 = (long long)blockIdx.x * chunk;
  const long long i1 = i0 + chunk < len ? i0 + chunk : len;
  const int j0 = blockIdx.y * MDG;
  const int nv = k - j0 < MDG ? k - j0 : MDG;
  double sr[MDG], si[MDG];
#pragma unroll
  for (int t = 0; t < MDG; ++t) { sr[t] = 0; si[t] = 0; }
  const zd* Vb = V + (long long)j0 * ld;
  if (nv == MDG) {
    for (long long i = i0 + threadIdx.x; i < i1; i += RB) {
      const zd x = w[i];
#pragma unroll
      for (int t = 0; t < MDG; ++t) {
        const zd v = Vb[(long long)t * ld + i];
        sr[t] += v.x * x.x + v.y * x.y;
        si[t] += v.x * x.y - v.y * x.x;
      }
    }
  } else {
    for (long long i = i0 + threadIdx.x; i < i1; i += RB) {
      const zd x = w[i];
#pragma unroll
      for (int t = 0; t < MDG; ++t) {
        if (t < nv) {
          const zd v = Vb[(long long)t * ld + i];
          sr[t] += v.x * x.x + v.y * x.y;
          si[t] += v.x * x.y - v.y * x.x;
        }
      }
    }
  }
#pragma unroll
  for (int t = 0; t < MDG; ++t) {
    sr[t] = warp_sum(sr[t]);
    si[t] = warp_sum(si[t]);
  }
  const int wv = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int t = 0; t < MDG; ++t) { sh[wv][2 * t] = sr[t]; sh[wv][2 * t + 1] = si[t]; }
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int t = threadIdx.x;
    double a = 0, b = 0;
#pragma unroll
    for (int q = 0; q < RB / 64; ++q) { a += sh[q][2 * t]; b += sh[q][2 * t + 1]; }
    part[(long long)(j0 + t) * np + blockIdx.x] = zmk(a, b);
  }
}
__global__ __launch_bounds__(RB) void k_mdot2(const zd* __restrict__ part, int np, zd* __restrict__ h) {
  __shared__ double sh[4];
  int j = blockIdx.x;
  double a = 0, b = 0;
  for (int p = threadIdx.x; p < np; p += RB) {
    zd v = part[(long long)j * np + p];
    a += v.x;
    b += v.y;
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) h[j] = zmk(a, b);
}

int multi_dot(const zd* V, long long ld, int k, const zd* w, long long len, zd* h, zd* scratch,
              hipStream_t st) {
  if (k <= 0) return 0;
  const int np = mdot_parts(len);
  hipLaunchKernelGGL(k_mdot1, dim3(np, (k + MDG - 1) / MDG), dim3(RB), 0, st, V, ld, k, w, len, scratch, np);
  hipLaunchKernelGGL(k_mdot2, dim3(k), dim3(RB), 0, st, scratch, np, h);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ---------------------------------------------------------------- multi-axpy -----------------
__global__ __launch_bounds__(RB) void k_maxpy(const zd* __restrict__ V, long long ld, int k,
                                              const zd* __restrict__ h, zd* __restrict__ w,
                                              long long len, int accumulate, double coeff) {
  __shared__ zd hs[128];
  for (int t = threadIdx.x; t < k; t += RB) hs[t] = h[t];
  __syncthreads();
  long long stride = (long long)gridDim.x * RB;
  for (long long i = (long long)blockIdx.x * RB + threadIdx.x; i < len; i += stride) {
    double ar = 0, ai = 0;
    for (int j = 0; j < k; ++j) {
      zd v = V[(long long)j * ld + i];
      zd c = hs[j];
      ar += c.x * v.x - c.y * v.y;
      ai += c.x * v.y + c.y * v.x;
    }
    zd o = accumulate ? w[i] : zmk(0, 0);
    w[i] = zmk(o.x + coeff * ar, o.y + coeff * ai);
  }
}

int multi_axpy(const zd* V, long long ld, int k, const zd* h, zd* w, long long len, int accumulate,
               double coeff, hipStream_t st) {
  if (k > 128) return -1;
  long long nb = (len + RB - 1) / RB;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_maxpy, dim3((int)nb), dim3(RB), 0, st, V, ld, k, h, w, len, accumulate, coeff);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ---------------------------------------------------------------- norms ----------------------
__global__ __launch_bounds__(RB) void k_sumsq1(const zd* __restrict__ w, long long len, double* part, int np) {
  __shared__ double sh[4];
  long long chunk = (len + np - 1) / np;
  long long i0 = (long long)blockIdx.x * chunk;
  long long i1 = i0 + chunk < len ? i0 + chunk : len;
  double s = 0;
  for (long long i = i0 + threadIdx.x; i < i1; i += RB) {
    zd x = w[i];
    s += x.x * x.x + x.y * x.y;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(RB) void k_sqrt_sum2(const double* part, int np, double* out) {
  __shared__ double sh[4];
  double s = 0;
  for (int p = threadIdx.x; p < np; p += RB) s += part[p];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

int nrm2(const zd* w, long long len, double* out, double* scratch, hipStream_t st) {
  int np = nparts(len);
  hipLaunchKernelGGL(k_sumsq1, dim3(np), dim3(RB), 0, st, w, len, scratch, np);
  hipLaunchKernelGGL(k_sqrt_sum2, dim3(1), dim3(RB), 0, st, scratch, np, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_scale_inv(zd* w, long long len, const double* s) {
  double f = 1.0 / s[0];
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    zd x = w[i];
    w[i] = zmk(x.x * f, x.y * f);
  }
}
static int grid_for(long long len) {
  long long nb = (len + RB - 1) / RB;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  return (int)nb;
}
int scale_by_inv(zd* w, long long len, const double* s, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv, dim3(grid_for(len)), dim3(RB), 0, st, w, len, s);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// The end of Arnoldi step j: w <- w / s, and the step's column of the Hessenberg matrix written on
// the device, so that the host need not read it back at every step.  Workgroup 0 stores
// Hd[i][j] = h1[i] + h2[i] (i <= j, the two Gram-Schmidt passes), Hd[j+1][j] = s and sub[j] = s.
// A norm that is not positive (breakdown: w is exactly zero) leaves w as it is.
__global__ void k_scale_inv_hcol(zd* w, long long len, const double* s, const zd* h1, const zd* h2, zd* Hd,
                                 int ld, int j, double* sub) {
  const double sv = s[0];
  if (blockIdx.x == 0) {
    for (int i = threadIdx.x; i <= j; i += blockDim.x) {
      const zd a = h1[i], b = h2[i];
      Hd[(long long)i * ld + j] = zmk(a.x + b.x, a.y + b.y);
    }
    if (threadIdx.x == 0) {
      Hd[(long long)(j + 1) * ld + j] = zmk(sv, 0.0);
      sub[j] = sv;
    }
  }
  if (!(sv > 0)) return;
  const double f = 1.0 / sv;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    zd x = w[i];
    w[i] = zmk(x.x * f, x.y * f);
  }
}
int scale_by_inv_hcol(zd* w, long long len, const double* s, const zd* h1, const zd* h2, zd* Hd, int ld, int j,
                      double* sub, hipStream_t st) {
  hipLaunchKernelGGL(k_scale_inv_hcol, dim3(grid_for(len)), dim3(RB), 0, st, w, len, s, h1, h2, Hd, ld, j, sub);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// The whole CGS2 step of Arnoldi for a small system in one workgroup: w (len <= CG_MAXLEN
// entries) is held in LDS, each pass takes the k dot products with the basis (wave c of the
// workgroup owns basis vectors c, c + CG_W, ...) and then the update of w, and the step ends with
// the norm, the scaling and the Hessenberg column (the same outputs as scale_by_inv_hcol after
// two multi_dot / multi_axpy passes and nrm2).  Each basis vector is read once per dot and once
// per update from L2; no partial sums leave the workgroup, so one launch replaces eight.
static constexpr int CG_T = 1024;
static constexpr int CG_W = CG_T / 64;
static constexpr int CG_MAXLEN = 4096;
__global__ __launch_bounds__(CG_T) void k_cgs2_small(const zd* __restrict__ V, long long ld, int k,
                                                     zd* __restrict__ w, int len, zd* __restrict__ Hd, int ldh,
                                                     double* __restrict__ sub) {
  __shared__ zd ws[CG_MAXLEN];
  __shared__ zd hs[64];
  __shared__ double red[CG_W];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int i = t; i < len; i += CG_T) ws[i] = w[i];
  zd hacc = zmk(0.0, 0.0);
  __syncthreads();
  for (int pass = 0; pass < 2; ++pass) {
    for (int c = wv; c < k; c += CG_W) {
      const zd* Vc = V + (long long)c * ld;
      double sr = 0, si = 0;
      for (int i = lane; i < len; i += 64) {
        const zd v = Vc[i], x = ws[i];
        sr += v.x * x.x + v.y * x.y;
        si += v.x * x.y - v.y * x.x;
      }
      sr = warp_sum(sr);
      si = warp_sum(si);
      if (lane == 0) hs[c] = zmk(sr, si);
    }
    __syncthreads();
    if (t < k) hacc = zmk(hacc.x + hs[t].x, hacc.y + hs[t].y);
    for (int i = t; i < len; i += CG_T) {
      double ar = 0, ai = 0;
      for (int c = 0; c < k; ++c) {
        const zd v = V[(long long)c * ld + i], h = hs[c];
        ar += h.x * v.x - h.y * v.y;
        ai += h.x * v.y + h.y * v.x;
      }
      const zd x = ws[i];
      ws[i] = zmk(x.x - ar, x.y - ai);
    }
    __syncthreads();
  }
  double sq = 0;
  for (int i = t; i < len; i += CG_T) {
    const zd x = ws[i];
    sq += x.x * x.x + x.y * x.y;
  }
  sq = warp_sum(sq);
  if (lane == 0) red[wv] = sq;
  __syncthreads();
  double tot = 0;
  for (int q = 0; q < CG_W; ++q) tot += red[q];
  const double nrm = sqrt(tot);
  const int j = k - 1;
  if (t < k) Hd[(long long)t * ldh + j] = hacc;
  if (t == 0) {
    Hd[(long long)(j + 1) * ldh + j] = zmk(nrm, 0.0);
    sub[j] = nrm;
  }
  const double f = nrm > 0 ? 1.0 / nrm : 1.0;
  for (int i = t; i < len; i += CG_T) {
    const zd x = ws[i];
    w[i] = zmk(x.x * f, x.y * f);
  }
}
int cgs2_small(const zd* V, long long ld, int k, zd* w, long long len, zd* Hd, int ldh, double* sub, hipStream_t st) {
  if (len < 1 || len > CG_MAXLEN || k < 1 || k > 64) return -1;
  hipLaunchKernelGGL(k_cgs2_small, dim3(1), dim3(CG_T), 0, st, V, ld, k, w, (int)len, Hd, ldh, sub);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_axpby(zd a, const zd* x, zd b, zd* y, long long len) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    zd xv = x[i], yv = y[i];
    y[i] = zadd(zmul(a, xv), zmul(b, yv));
  }
}
int axpby(zd a, const zd* x, zd b, zd* y, long long len, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3(grid_for(len)), dim3(RB), 0, st, a, x, b, y, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
__global__ void k_copy(const zd* __restrict__ x, zd* __restrict__ y, long long len) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) y[i] = x[i];
}
// device-to-device copies of the solvers: a plain streaming kernel on the context's stream
int copy(const zd* x, zd* y, long long len, hipStream_t st) {
  if (len <= 0) return 0;
  hipLaunchKernelGGL(k_copy, dim3(grid_for(len)), dim3(RB), 0, st, x, y, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
__global__ void k_zero(unsigned int* p, long long nwords) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < nwords; i += stride) p[i] = 0u;
}
int fill_zero(void* p, long long bytes, hipStream_t st) {
  if (bytes <= 0) return 0;
  if (bytes % 4) return -1;
  hipLaunchKernelGGL(k_zero, dim3(grid_for(bytes / 4)), dim3(RB), 0, st, (unsigned int*)p, bytes / 4);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
__global__ void k_to64(const zd* x, zf* y, long long len) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    y[i] = make_float2((float)x[i].x, (float)x[i].y);
}
__global__ void k_to128(const zf* x, zd* y, long long len) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    y[i] = zmk(x[i].x, x[i].y);
}
int to_c64(const zd* x, zf* y, long long len, hipStream_t st) {
  hipLaunchKernelGGL(k_to64, dim3(grid_for(len)), dim3(RB), 0, st, x, y, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
int to_c128(const zf* x, zd* y, long long len, hipStream_t st) {
  hipLaunchKernelGGL(k_to128, dim3(grid_for(len)), dim3(RB), 0, st, x, y, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// ---------------------------------------------------------------- matrix helpers ------------
// X <- (X + X^H)/2 in place, in pairs of 32 x 32 tiles (bm <= bn): both tiles are read and
// written row by row, the transposed one through LDS
__global__ __launch_bounds__(RB) void k_hermitize(zd* X, int n) {
  __shared__ zd a[32][33], b[32][33];
  const int tn = (n + 31) / 32;
  int t = blockIdx.x, bm = 0;
  while (t >= tn - bm) { t -= tn - bm; ++bm; }
  const int bn = bm + t;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int r1 = bm * 32 + yy, c1 = bn * 32 + tx;  // upper tile
    const int r2 = bn * 32 + yy, c2 = bm * 32 + tx;  // lower tile
    a[yy][tx] = (r1 < n && c1 < n) ? X[(long long)r1 * n + c1] : zmk(0, 0);
    b[yy][tx] = (r2 < n && c2 < n) ? X[(long long)r2 * n + c2] : zmk(0, 0);
  }
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    // upper entry (r1, c1): (a[yy][tx] + conj(b[tx][yy])) / 2; its mirror is (c1, r1)
    const int r1 = bm * 32 + yy, c1 = bn * 32 + tx;
    const zd u = a[yy][tx], v = b[tx][yy];
    zd m = zmk(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
    if (r1 == c1) m.y = 0.0;
    if (r1 < n && c1 < n && (bm < bn || r1 <= c1)) X[(long long)r1 * n + c1] = m;
    // lower entry (r2, c2) = conj of upper entry (c2, r2) = (a[tx][yy] + conj(b[yy][tx])) / 2
    const int r2 = bn * 32 + yy, c2 = bm * 32 + tx;
    const zd u2 = a[tx][yy], v2 = b[yy][tx];
    const zd m2 = zmk(0.5 * (u2.x + v2.x), -0.5 * (u2.y - v2.y));
    if (r2 < n && c2 < n && (bm < bn || r2 > c2)) X[(long long)r2 * n + c2] = m2;
  }
}
__global__ __launch_bounds__(RB) void k_trace(const zd* X, int n, zd* out) {
  __shared__ double sh[4];
  double a = 0, b = 0;
  for (int i = threadIdx.x; i < n; i += RB) {
    zd v = X[(long long)i * n + i];
    a += v.x;
    b += v.y;
  }
  a = block_sum(a, sh);
  b = block_sum(b, sh);
  if (threadIdx.x == 0) out[0] = zmk(a, b);
}
__global__ void k_scale_by_trace(zd* X, long long len, const zd* tr) {
  double f = 1.0 / tr[0].x;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    zd x = X[i];
    X[i] = zmk(x.x * f, x.y * f);
  }
}
int hermitize(zd* X, int n, int normalize_trace, zd* trace_out, double* scratch, hipStream_t st) {
  (void)scratch;
  long long len = (long long)n * n;
  {
    const long long tn = (n + 31) / 32;
    hipLaunchKernelGGL(k_hermitize, dim3((int)(tn * (tn + 1) / 2)), dim3(RB), 0, st, X, n);
  }
  if (trace_out) hipLaunchKernelGGL(k_trace, dim3(1), dim3(RB), 0, st, X, n, trace_out);
  if (normalize_trace && trace_out)
    hipLaunchKernelGGL(k_scale_by_trace, dim3(grid_for(len)), dim3(RB), 0, st, X, len, trace_out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
int trace(const zd* X, int n, zd* out, double* scratch, hipStream_t st) {
  (void)scratch;
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(RB), 0, st, X, n, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// column sums of |x|^2 and column max |x| over row chunks
__global__ __launch_bounds__(RB) void k_colnorm1(const zd* X, int n, int rchunk, double* psum, double* pmax,
                                                 double* pdiag) {
  // block: 64 columns x 4 row groups
  __shared__ double ss[4][64], sm[4][64];
  int c = blockIdx.x * 64 + (threadIdx.x & 63);
  int rg = threadIdx.x >> 6;
  int r0 = blockIdx.y * rchunk;
  int r1 = r0 + rchunk < n ? r0 + rchunk : n;
  double s = 0, mx = 0, di = 0;
  if (c < n) {
    for (int r = r0 + rg; r < r1; r += 4) {
      zd v = X[(long long)r * n + c];
      double a2 = v.x * v.x + v.y * v.y;
      s += a2;
      mx = fmax(mx, a2);
      if (r == c) di = fabs(v.y);
    }
  }
  ss[rg][threadIdx.x & 63] = s;
  sm[rg][threadIdx.x & 63] = mx;
  (void)di;
  __syncthreads();
  if (rg == 0 && c < n) {
    double t = ss[0][threadIdx.x] + ss[1][threadIdx.x] + ss[2][threadIdx.x] + ss[3][threadIdx.x];
    double m = fmax(fmax(sm[0][threadIdx.x], sm[1][threadIdx.x]), fmax(sm[2][threadIdx.x], sm[3][threadIdx.x]));
    psum[(long long)blockIdx.y * n + c] = t;
    pmax[(long long)blockIdx.y * n + c] = m;
  }
  if (c < n && c >= r0 && c < r1 && pdiag) {
    // diagonal entry lives in this row chunk: record |Im x_cc|
    zd v = X[(long long)c * n + c];
    if (rg == 0) pdiag[c] = fabs(v.y);
  }
}
// per-column totals over the row chunks (one thread per column, contiguous across threads), then
// per-block partials of (sum |x|^2, sum of column 2-norms, max |x|^2, max |Im x_cc|)
__global__ __launch_bounds__(RB) void k_colnorm2(int n, int nrc, const double* psum, const double* pmax,
                                                 const double* pdiag, double* part) {
  __shared__ double sh[4];
  double fro = 0, mx = 0, colsum = 0, dmx = 0;
  const int c = blockIdx.x * RB + threadIdx.x;
  if (c < n) {
    double s = 0, m = 0;
    for (int r = 0; r < nrc; ++r) {
      s += psum[(long long)r * n + c];
      m = fmax(m, pmax[(long long)r * n + c]);
    }
    fro = s;
    mx = m;
    colsum = sqrt(s);
    dmx = pdiag[c];
  }
  fro = block_sum(fro, sh);
  colsum = block_sum(colsum, sh);
  mx = block_max(mx, sh);
  dmx = block_max(dmx, sh);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = fro;
    part[4 * blockIdx.x + 1] = colsum;
    part[4 * blockIdx.x + 2] = mx;
    part[4 * blockIdx.x + 3] = dmx;
  }
}
__global__ __launch_bounds__(RB) void k_colnorm3(int nb, const double* part, double* out) {
  __shared__ double sh[4];
  double fro = 0, mx = 0, colsum = 0, dmx = 0;
  for (int b = threadIdx.x; b < nb; b += RB) {
    fro += part[4 * b];
    colsum += part[4 * b + 1];
    mx = fmax(mx, part[4 * b + 2]);
    dmx = fmax(dmx, part[4 * b + 3]);
  }
  fro = block_sum(fro, sh);
  colsum = block_sum(colsum, sh);
  mx = block_max(mx, sh);
  dmx = block_max(dmx, sh);
  if (threadIdx.x == 0) {
    out[0] = sqrt(fro);
    out[1] = sqrt(mx);
    out[2] = colsum;
    out[3] = dmx;
  }
}
int mat_norms(const zd* X, int n, double* out, double* scratch, hipStream_t st) {
  int nrc = (n + 63) / 64;
  if (nrc > 32) nrc = 32;
  int rchunk = (n + nrc - 1) / nrc;
  double* psum = scratch;
  double* pmax = scratch + (long long)nrc * n;
  double* pdiag = scratch + 2LL * nrc * n;
  double* part = pdiag + n;
  const int nb = (n + RB - 1) / RB;
  hipLaunchKernelGGL(k_colnorm1, dim3((n + 63) / 64, nrc), dim3(RB), 0, st, X, n, rchunk, psum, pmax, pdiag);
  hipLaunchKernelGGL(k_colnorm2, dim3(nb), dim3(RB), 0, st, n, nrc, psum, pmax, pdiag, part);
  hipLaunchKernelGGL(k_colnorm3, dim3(1), dim3(RB), 0, st, nb, part, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_add_identity(zd* X, int n, zd c) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) X[(long long)i * n + i] = zadd(X[(long long)i * n + i], c);
}
int add_identity(zd* X, int n, zd c, hipStream_t st) {
  hipLaunchKernelGGL(k_add_identity, dim3((n + RB - 1) / RB), dim3(RB), 0, st, X, n, c);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
__global__ void k_add_identity_dev(zd* X, int n, const zd* t, zd c) {
  const zd a = zmul(c, t[0]);
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) X[(long long)i * n + i] = zadd(X[(long long)i * n + i], a);
}
int add_identity_trace(zd* X, int n, const zd* Y, zd c, zd* scratch_tr, hipStream_t st) {
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(RB), 0, st, Y, n, scratch_tr);
  hipLaunchKernelGGL(k_add_identity_dev, dim3((n + RB - 1) / RB), dim3(RB), 0, st, X, n, (const zd*)scratch_tr, c);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_sm_coef(const zd* trZ, zd c, zd trW, zd* coef) {
  // coef = c Tr(Z) / (1 - c Tr W)
  zd num = zmul(c, trZ[0]);
  zd den = zsub(zmk(1.0, 0.0), zmul(c, trW));
  coef[0] = zdiv(num, den);
}
__global__ void k_axpy_dev(const zd* coef, const zd* W, zd* Z, long long len) {
  zd a = coef[0];
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    Z[i] = zadd(Z[i], zmul(a, W[i]));
}
int sherman_morrison(zd* Z, const zd* W, int n, zd c, zd trW, zd* scratch_tr, double* scratch,
                     hipStream_t st) {
  (void)scratch;
  hipLaunchKernelGGL(k_trace, dim3(1), dim3(RB), 0, st, Z, n, scratch_tr);
  hipLaunchKernelGGL(k_sm_coef, dim3(1), dim3(1), 0, st, scratch_tr, c, trW, scratch_tr + 1);
  long long len = (long long)n * n;
  hipLaunchKernelGGL(k_axpy_dev, dim3(grid_for(len)), dim3(RB), 0, st, scratch_tr + 1, W, Z, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_make_G(const zd* H, const zd* W, zd* G, long long len) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) {
    zd h = H[i], w = W[i];
    // -i h - w/2
    G[i] = zmk(h.y - 0.5 * w.x, -h.x - 0.5 * w.y);
  }
}
int make_generator(const zd* H, const zd* W, zd* G, int n, hipStream_t st) {
  long long len = (long long)n * n;
  hipLaunchKernelGGL(k_make_G, dim3(grid_for(len)), dim3(RB), 0, st, H, W, G, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_scale_cols(zd* X, int n, const double* s, int invert) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    int j = (int)(t % n);
    double f = invert ? 1.0 / s[j] : s[j];
    X[t] = zscale(X[t], f);
  }
}
int scale_cols(zd* X, int n, const double* s, int invert, hipStream_t st) {
  long long len = (long long)n * n;
  hipLaunchKernelGGL(k_scale_cols, dim3(grid_for(len)), dim3(RB), 0, st, X, n, s, invert);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
// Euclidean norm of every column: 16 waves per block of 64 columns, wave w summing rows
// i = w (mod 16); the partial sums are added in a fixed order (deterministic).
static constexpr int CN_W = 16;
__global__ __launch_bounds__(64 * CN_W) void k_col_norms(const zd* X, int n, double* out) {
  __shared__ double ps[CN_W][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  double s = 0;
  if (j < n)
    for (int i = w; i < n; i += CN_W) s += zabs2(X[(long long)i * n + j]);
  ps[w][lane] = s;
  __syncthreads();
  if (w == 0 && j < n) {
    double t = 0;
    for (int q = 0; q < CN_W; ++q) t += ps[q][lane];
    out[j] = sqrt(t);
  }
}
int col_norms(const zd* X, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_col_norms, dim3((n + 63) / 64), dim3(64 * CN_W), 0, st, X, n, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// y = A x (one wave per row) or y = A^H x (one thread per column)
__global__ void k_gemv_n(const zd* A, int n, const zd* x, zd* y) {
  int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  int lane = threadIdx.x & 63;
  if (row >= n) return;
  double a = 0, b = 0;
  for (int j = lane; j < n; j += 64) {
    zd p = zmul(A[(long long)row * n + j], x[j]);
    a += p.x;
    b += p.y;
  }
  a = warp_sum(a);
  b = warp_sum(b);
  if (lane == 0) y[row] = zmk(a, b);
}
__global__ void k_gemv_c(const zd* A, int n, const zd* x, zd* y) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double a = 0, b = 0;
  for (int i = 0; i < n; ++i) {
    zd p = zcmul(A[(long long)i * n + j], x[i]);
    a += p.x;
    b += p.y;
  }
  y[j] = zmk(a, b);
}
// A^H x in two passes for large n: workgroup (column block, row chunk) sums 32 rows of 64
// columns into part[chunk][j]; the second pass adds the chunks (fixed order, deterministic)
static constexpr int GEMV_RC = 32;
__global__ void k_gemv_c_part(const zd* A, int n, const zd* x, zd* part) {
  const int j = blockIdx.x * 64 + threadIdx.x;
  const int i0 = blockIdx.y * GEMV_RC;
  if (j >= n) return;
  const int i1 = min(n, i0 + GEMV_RC);
  double a = 0, b = 0;
  for (int i = i0; i < i1; ++i) {
    zd p = zcmul(A[(long long)i * n + j], x[i]);
    a += p.x;
    b += p.y;
  }
  part[(long long)blockIdx.y * n + j] = zmk(a, b);
}
// second pass: 4 waves per 64 columns, wave w adding chunks c = w (mod 4); the four partial
// sums are then added in a fixed order (deterministic)
__global__ __launch_bounds__(256) void k_gemv_c_sum(const zd* part, int n, int chunks, zd* y) {
  __shared__ zd ps[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  double a = 0, b = 0;
  if (j < n)
    for (int c = w; c < chunks; c += 4) {
      const zd p = part[(long long)c * n + j];
      a += p.x;
      b += p.y;
    }
  ps[w][lane] = zmk(a, b);
  __syncthreads();
  if (w == 0 && j < n) y[j] = zadd(zadd(ps[0][lane], ps[1][lane]), zadd(ps[2][lane], ps[3][lane]));
}
long long gemv_scratch_elems(int n) { return (long long)((n + GEMV_RC - 1) / GEMV_RC) * n; }
int gemv(const zd* A, int n, int opA, const zd* x, zd* y, zd* scratch, hipStream_t st) {
  if (opA == OP_N) {
    hipLaunchKernelGGL(k_gemv_n, dim3((n + 3) / 4), dim3(256), 0, st, A, n, x, y);
  } else if (scratch && n > 2 * GEMV_RC) {
    const int chunks = (n + GEMV_RC - 1) / GEMV_RC;
    hipLaunchKernelGGL(k_gemv_c_part, dim3((n + 63) / 64, chunks), dim3(64), 0, st, A, n, x, scratch);
    hipLaunchKernelGGL(k_gemv_c_sum, dim3((n + 63) / 64), dim3(256), 0, st, (const zd*)scratch, n, chunks, y);
  } else {
    hipLaunchKernelGGL(k_gemv_c, dim3((n + 63) / 64), dim3(64), 0, st, A, n, x, y);
  }
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

__global__ void k_conj_copy(const zd* x, zd* y, long long len) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride) y[i] = zconj(x[i]);
}
int conj_copy(const zd* x, zd* y, long long len, hipStream_t st) {
  hipLaunchKernelGGL(k_conj_copy, dim3(grid_for(len)), dim3(RB), 0, st, x, y, len);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
__global__ void k_flip_ct(const zd* X, zd* Y, int n) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    int i = (int)(t / n), j = (int)(t - (long long)i * n);
    Y[t] = zconj(X[(long long)(n - 1 - j) * n + (n - 1 - i)]);
  }
}
__global__ void k_flip_rev(const zd* X, zd* Y, int n) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    int i = (int)(t / n), j = (int)(t - (long long)i * n);
    Y[t] = X[(long long)(n - 1 - i) * n + (n - 1 - j)];
  }
}
int flip_rev(const zd* X, zd* Y, int n, hipStream_t st) {
  long long len = (long long)n * n;
  hipLaunchKernelGGL(k_flip_rev, dim3(grid_for(len)), dim3(RB), 0, st, X, Y, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}
int flip_conj_transpose(const zd* X, zd* Y, int n, hipStream_t st) {
  long long len = (long long)n * n;
  hipLaunchKernelGGL(k_flip_ct, dim3(grid_for(len)), dim3(RB), 0, st, X, Y, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

}  // namespace lindx
