// Kernel-level entry points declared in include/lind_internal.h (unit tests, per-kernel timing).
#include "kernels.hpp"
#include "../../include/lind_internal.h"

using namespace lindx;

// the split-K run count of the pre-split BF16 product (host only, no device work)
extern "C" int lindx_p4_pick_split(long long tiles, int nbatch, int k_len, int cus) {
  if (tiles < 0 || nbatch < 0 || k_len < 0 || cus < 0) return -1;
  return p4_pick_split(tiles, nbatch, k_len, cus);
}

// the K-split plan of a single small product (host only, no device work)
extern "C" int lindx_gemm_ksplit(int prec, int M, int N, int K, long long ws_bytes) {
  if (prec < 0 || prec > 2) return -1;
  return gemm_small_ksplit(prec, M, N, K, ws_bytes);
}

extern "C" int lindx_gemm(int prec, int M, int N, int K, int nbatch, const void* A, long long lda, long long sA,
                          int opA, const void* B, long long ldb, long long sB, int opB, void* C, long long ldc,
                          double alpha_re, double alpha_im, int beta, int out64, int flags, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 1 || nbatch < 1 || prec < 0 || prec > 2) return -1;
  if ((opA != OP_N && opA != OP_C) || (opB != OP_N && opB != OP_C)) return -1;
  GemmDesc g;
  g.M = M; g.N = N; g.K = K; g.nbatch = nbatch;
  g.A = A; g.lda = lda; g.sA = sA; g.opA = opA;
  g.B = B; g.ldb = ldb; g.sB = sB; g.opB = opB;
  g.C = C; g.ldc = ldc;
  g.ar = alpha_re; g.ai = alpha_im; g.beta = beta; g.out64 = out64;
  g.tri = flags & 1;
  // a batch reduction that would split over K gets its workspace here (tests only)
  long long wsb = gemm_ws_bytes(prec, M, N, nbatch);
  void* ws = nullptr;
  if (wsb > 0) {
    if (hipMalloc(&ws, (size_t)wsb) != hipSuccess) return -5;
    g.ws = ws;
  }
  int rc = gemm(prec, g, (hipStream_t)stream);
  if (ws) {
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = -4;
    hipFree(ws);
  }
  return rc;
}

namespace lindx {
int schur_factor_ex(zd* A, zd* Z, int n, hipStream_t st, double* t_hess, double* t_qr, int mode);
}

extern "C" int lindx_schur(void* A, void* Z, int n, int mode, void* stream) {
  if (!A || !Z || n < 1) return -1;
  return schur_factor_ex((zd*)A, (zd*)Z, n, (hipStream_t)stream, nullptr, nullptr, mode);
}

extern "C" int lindx_small_eig(const void* A, int m, void* w, void* Y, void* stream) {
  if (!A || !w || m < 1 || m > 64) return -1;
  int* info = nullptr;
  if (hipMalloc(&info, sizeof(int)) != hipSuccess) return -5;
  int rc = small_eig((const zd*)A, m, m, (zd*)w, (zd*)Y, info, (hipStream_t)stream);
  int h = 0;
  if (!rc) rc = hipMemcpy(&h, info, sizeof(int), hipMemcpyDeviceToHost) == hipSuccess ? 0 : -4;
  hipFree(info);
  if (rc) return rc;
  return h ? -3 : 0;
}

static int with_square_ws(int n, int (*f)(const zd*, zd*, zd*, int, hipStream_t), const void* in, void* out,
                          void* stream) {
  if (n == 0) return 0;
  if (n < 0 || n > 10240) return -1;
  zd* ws = nullptr;
  if (hipMalloc(&ws, sizeof(zd) * (size_t)n * (size_t)n) != hipSuccess) return -5;
  int rc = f((const zd*)in, ws, (zd*)out, n, (hipStream_t)stream);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == 0) rc = -4;
  hipFree(ws);
  return rc;
}
// Ritz pair of an upper Hessenberg H (k x k complex128, device) nearest sigma (synchronous):
// out (device, k + 2 complex128) = [theta, y_1 .. y_k, (||H y - theta y||, 0)], iterations in *iters
extern "C" int lindx_ritz_near(const void* H, int k, double sr, double si, void* out, int* iters, void* stream) {
  if (!H || !out || k < 1 || k > 64) return -1;
  int* di = nullptr;
  if (hipMalloc(&di, sizeof(int)) != hipSuccess) return -5;
  int rc = ritz_near((const zd*)H, k, k, zmk(sr, si), (zd*)out, di, (hipStream_t)stream);
  if (!rc && iters && hipMemcpyAsync(iters, di, sizeof(int), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
    rc = -4;
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == 0) rc = -4;
  hipFree(di);
  return rc;
}

extern "C" int lindx_trevec(const void* T, void* Y, int n, void* stream) {
  return with_square_ws(n, trevec, T, Y, stream);
}
extern "C" int lindx_triinv(const void* Y, void* Yinv, int n, void* stream) {
  return with_square_ws(n, triinv_unit, Y, Yinv, stream);
}
extern "C" int lindx_trisylv(const void* T, void* X, int n, double sr, double si, void* stream) {
  zd* ws = nullptr;
  if (hipMalloc(&ws, sizeof(zd) * (size_t)trisylv_ws_elems(n > 0 ? n : 1)) != hipSuccess) return -5;
  int rc = trisylv((const zd*)T, (zd*)X, n, zmk(sr, si), ws, (hipStream_t)stream);
  if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess && rc == 0) rc = -4;
  hipFree(ws);
  if (rc) return rc;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : -4;
}

// the same solve with the block eigenbases of T's diagonal blocks for pairs whose condition
// numbers are <= thr; kap (host, optional, ceil(n / 32) doubles) receives those condition numbers
extern "C" int lindx_trisylv_blk(const void* T, void* X, int n, double sr, double si, double thr, double* kap,
                                 void* stream) {
  if (n < 1 || !T || !X) return -1;
  hipStream_t st = (hipStream_t)stream;
  const long long be = trisylv_blk_elems(n), nbk = (n + 31) / 32;
  zd *ws = nullptr, *y = nullptr, *yi = nullptr;
  double* kd = nullptr;
  int rc = 0;
  if (hipMalloc(&ws, sizeof(zd) * (size_t)trisylv_ws_elems(n)) != hipSuccess ||
      hipMalloc(&y, sizeof(zd) * (size_t)be) != hipSuccess || hipMalloc(&yi, sizeof(zd) * (size_t)be) != hipSuccess ||
      hipMalloc(&kd, sizeof(double) * (size_t)nbk) != hipSuccess)
    rc = -5;
  if (!rc) rc = trisylv_blk_setup((const zd*)T, n, y, yi, kd, st);
  TsBlk blk;
  blk.Y = y; blk.Yi = yi; blk.kap = kd; blk.thr = thr;
  if (!rc) rc = trisylv((const zd*)T, (zd*)X, n, zmk(sr, si), ws, st, &blk);
  if (!rc && kap && hipMemcpyAsync(kap, kd, sizeof(double) * (size_t)nbk, hipMemcpyDeviceToHost, st) != hipSuccess)
    rc = -4;
  if (hipStreamSynchronize(st) != hipSuccess && rc == 0) rc = -4;
  for (void* p : {(void*)ws, (void*)y, (void*)yi, (void*)kd})
    if (p) hipFree(p);
  return rc;
}

__global__ void k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, long long n) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}
extern "C" int lindx_copy(void* dst, const void* src, long long nbytes, void* stream) {
  if (!dst || !src || nbytes <= 0 || (nbytes % 16)) return -1;
  long long n = nbytes / 16;
  long long nb = (n + 255) / 256;
  if (nb > 65536) nb = 65536;
  hipLaunchKernelGGL(k_copy16, dim3((int)nb), dim3(256), 0, (hipStream_t)stream, (const uint4*)src, (uint4*)dst, n);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// C = sum_b op(A_b) op(B_b) through the pre-split BF16 product (complex128 in and out).
// op(A) = A_b (M x K, row-major) or A_b^H (A_b stored K x M); op(B) = B_b (K x N) or B_b^H
// (B_b stored N x K); batches are consecutive blocks.  out_mode: 0 planes, 1 transposed planes
// (both read back as complex128), 2 split-K partials reduced to complex128.  dr, dc (optional,
// planes modes): divide entry (m, n) by dr_m + dc_n.
extern "C" int lindx_p4_test(const void* A, const void* B, int M, int N, int K, int nbatch, int opA, int opB,
                             int out_mode, const void* dr, const void* dc, void* C, void* stream) {
  const int tri = (out_mode >> 2) & 1;  // bit 2: Hermitian result from the upper tiles
  out_mode &= 3;
  if (!A || !B || !C || M < 1 || N < 1 || K < 1 || nbatch < 1 || out_mode < 0 || out_mode > 2) return -1;
  if (tri && M != N) return -1;
  if ((opA != OP_N && opA != OP_C) || (opB != OP_N && opB != OP_C)) return -1;
  if (out_mode != 2 && nbatch != 1) return -1;
  hipStream_t st = (hipStream_t)stream;
  P4 pa, pb, pc;
  int rc = p4_alloc(pa, (long long)nbatch * M, K);
  if (!rc) rc = p4_alloc(pb, (long long)nbatch * N, K);
  if (!rc && out_mode != 2) rc = (out_mode == 0) ? p4_alloc(pc, M, N) : p4_alloc(pc, N, M);
  float2* ws = nullptr;
  int nsplit = 1;
  if (!rc && out_mode == 2) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) rc = -4;
    const long long tm = (M + 127) / 128, tn = (N + 127) / 128;
    nsplit = p4_pick_split(tri ? tm * (tm + 1) / 2 : tm * tn, nbatch, K, device_cus(dev));
    if (hipMalloc((void**)&ws, sizeof(float2) * (size_t)nsplit * M * N) != hipSuccess) rc = -5;
  }
  const zd* Ad = (const zd*)A;
  const zd* Bd = (const zd*)B;
  for (int b = 0; b < nbatch && !rc; ++b) {
    P4 sa = pa, sb = pb;
    sa.p = pa.p + (long long)b * M * pa.ld;
    sb.p = pb.p + (long long)b * N * pb.ld;
    // A planes: rows m, k contiguous
    if (opA == OP_N) rc = p4_split(Ad + (long long)b * M * K, 1, K, M, K, 0, 0, sa, st);
    else rc = p4_split(Ad + (long long)b * M * K, 1, M, K, M, 1, 0, sa, st);  // conjugated in the kernel
    if (rc) break;
    // B planes: rows n, k contiguous
    if (opB == OP_N) rc = p4_split(Bd + (long long)b * N * K, 1, N, K, N, 1, 0, sb, st);
    else rc = p4_split(Bd + (long long)b * N * K, 1, K, N, K, 0, 0, sb, st);  // conjugated in the kernel
  }
  if (!rc) {
    P4Desc g;
    g.M = M; g.N = N; g.K = K; g.nbatch = nbatch; g.nsplit = nsplit;
    g.A = pa.p; g.lda = pa.ld; g.pA = pa.pstride; g.sA = (long long)M * pa.ld;
    g.B = pb.p; g.ldb = pb.ld; g.pB = pb.pstride; g.sB = (long long)N * pb.ld;
    g.conjA = opA == OP_C;
    g.conjB = opB == OP_C;
    g.out = out_mode == 0 ? P4OUT_PLANES : (out_mode == 1 ? P4OUT_PLANES_T : P4OUT_WS);
    g.C = pc.p; g.ldc = pc.ld; g.pC = pc.pstride;
    g.dr = (const zd*)dr; g.dc = (const zd*)dc;
    g.ws = ws; g.out64 = C; g.ldo = N; g.alpha = 1.0;
    g.tri = tri;
    rc = p4_gemm(g, st);
    if (!rc && out_mode != 2) rc = p4_join(pc, M, N, out_mode == 1, (zd*)C, N, st);
  }
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = -4;
  for (void* p : {(void*)pa.p, (void*)pb.p, (void*)pc.p, (void*)ws})
    if (p) hipFree(p);
  return rc;
}


// One Gram-Schmidt step of the Arnoldi and GMRES drivers (classical, twice): h1 = V^H w,
// w -= V h1, h2 = V^H w, w -= V h2, nrm = ||w||, with the basis taken in chunks as the drivers do
// (64 vectors per dot launch, 128 per update launch).  h: device, 2k complex128 (h1 then h2).
extern "C" int lindx_cgs2(const void* V, long long ld, int k, void* w, long long len, void* h, void* nrm,
                          int reps, void* stream) {
  if (!V || !w || !h || !nrm || k < 1 || len < 1 || ld < len || reps < 1) return -1;
  hipStream_t st = (hipStream_t)stream;
  void* scr = nullptr;
  const size_t scr_bytes = sizeof(zd) * (size_t)64 * 1024 + 4096;
  if (hipMalloc(&scr, scr_bytes) != hipSuccess) return -5;
  const zd* Vz = (const zd*)V;
  zd* wz = (zd*)w;
  zd* hz = (zd*)h;
  int rc = 0;
  for (int r = 0; r < reps && !rc; ++r) {
    for (int pass = 0; pass < 2 && !rc; ++pass) {
      zd* hp = hz + (long long)pass * k;
      for (int c0 = 0; c0 < k && !rc; c0 += 64)
        rc = multi_dot(Vz + (long long)c0 * ld, ld, std::min(64, k - c0), wz, len, hp + c0, (zd*)scr, st);
      for (int c0 = 0; c0 < k && !rc; c0 += 128)
        rc = multi_axpy(Vz + (long long)c0 * ld, ld, std::min(128, k - c0), hp + c0, wz, len, 1, -1.0, st);
    }
    if (!rc) rc = nrm2(wz, len, (double*)nrm, (double*)scr, st);
  }
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = -4;
  hipFree(scr);
  return rc;
}

// The one-workgroup form of the same step used for small systems (len <= 4096, k <= 64): w is
// replaced by w2 / ||w2||; hcol (device, k + 1 complex128) receives the Hessenberg column
// (h1 + h2, then ||w2||) and nrm (device double) the norm as the driver's subdiagonal record.
extern "C" int lindx_cgs2_small(const void* V, long long ld, int k, void* w, long long len, void* hcol, void* nrm,
                                void* stream) {
  if (!V || !w || !hcol || !nrm || k < 1 || k > 64 || len < 1 || len > 4096 || ld < len) return -1;
  hipStream_t st = (hipStream_t)stream;
  zd* Hd = nullptr;
  double* sub = nullptr;
  if (hipMalloc(&Hd, sizeof(zd) * (size_t)(k + 1) * k) != hipSuccess) return -5;
  if (hipMalloc(&sub, sizeof(double) * (size_t)k) != hipSuccess) {
    hipFree(Hd);
    return -5;
  }
  int rc = cgs2_small((const zd*)V, ld, k, (zd*)w, len, Hd, k, sub, st);
  if (!rc && hipMemcpy2DAsync(hcol, sizeof(zd), Hd + (k - 1), sizeof(zd) * k, sizeof(zd), k + 1,
                              hipMemcpyDeviceToDevice, st) != hipSuccess)
    rc = -4;
  if (!rc && hipMemcpyAsync(nrm, sub + (k - 1), sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess) rc = -4;
  if (hipStreamSynchronize(st) != hipSuccess && !rc) rc = -4;
  hipFree(sub);
  hipFree(Hd);
  return rc;
}
