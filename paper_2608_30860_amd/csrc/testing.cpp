// Kernel-level entry points declared in include/lind_internal.h (unit tests, per-kernel timing).
#include "kernels.hpp"
#include "../../include/lind_internal.h"

using namespace lindx;

extern "C" int lindx_gemm(int prec, int M, int N, int K, int nbatch, const void* A, long long lda, long long sA,
                          int opA, const void* B, long long ldb, long long sB, int opB, void* C, long long ldc,
                          double alpha_re, double alpha_im, int beta, int out64, void* stream) {
  if (!A || !B || !C || M < 0 || N < 0 || K < 1 || nbatch < 1 || prec < 0 || prec > 2) return -1;
  if ((opA != OP_N && opA != OP_C) || (opB != OP_N && opB != OP_C)) return -1;
  GemmDesc g;
  g.M = M; g.N = N; g.K = K; g.nbatch = nbatch;
  g.A = A; g.lda = lda; g.sA = sA; g.opA = opA;
  g.B = B; g.ldb = ldb; g.sB = sB; g.opB = opB;
  g.C = C; g.ldc = ldc;
  g.ar = alpha_re; g.ai = alpha_im; g.beta = beta; g.out64 = out64;
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
int schur_factor_ex(zd* A, zd* Z, int n, hipStream_t st, double* t_hess, double* t_qr, int stop_after_hessenberg);
}

extern "C" int lindx_schur(void* A, void* Z, int n, int stop_after_hessenberg, void* stream) {
  if (!A || !Z || n < 1) return -1;
  return schur_factor_ex((zd*)A, (zd*)Z, n, (hipStream_t)stream, nullptr, nullptr, stop_after_hessenberg);
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

extern "C" int lindx_trevec(const void* T, void* Y, int n, void* stream) {
  int rc = trevec((const zd*)T, (zd*)Y, n, (hipStream_t)stream);
  if (rc) return rc;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : -4;
}
extern "C" int lindx_triinv(const void* Y, void* Yinv, int n, void* stream) {
  int rc = triinv_unit((const zd*)Y, (zd*)Yinv, n, (hipStream_t)stream);
  if (rc) return rc;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : -4;
}
extern "C" int lindx_trisylv(const void* T, void* X, int n, double sr, double si, void* stream) {
  int rc = trisylv((const zd*)T, (zd*)X, n, zmk(sr, si), (hipStream_t)stream);
  if (rc) return rc;
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : -4;
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
