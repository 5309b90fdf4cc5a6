// Shared device/host helpers for the lindx HIP library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

namespace lindx {

// complex numbers as plain structs: double2 / float2 (x = re, y = im)
typedef double2 zd;
typedef float2 zf;

__host__ __device__ inline zd zmk(double r, double i) { zd z; z.x = r; z.y = i; return z; }
__host__ __device__ inline zf cmk(float r, float i) { zf z; z.x = r; z.y = i; return z; }
__host__ __device__ inline zd zadd(zd a, zd b) { return zmk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline zd zsub(zd a, zd b) { return zmk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline zd zmul(zd a, zd b) { return zmk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__host__ __device__ inline zd zconj(zd a) { return zmk(a.x, -a.y); }
__host__ __device__ inline zd zscale(zd a, double s) { return zmk(a.x * s, a.y * s); }
__host__ __device__ inline double zabs2(zd a) { return a.x * a.x + a.y * a.y; }
// conj(a) * b
__host__ __device__ inline zd zcmul(zd a, zd b) { return zmk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x); }
__host__ __device__ inline zd zdiv(zd a, zd b) {
  // Smith's algorithm
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, den = b.x + b.y * r;
    return zmk((a.x + a.y * r) / den, (a.y - a.x * r) / den);
  } else {
    double r = b.x / b.y, den = b.x * r + b.y;
    return zmk((a.x * r + a.y) / den, (a.y * r - a.x) / den);
  }
}

// Operand modes of a matrix product: N = as stored, C = conjugate transpose.
enum { OP_N = 0, OP_C = 2 };

}  // namespace lindx

#define LX_CHECK(expr)                                                              \
  do {                                                                              \
    hipError_t e__ = (expr);                                                        \
    if (e__ != hipSuccess) {                                                        \
      fprintf(stderr, "lindx: HIP error %s at %s:%d\n", hipGetErrorString(e__),     \
              __FILE__, __LINE__);                                                  \
      return -4;                                                                    \
    }                                                                               \
  } while (0)
