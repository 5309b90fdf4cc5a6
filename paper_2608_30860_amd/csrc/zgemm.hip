// Complex matrix products on CDNA4 matrix cores (gfx950).
//
// C = alpha * sum_b op(A_b) op(B_b) (+ C), with fused epilogues:
//   EPI_DIV       C_ij = alpha * acc_ij / (dr_i + dc_j + dz)      -- the elementwise divide of the
//                 eigenbasis Lyapunov solve (eq. lyapu_eig_solution), fused into the second
//                 basis-change product so the divided matrix never makes an extra HBM round trip
//   EPI_HERM_ADD  C_ij = alpha * acc_ij + E_ij + conj(E_ji)       -- adds P + P^H, used for the
//                 FP64 residual L(rho) = G rho + (G rho)^H + sum_j L_j rho L_j^H of a Hermitian rho
//
// A complex product is four real products on planar (re, im) tiles staged in LDS.
//  * FP64: v_mfma_f64_16x16x4f64, complex128 operands.
//  * FP32: v_mfma_f32_16x16x4f32, complex64 operands.
//  * BF16X3: each FP32 operand is split on the fly into hi = bf16(x), lo = bf16(x - hi)
//    (round to nearest even) and every real product is hi*hi + hi*lo + lo*hi with FP32
//    accumulation (v_mfma_f32_16x16x32_bf16): 12 bf16 products per complex tile product.
// The batch dimension b is a reduction: the d jump products sum_j Y_j L_j^H run as one launch
// whose K loop walks (j, k).
#include "kernels.hpp"

namespace lindx {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <typename T> struct CT;
template <> struct CT<double> { typedef double2 type; typedef v4d acc; };
template <> struct CT<float> { typedef float2 type; typedef v4f acc; };

__device__ inline v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline v4f mfma(float a, float b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Map a linear workgroup id to a (tile_m, tile_n) pair so that the workgroups that the
// dispatcher places on one XCD (ids congruent mod 8) get a contiguous run of tiles in
// row-major order and share A panels in that XCD's L2.
__device__ inline void tile_of(int bid, int tm, int tn, int& bm, int& bn) {
  int T = tm * tn;
  int t = bid;
  if ((T & 7) == 0) t = (bid & 7) * (T >> 3) + (bid >> 3);
  bm = t / tn;
  bn = t - bm * tn;
}

template <typename CplxOut>
__device__ inline void store_out(CplxOut* p, double re, double im);
template <> __device__ inline void store_out<double2>(double2* p, double re, double im) {
  *p = make_double2(re, im);
}
template <> __device__ inline void store_out<float2>(float2* p, double re, double im) {
  *p = make_float2((float)re, (float)im);
}
template <typename CplxIn>
__device__ inline double2 load_c(const CplxIn* p);
template <> __device__ inline double2 load_c<double2>(const double2* p) { return *p; }
template <> __device__ inline double2 load_c<float2>(const float2* p) {
  float2 v = *p;
  return make_double2(v.x, v.y);
}

template <typename CplxOut>
__device__ inline void epilogue_store(const GemmDesc& g, int row, int col, double cr, double ci) {
  if (row >= g.M || col >= g.N) return;
  double re = g.ar * cr - g.ai * ci;
  double im = g.ar * ci + g.ai * cr;
  if (g.epi == EPI_DIV) {
    zd den = zmk(g.dr[row].x + g.dc[col].x + g.dzr, g.dr[row].y + g.dc[col].y + g.dzi);
    zd q = zdiv(zmk(re, im), den);
    re = q.x;
    im = q.y;
  } else if (g.epi == EPI_HERM_ADD) {
    const CplxOut* E = (const CplxOut*)g.E;
    double2 e1 = load_c<CplxOut>(E + (long long)row * g.lde + col);
    double2 e2 = load_c<CplxOut>(E + (long long)col * g.lde + row);
    re += e1.x + e2.x;
    im += e1.y - e2.y;
  }
  CplxOut* C = (CplxOut*)g.C + (long long)row * g.ldc + col;
  if (g.beta) {
    double2 c0 = load_c<CplxOut>(C);
    re += c0.x;
    im += c0.y;
  }
  store_out<CplxOut>(C, re, im);
}

// ---------------------------------------------------------------------------------------------
// FP64 / FP32 kernel.  BM x BN block tile, BK complex entries of K per stage, 4 waves in a
// 2 x 2 grid each owning a (BM/2) x (BN/2) sub-tile of 16 x 16 MFMA tiles.
// LDS holds planar re/im tiles in [k][m] and [k][n] order, padded by PAD elements per row.
// Global -> register prefetch of the next stage overlaps the MFMAs of the current one.
// ---------------------------------------------------------------------------------------------
template <typename T, int BM, int BN, int BK, typename CplxOut>
__global__ __launch_bounds__(256) void zgemm_kernel(GemmDesc g) {
  typedef typename CT<T>::type CplxT;
  typedef typename CT<T>::acc Acc;
  constexpr int PAD = (sizeof(T) == 8) ? 1 : 2;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int EA = BM * BK / 256, EB = BK * BN / 256;
  __shared__ T As[2][BK][BM + PAD];
  __shared__ T Bs[2][BK][BN + PAD];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  int bm, bn;
  tile_of(blockIdx.x, tm, tn, bm, bn);
  const int m0 = bm * BM, n0 = bn * BN;

  const CplxT* Ag = (const CplxT*)g.A;
  const CplxT* Bg = (const CplxT*)g.B;
  const int ktiles = (g.K + BK - 1) / BK;
  const int total = ktiles * g.nbatch;

  CplxT ra[EA], rb[EB];

  auto gload = [&](int it) {
    const int b = it / ktiles;
    const int k0 = (it - b * ktiles) * BK;
    const CplxT* Ab = Ag + (long long)b * g.sA;
    const CplxT* Bb = Bg + (long long)b * g.sB;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + e * 256;
      int m, k;
      if (g.opA == OP_N) { m = idx / BK; k = idx - m * BK; }
      else { k = idx / BM; m = idx - k * BM; }
      int gm = m0 + m, gk = k0 + k;
      CplxT v;
      v.x = 0; v.y = 0;
      if (gm < g.M && gk < g.K) {
        if (g.opA == OP_N) v = Ab[(long long)gm * g.lda + gk];
        else { v = Ab[(long long)gk * g.lda + gm]; v.y = -v.y; }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + e * 256;
      int n, k;
      if (g.opB == OP_N) { k = idx / BN; n = idx - k * BN; }
      else { n = idx / BK; k = idx - n * BK; }
      int gn = n0 + n, gk = k0 + k;
      CplxT v;
      v.x = 0; v.y = 0;
      if (gn < g.N && gk < g.K) {
        if (g.opB == OP_N) v = Bb[(long long)gk * g.ldb + gn];
        else { v = Bb[(long long)gn * g.ldb + gk]; v.y = -v.y; }
      }
      rb[e] = v;
    }
  };

  // planar storage: separate arrays for re and im
  __shared__ T Ai_s[2][BK][BM + PAD];
  __shared__ T Bi_s[2][BK][BN + PAD];
  auto store_stage = [&](int buf) {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + e * 256;
      int m, k;
      if (g.opA == OP_N) { m = idx / BK; k = idx - m * BK; }
      else { k = idx / BM; m = idx - k * BM; }
      As[buf][k][m] = ra[e].x;
      Ai_s[buf][k][m] = ra[e].y;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + e * 256;
      int n, k;
      if (g.opB == OP_N) { k = idx / BN; n = idx - k * BN; }
      else { n = idx / BK; k = idx - n * BK; }
      Bs[buf][k][n] = rb[e].x;
      Bi_s[buf][k][n] = rb[e].y;
    }
  };

  Acc cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      cr[i][j] = Acc{0, 0, 0, 0};
      ci[i][j] = Acc{0, 0, 0, 0};
    }

  if (total > 0) {
    gload(0);
    store_stage(0);
  }
  __syncthreads();
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    if (it + 1 < total) gload(it + 1);
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      const int kr = kk + (lane >> 4);
      T ar[TM], ai[TM], br[TN], bi[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        ar[i] = As[buf][kr][wm0 + i * 16 + (lane & 15)];
        ai[i] = Ai_s[buf][kr][wm0 + i * 16 + (lane & 15)];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        br[j] = Bs[buf][kr][wn0 + j * 16 + (lane & 15)];
        bi[j] = Bi_s[buf][kr][wn0 + j * 16 + (lane & 15)];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        T nai = -ai[i];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          cr[i][j] = mfma(ar[i], br[j], cr[i][j]);
          cr[i][j] = mfma(nai, bi[j], cr[i][j]);
          ci[i][j] = mfma(ar[i], bi[j], ci[i][j]);
          ci[i][j] = mfma(ai[i], br[j], ci[i][j]);
        }
      }
    }
    if (it + 1 < total) store_stage(buf ^ 1);
    __syncthreads();
  }

  // accumulator layout of the 16 x 16 output tile: lane l, register r holds column l % 16 and
  // row 4*(l/16) + r for the FP32 instruction, row 4*r + l/16 for the FP64 instruction
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rr = (sizeof(T) == 8) ? (4 * r + (lane >> 4)) : (4 * (lane >> 4) + r);
        int row = m0 + wm0 + i * 16 + rr;
        int col = n0 + wn0 + j * 16 + (lane & 15);
        epilogue_store<CplxOut>(g, row, col, (double)cr[i][j][r], (double)ci[i][j][r]);
      }
}

// ---------------------------------------------------------------------------------------------
// BF16X3 kernel.  Operands complex64 in HBM; split into (hi, lo) bf16 planes while staging to
// LDS.  LDS rows are k-contiguous ([m][k], [n][k]) so one 16-byte read feeds one MFMA operand.
// ---------------------------------------------------------------------------------------------
__device__ inline void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

__device__ inline v8bf negate8(v8bf v) {
  v4u u = __builtin_bit_cast(v4u, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(v8bf, u);
}

__device__ inline v4f mfma_bf(v8bf a, v8bf b, v4f c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int BM, int BN, typename CplxOut>
__global__ __launch_bounds__(256) void zgemm_bf16x3_kernel(GemmDesc g) {
  constexpr int BK = 32;
  constexpr int KP = BK + 8;  // padded row length (bf16 elements), keeps 16-byte alignment
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int EA = BM * BK / 256, EB = BK * BN / 256;
  // planes: 0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo
  __shared__ __attribute__((aligned(16))) __bf16 As[4][BM][KP];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[4][BN][KP];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  int bm, bn;
  tile_of(blockIdx.x, tm, tn, bm, bn);
  const int m0 = bm * BM, n0 = bn * BN;

  const float2* Ag = (const float2*)g.A;
  const float2* Bg = (const float2*)g.B;
  const int ktiles = (g.K + BK - 1) / BK;
  const int total = ktiles * g.nbatch;

  float2 ra[EA], rb[EB];
  auto gload = [&](int it) {
    const int b = it / ktiles;
    const int k0 = (it - b * ktiles) * BK;
    const float2* Ab = Ag + (long long)b * g.sA;
    const float2* Bb = Bg + (long long)b * g.sB;
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + e * 256;
      int m, k;
      if (g.opA == OP_N) { m = idx / BK; k = idx - m * BK; }
      else { k = idx / BM; m = idx - k * BM; }
      int gm = m0 + m, gk = k0 + k;
      float2 v = make_float2(0.f, 0.f);
      if (gm < g.M && gk < g.K) {
        if (g.opA == OP_N) v = Ab[(long long)gm * g.lda + gk];
        else { v = Ab[(long long)gk * g.lda + gm]; v.y = -v.y; }
      }
      ra[e] = v;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + e * 256;
      int n, k;
      if (g.opB == OP_N) { k = idx / BN; n = idx - k * BN; }
      else { n = idx / BK; k = idx - n * BK; }
      int gn = n0 + n, gk = k0 + k;
      float2 v = make_float2(0.f, 0.f);
      if (gn < g.N && gk < g.K) {
        if (g.opB == OP_N) v = Bb[(long long)gk * g.ldb + gn];
        else { v = Bb[(long long)gn * g.ldb + gk]; v.y = -v.y; }
      }
      rb[e] = v;
    }
  };
  auto store_stage = [&]() {
#pragma unroll
    for (int e = 0; e < EA; ++e) {
      int idx = tid + e * 256;
      int m, k;
      if (g.opA == OP_N) { m = idx / BK; k = idx - m * BK; }
      else { k = idx / BM; m = idx - k * BM; }
      __bf16 h, l;
      split_bf16(ra[e].x, h, l);
      As[0][m][k] = h; As[1][m][k] = l;
      split_bf16(ra[e].y, h, l);
      As[2][m][k] = h; As[3][m][k] = l;
    }
#pragma unroll
    for (int e = 0; e < EB; ++e) {
      int idx = tid + e * 256;
      int n, k;
      if (g.opB == OP_N) { k = idx / BN; n = idx - k * BN; }
      else { n = idx / BK; k = idx - n * BK; }
      __bf16 h, l;
      split_bf16(rb[e].x, h, l);
      Bs[0][n][k] = h; Bs[1][n][k] = l;
      split_bf16(rb[e].y, h, l);
      Bs[2][n][k] = h; Bs[3][n][k] = l;
    }
  };

  v4f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      cr[i][j] = v4f{0, 0, 0, 0};
      ci[i][j] = v4f{0, 0, 0, 0};
    }

  const int kofs = 8 * (lane >> 4);
  for (int it = 0; it < total; ++it) {
    gload(it);
    __syncthreads();
    store_stage();
    __syncthreads();
    v8bf br[TN][4];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        br[j][p] = *(const v8bf*)&Bs[p][wn0 + j * 16 + (lane & 15)][kofs];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      v8bf a[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) a[p] = *(const v8bf*)&As[p][wm0 + i * 16 + (lane & 15)][kofs];
      v8bf nih = negate8(a[2]), nil = negate8(a[3]);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        // re: Ar Br - Ai Bi
        cr[i][j] = mfma_bf(a[0], br[j][0], cr[i][j]);
        cr[i][j] = mfma_bf(a[0], br[j][1], cr[i][j]);
        cr[i][j] = mfma_bf(a[1], br[j][0], cr[i][j]);
        cr[i][j] = mfma_bf(nih, br[j][2], cr[i][j]);
        cr[i][j] = mfma_bf(nih, br[j][3], cr[i][j]);
        cr[i][j] = mfma_bf(nil, br[j][2], cr[i][j]);
        // im: Ar Bi + Ai Br
        ci[i][j] = mfma_bf(a[0], br[j][2], ci[i][j]);
        ci[i][j] = mfma_bf(a[0], br[j][3], ci[i][j]);
        ci[i][j] = mfma_bf(a[1], br[j][2], ci[i][j]);
        ci[i][j] = mfma_bf(a[2], br[j][0], ci[i][j]);
        ci[i][j] = mfma_bf(a[2], br[j][1], ci[i][j]);
        ci[i][j] = mfma_bf(a[3], br[j][0], ci[i][j]);
      }
    }
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        int col = n0 + wn0 + j * 16 + (lane & 15);
        epilogue_store<CplxOut>(g, row, col, (double)cr[i][j][r], (double)ci[i][j][r]);
      }
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------
template <typename K>
static int launch(K kern, int BM, int BN, const GemmDesc& g, hipStream_t st) {
  int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  if (tm <= 0 || tn <= 0) return 0;
  hipLaunchKernelGGL(kern, dim3(tm * tn), dim3(256), 0, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int gemm(int prec, const GemmDesc& g, hipStream_t st) {
  if (g.M <= 0 || g.N <= 0) return 0;
  if (g.K <= 0 || g.nbatch <= 0) return -1;  // callers never ask for an empty reduction
  if (prec == PREC_F64) {
    if (g.M >= 1024 && g.N >= 1024) return launch(zgemm_kernel<double, 128, 64, 16, double2>, 128, 64, g, st);
    return launch(zgemm_kernel<double, 64, 64, 16, double2>, 64, 64, g, st);
  }
  if (prec == PREC_F32) {
    if (g.out64) return launch(zgemm_kernel<float, 64, 64, 16, double2>, 64, 64, g, st);
    if (g.M >= 1024 && g.N >= 1024) return launch(zgemm_kernel<float, 128, 128, 16, float2>, 128, 128, g, st);
    return launch(zgemm_kernel<float, 64, 64, 16, float2>, 64, 64, g, st);
  }
  if (prec == PREC_BF16X3) {
    if (g.out64) return launch(zgemm_bf16x3_kernel<64, 64, double2>, 64, 64, g, st);
    if (g.M >= 1024 && g.N >= 1024) return launch(zgemm_bf16x3_kernel<128, 128, float2>, 128, 128, g, st);
    return launch(zgemm_bf16x3_kernel<64, 64, float2>, 64, 64, g, st);
  }
  return -1;
}

}  // namespace lindx
