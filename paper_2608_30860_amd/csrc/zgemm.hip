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

// tile t of the upper triangle (bm <= bn) of a tm x tm grid, row-major, after the round robin
// over the 8 XCDs
__device__ inline void tile_upper64(int bid, int tm, int& bm, int& bn) {
  const int T = tm * (tm + 1) / 2;
  int t = ((T & 7) == 0) ? (bid & 7) * (T >> 3) + (bid >> 3) : bid;
  int r = 0;
  while (t >= tm - r) { t -= tm - r; ++r; }
  bm = r;
  bn = r + t;
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
  const int tiles = tm * tn;
  const int split = blockIdx.x / tiles;
  int bm, bn;
  tile_of(blockIdx.x - split * tiles, tm, tn, bm, bn);
  const int m0 = bm * BM, n0 = bn * BN;

  const CplxT* Ag = (const CplxT*)g.A;
  const CplxT* Bg = (const CplxT*)g.B;
  const int ktiles = (g.K + BK - 1) / BK;
  const int bps = g.nbatch / g.nsplit;
  const int it_begin = split * bps * ktiles;
  const int total = bps * ktiles;

  CplxT ra[EA], rb[EB];

  auto gload = [&](int itl) {
    const int it = it_begin + itl;
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
      T nai[TM];
#pragma unroll
      for (int i = 0; i < TM; ++i) nai[i] = -ai[i];
      // four real products per complex tile product, grouped so consecutive MFMAs use
      // independent accumulators
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) cr[i][j] = mfma(ar[i], br[j], cr[i][j]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) ci[i][j] = mfma(ar[i], bi[j], ci[i][j]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) cr[i][j] = mfma(nai[i], bi[j], cr[i][j]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) ci[i][j] = mfma(ai[i], br[j], ci[i][j]);
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
        if (g.nsplit > 1) {
          if (row < g.M && col < g.N) {
            CplxT* W = (CplxT*)g.ws + ((long long)split * g.M + row) * g.N + col;
            CplxT v;
            v.x = cr[i][j][r];
            v.y = ci[i][j][r];
            *W = v;
          }
        } else {
          epilogue_store<CplxOut>(g, row, col, (double)cr[i][j][r], (double)ci[i][j][r]);
        }
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

typedef __bf16 v8bf_t __attribute__((ext_vector_type(8)));

// Staging of one operand tile (R rows x 32 k, complex64) into four bf16 planes [plane][row][k]:
// each thread owns chunks of 8 consecutive k of one row.  KC: the k index is contiguous in
// memory (A as stored, B conjugate-transposed); otherwise the row index is (A^H, B as stored).
// CONJ: the operand is a conjugate transpose (A^H or B^H).
// Interior tiles take an unpredicated path (16-byte loads when KC and the rows are 16-byte
// aligned); edge tiles predicate every element.
// LDS rows hold 32 bf16 (64 bytes) with the four 16-byte k chunks XOR-swizzled by row bits 2..3,
// so 16 lanes reading one chunk of 16 consecutive rows (an MFMA operand) hit 16 distinct bank groups
__device__ inline int swz(int row, int k8) { return ((k8 ^ ((row >> 2) & 3)) << 3); }

template <int R, bool KC, bool CONJ>
struct Stage {
  static constexpr int CH = R * 4 / 256;  // chunks per thread (R * 32 / 8 / 256)
  float2 v[CH][8];
  __device__ inline void chunk(int c, int tid, int& row, int& k8) const {
    const int id = tid + c * 256;
    if (KC) { row = id >> 2; k8 = id & 3; }
    else { row = id % R; k8 = id / R; }
  }
  __device__ inline void load(const float2* __restrict__ base, long long ld, int rows_valid, int k_valid, int r0,
                              int k0, bool vec_ok, int tid) {
    const bool full = (r0 + R <= rows_valid) && (k0 + 32 <= k_valid);
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      int row, k8;
      chunk(c, tid, row, k8);
      const int gr = r0 + row;
      const int gk0 = k0 + k8 * 8;
      if (full) {
        if (KC) {
          const float2* p = base + (long long)gr * ld + gk0;
          if (vec_ok) {
            const float4* q = (const float4*)p;
#pragma unroll
            for (int h = 0; h < 4; ++h) {
              float4 x = q[h];
              v[c][2 * h] = make_float2(x.x, x.y);
              v[c][2 * h + 1] = make_float2(x.z, x.w);
            }
          } else {
#pragma unroll
            for (int i = 0; i < 8; ++i) v[c][i] = p[i];
          }
        } else {
          const float2* p = base + (long long)gk0 * ld + gr;
#pragma unroll
          for (int i = 0; i < 8; ++i) v[c][i] = p[(long long)i * ld];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int gk = gk0 + i;
          float2 x = make_float2(0.f, 0.f);
          if (gr < rows_valid && gk < k_valid) x = KC ? base[(long long)gr * ld + gk] : base[(long long)gk * ld + gr];
          v[c][i] = x;
        }
      }
      if (CONJ) {
#pragma unroll
        for (int i = 0; i < 8; ++i) v[c][i].y = -v[c][i].y;
      }
    }
  }
  __device__ inline void store(__bf16 (*S)[R][32], int tid) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      int row, k8;
      chunk(c, tid, row, k8);
      v8bf_t rh, rl, ih, il;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        __bf16 h = (__bf16)v[c][i].x;
        rh[i] = h;
        rl[i] = (__bf16)(v[c][i].x - (float)h);
        h = (__bf16)v[c][i].y;
        ih[i] = h;
        il[i] = (__bf16)(v[c][i].y - (float)h);
      }
      const int ko = swz(row, k8);
      *(v8bf_t*)&S[0][row][ko] = rh;
      *(v8bf_t*)&S[1][row][ko] = rl;
      *(v8bf_t*)&S[2][row][ko] = ih;
      *(v8bf_t*)&S[3][row][ko] = il;
    }
  }
};

template <int BM, int BN, bool AKC, bool BKC, typename CplxOut>
__global__ __launch_bounds__(256) void zgemm_bf16x3_kernel(GemmDesc g) {
  constexpr int BK = 32;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  // planes (0 re_hi, 1 re_lo, 2 im_hi, 3 im_lo) x rows x 32 bf16
  __shared__ __attribute__((aligned(16))) __bf16 As[4][BM][32];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[4][BN][32];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm0 = (wave >> 1) * WM;
  const int wn0 = (wave & 1) * WN;
  const int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  const int tiles = tm * tn;
  const int split = blockIdx.x / tiles;
  int bm, bn;
  tile_of(blockIdx.x - split * tiles, tm, tn, bm, bn);
  const int m0 = bm * BM, n0 = bn * BN;

  const float2* Ag = (const float2*)g.A;
  const float2* Bg = (const float2*)g.B;
  const int ktiles = (g.K + BK - 1) / BK;
  const int bps = g.nbatch / g.nsplit;
  const int it_begin = split * bps * ktiles;
  const int total = bps * ktiles;
  const bool vec_a = ((g.lda & 1) == 0) && ((g.sA & 1) == 0) && ((((unsigned long long)g.A) & 15) == 0);
  const bool vec_b = ((g.ldb & 1) == 0) && ((g.sB & 1) == 0) && ((((unsigned long long)g.B) & 15) == 0);

  Stage<BM, AKC, !AKC> sa;  // A^H: rows of A^H are columns of A (not k-contiguous), conjugated
  Stage<BN, BKC, BKC> sb;   // B^H: k-contiguous, conjugated
  auto gload = [&](int itl) {
    const int it = it_begin + itl;
    const int b = it / ktiles;
    const int k0 = (it - b * ktiles) * BK;
    sa.load(Ag + (long long)b * g.sA, g.lda, g.M, g.K, m0, k0, vec_a, tid);
    sb.load(Bg + (long long)b * g.sB, g.ldb, g.N, g.K, n0, k0, vec_b, tid);
  };

  v4f cr[TM][TN], ci[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      cr[i][j] = v4f{0, 0, 0, 0};
      ci[i][j] = v4f{0, 0, 0, 0};
    }

  const int kq = lane >> 4;  // which 8-wide k chunk this lane feeds to the MFMA
  if (total > 0) gload(0);
  for (int it = 0; it < total; ++it) {
    __syncthreads();
    sa.store(As, tid);
    sb.store(Bs, tid);
    __syncthreads();
    // prefetch the next stage into registers; the loads stay in flight during the MFMAs below
    if (it + 1 < total) gload(it + 1);
    v8bf br[TN][4], ar[TM][4], an[TM][2];
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int p = 0; p < 4; ++p)
        br[j][p] = *(const v8bf*)&Bs[p][wn0 + j * 16 + (lane & 15)][swz(wn0 + j * 16 + (lane & 15), kq)];
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int p = 0; p < 4; ++p) ar[i][p] = *(const v8bf*)&As[p][wm0 + i * 16 + (lane & 15)][swz(wm0 + i * 16 + (lane & 15), kq)];
      an[i][0] = negate8(ar[i][2]);
      an[i][1] = negate8(ar[i][3]);
    }
    // twelve bf16 products per complex tile product; each group below issues TM*TN independent
    // MFMAs so that no accumulator is used by two consecutive instructions
#define LX_GROUP(ACC, AOP, BP)                                        \
  _Pragma("unroll") for (int i = 0; i < TM; ++i)                      \
    _Pragma("unroll") for (int j = 0; j < TN; ++j) ACC[i][j] = mfma_bf(AOP, br[j][BP], ACC[i][j]);
    LX_GROUP(cr, ar[i][0], 0)   // re += Ar_hi Br_hi
    LX_GROUP(ci, ar[i][0], 2)   // im += Ar_hi Bi_hi
    LX_GROUP(cr, ar[i][0], 1)   // re += Ar_hi Br_lo
    LX_GROUP(ci, ar[i][0], 3)   // im += Ar_hi Bi_lo
    LX_GROUP(cr, ar[i][1], 0)   // re += Ar_lo Br_hi
    LX_GROUP(ci, ar[i][1], 2)   // im += Ar_lo Bi_hi
    LX_GROUP(cr, an[i][0], 2)   // re -= Ai_hi Bi_hi
    LX_GROUP(ci, ar[i][2], 0)   // im += Ai_hi Br_hi
    LX_GROUP(cr, an[i][0], 3)   // re -= Ai_hi Bi_lo
    LX_GROUP(ci, ar[i][2], 1)   // im += Ai_hi Br_lo
    LX_GROUP(cr, an[i][1], 2)   // re -= Ai_lo Bi_hi
    LX_GROUP(ci, ar[i][3], 0)   // im += Ai_lo Br_hi
#undef LX_GROUP
  }

#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int row = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        int col = n0 + wn0 + j * 16 + (lane & 15);
        if (g.nsplit > 1) {
          if (row < g.M && col < g.N)
            ((float2*)g.ws)[((long long)split * g.M + row) * g.N + col] = make_float2(cr[i][j][r], ci[i][j][r]);
        } else {
          epilogue_store<CplxOut>(g, row, col, (double)cr[i][j][r], (double)ci[i][j][r]);
        }
      }
}

// ---------------------------------------------------------------------------------------------
// FP64 kernel with direct-to-LDS staging.  Block tile 128 x 128, 16 complex k per stage, two LDS
// stages (2 x 64 KB): buffer_load_dwordx4 ... lds moves one complex128 per lane straight into LDS
// while the matrix cores work on the other stage.  Out-of-range rows and k come back as zeros from
// the bounds check of the buffer resource, so ragged edges need no separate path.
// Per operand the tile is held either "row-k" (rows = m or n, 16 k per 256-byte row, slot of k
// XOR-swizzled by the row's low four bits) when k is contiguous in memory (A as stored, B^H), or
// "k-row" (rows = k, 128 m or n per row) otherwise (A^H, B as stored); both give the 16 lanes of
// an MFMA operand read 16 distinct bank groups.  8 waves in a 2 x 4 grid of 64 x 32 sub-tiles.
// ---------------------------------------------------------------------------------------------
typedef __attribute__((address_space(3))) void lds_void_t;
constexpr int Z64_TB = 128, Z64_BK = 16;

template <bool AN, bool BN>
__global__ __launch_bounds__(512) void zgemm64_dma(GemmDesc g, int a_bytes, int b_bytes) {
  __shared__ __attribute__((aligned(1024))) double2 S[2][2][Z64_TB * Z64_BK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave >> 2) * 64, wn0 = (wave & 3) * 32;
  const int tm = (g.M + Z64_TB - 1) / Z64_TB, tn = (g.N + Z64_TB - 1) / Z64_TB;
  const int tiles = g.tri ? tm * (tm + 1) / 2 : tm * tn;
  const int split = blockIdx.x / tiles;
  int bm, bn;
  if (g.tri) tile_upper64(blockIdx.x - split * tiles, tm, bm, bn);
  else tile_of(blockIdx.x - split * tiles, tm, tn, bm, bn);
  const int m0 = bm * Z64_TB, n0 = bn * Z64_TB;
  const int ktiles = (g.K + Z64_BK - 1) / Z64_BK;
  const int bps = g.nbatch / g.nsplit;
  const int it_begin = split * bps * ktiles;
  const int total = bps * ktiles;

  // loader: waves 0-3 stage A, 4-7 stage B, 8 wave-loads of 64 elements (1 KB) each.  Lane l of
  // wave-load q writes LDS element 64 q + l of the operand's tile.
  const int lop = wave >> 2;
  const bool rk = lop ? !BN : AN;
  const long long ld = lop ? g.ldb : g.lda;
  const long long bstride = lop ? g.sB : g.sA;
  const int x0 = lop ? n0 : m0;
  const int xvalid = lop ? g.N : g.M;
  __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)(lop ? g.B : g.A), (short)0,
                                                                   lop ? b_bytes : a_bytes, 0x00020000);
  long long eoff[8];  // element offset of this lane's element for k0 = 0, batch 0
  int kk[8];          // its k within the stage
  bool rowok[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = (wave & 3) * 8 + u;
    if (rk) {
      const int r = 4 * q + (lane >> 4);
      const int k = (lane & 15) ^ (r & 15);
      kk[u] = k;
      rowok[u] = x0 + r < xvalid;
      eoff[u] = (long long)(x0 + r) * ld + k;
    } else {
      const int k = q >> 1;
      const int r = 64 * (q & 1) + lane;
      kk[u] = k;
      rowok[u] = x0 + r < xvalid;
      eoff[u] = (long long)k * ld + x0 + r;
    }
  }
  auto issue = [&](int itl, int buf) {
    const int it = it_begin + itl;
    const int b = it / ktiles;
    const int k0 = (it - b * ktiles) * Z64_BK;
    const long long kofs = rk ? (long long)k0 : (long long)k0 * ld;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = (wave & 3) * 8 + u;
      const bool ok = rowok[u] && (k0 + kk[u] < g.K);
      const unsigned off = ok ? (unsigned)((b * bstride + kofs + eoff[u]) * 16) : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t*)&S[buf][lop][64 * q], 16, off, 0, 0, 0);
    }
  };

  v4d cr[4][2], ci[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = v4d{0, 0, 0, 0};
      ci[i][j] = v4d{0, 0, 0, 0};
    }
  if (total > 0) issue(0, 0);
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    __syncthreads();  // this stage has landed; every wave is done with the other buffer
    if (it + 1 < total) issue(it + 1, buf ^ 1);
#pragma unroll
    for (int st = 0; st < 4; ++st) {
      const int k = 4 * st + (lane >> 4);
      double2 a[4], bq[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = wm0 + i * 16 + (lane & 15);
        a[i] = AN ? S[buf][0][m * 16 + (k ^ (m & 15))] : S[buf][0][k * 128 + m];
        if (!AN) a[i].y = -a[i].y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int nn = wn0 + j * 16 + (lane & 15);
        bq[j] = BN ? S[buf][1][k * 128 + nn] : S[buf][1][nn * 16 + (k ^ (nn & 15))];
        if (!BN) bq[j].y = -bq[j].y;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double nai = -a[i].y;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = mfma(a[i].x, bq[j].x, cr[i][j]);
          ci[i][j] = mfma(a[i].x, bq[j].y, ci[i][j]);
          cr[i][j] = mfma(nai, bq[j].y, cr[i][j]);
          ci[i][j] = mfma(a[i].y, bq[j].x, ci[i][j]);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm0 + i * 16 + 4 * r + (lane >> 4);
        const int col = n0 + wn0 + j * 16 + (lane & 15);
        if (g.nsplit > 1) {
          if (row < g.M && col < g.N)
            ((double2*)g.ws)[((long long)split * g.M + row) * g.N + col] = make_double2(cr[i][j][r], ci[i][j][r]);
        } else {
          epilogue_store<double2>(g, row, col, cr[i][j][r], ci[i][j][r]);
          // Hermitian result: entry (col, row) is the conjugate
          if (g.tri && bm < bn) epilogue_store<double2>(g, col, row, cr[i][j][r], -ci[i][j][r]);
        }
      }
}

// ---------------------------------------------------------------------------------------------
// FP32 kernel with direct-to-LDS staging: the FP64 kernel's structure at half the element size.
// Block tile 128 x 128, 32 complex k per stage (again 256-byte rows, two 64 KB LDS stages), each
// lane's 16-byte buffer_load ... lds moving two consecutive complex64 (two k in a "row-k" tile,
// whose 16-byte chunks are XOR-swizzled by the row's low four bits; two m or n in a "k-row" tile,
// one 1 KB row per wave-load).  Requires even K (and even M or N for an operand held k-row), even
// leading and batch strides and 16-byte aligned bases, so that a chunk never straddles the end of a
// row or of the operand.  8 waves of 64 x 32 on
// v_mfma_f32_16x16x4f32, FP32 accumulation.
// ---------------------------------------------------------------------------------------------
constexpr int Z32_BK = 32;

template <bool AN, bool BN, typename CplxOut>
__global__ __launch_bounds__(512) void zgemm32_dma(GemmDesc g, int a_bytes, int b_bytes) {
  __shared__ __attribute__((aligned(1024))) float2 S[2][2][Z64_TB * Z32_BK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave >> 2) * 64, wn0 = (wave & 3) * 32;
  const int tm = (g.M + Z64_TB - 1) / Z64_TB, tn = (g.N + Z64_TB - 1) / Z64_TB;
  const int tiles = tm * tn;
  const int split = blockIdx.x / tiles;
  int bm, bn;
  tile_of(blockIdx.x - split * tiles, tm, tn, bm, bn);
  const int m0 = bm * Z64_TB, n0 = bn * Z64_TB;
  const int ktiles = (g.K + Z32_BK - 1) / Z32_BK;
  const int bps = g.nbatch / g.nsplit;
  const int it_begin = split * bps * ktiles;
  const int total = bps * ktiles;

  // loader: waves 0-3 stage A, 4-7 stage B, 8 wave-loads of 1 KB each.  Lane l of wave-load q
  // writes bytes [16 l, 16 l + 16) of the operand tile's 1 KB block q.
  const int lop = wave >> 2;
  const bool rk = lop ? !BN : AN;
  const long long ld = lop ? g.ldb : g.lda;
  const long long bstride = lop ? g.sB : g.sA;
  const int x0 = lop ? n0 : m0;
  const int xvalid = lop ? g.N : g.M;
  __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)(lop ? g.B : g.A), (short)0,
                                                                   lop ? b_bytes : a_bytes, 0x00020000);
  long long eoff[8];  // element offset of this lane's first element for k0 = 0, batch 0
  int kk[8];          // its k within the stage
  bool rowok[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int q = (wave & 3) * 8 + u;
    if (rk) {
      // rows 4q .. 4q + 3, 16 chunks of two k each; slot (lane & 15) holds chunk slot ^ (r & 15)
      const int r = 4 * q + (lane >> 4);
      const int k = 2 * ((lane & 15) ^ (r & 15));
      kk[u] = k;
      rowok[u] = x0 + r < xvalid;
      eoff[u] = (long long)(x0 + r) * ld + k;
    } else {
      // row k = q, elements 2 lane and 2 lane + 1 of the 128 m (or n)
      kk[u] = q;
      rowok[u] = x0 + 2 * lane < xvalid;
      eoff[u] = (long long)q * ld + x0 + 2 * lane;
    }
  }
  auto issue = [&](int itl, int buf) {
    const int it = it_begin + itl;
    const int b = it / ktiles;
    const int k0 = (it - b * ktiles) * Z32_BK;
    const long long kofs = rk ? (long long)k0 : (long long)k0 * ld;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int q = (wave & 3) * 8 + u;
      const bool ok = rowok[u] && (k0 + kk[u] < g.K);
      const unsigned off = ok ? (unsigned)((b * bstride + kofs + eoff[u]) * 8) : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rsrc, (lds_void_t*)&S[buf][lop][128 * q], 16, off, 0, 0, 0);
    }
  };

  v4f cr[4][2], ci[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      cr[i][j] = v4f{0, 0, 0, 0};
      ci[i][j] = v4f{0, 0, 0, 0};
    }
  // element (x, k) of a row-k tile: row x, chunk k / 2 in slot (k / 2) ^ (x & 15)
  auto rk_at = [](int x, int k) { return x * Z32_BK + 2 * ((k >> 1) ^ (x & 15)) + (k & 1); };
  if (total > 0) issue(0, 0);
  for (int it = 0; it < total; ++it) {
    const int buf = it & 1;
    __syncthreads();  // this stage has landed; every wave is done with the other buffer
    if (it + 1 < total) issue(it + 1, buf ^ 1);
#pragma unroll
    for (int st = 0; st < Z32_BK / 4; ++st) {
      const int k = 4 * st + (lane >> 4);
      float2 a[4], bq[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = wm0 + i * 16 + (lane & 15);
        a[i] = AN ? S[buf][0][rk_at(m, k)] : S[buf][0][k * 128 + m];
        if (!AN) a[i].y = -a[i].y;
      }
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int nn = wn0 + j * 16 + (lane & 15);
        bq[j] = BN ? S[buf][1][k * 128 + nn] : S[buf][1][rk_at(nn, k)];
        if (!BN) bq[j].y = -bq[j].y;
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float nai = -a[i].y;
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, bq[j].x, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, bq[j].y, ci[i][j], 0, 0, 0);
          cr[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(nai, bq[j].y, cr[i][j], 0, 0, 0);
          ci[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, bq[j].x, ci[i][j], 0, 0, 0);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        // the FP32 MFMA leaves rows 4 (lane / 16) + r of a 16 x 16 block in a lane (FP64: 4 r + lane / 16)
        const int row = m0 + wm0 + i * 16 + 4 * (lane >> 4) + r;
        const int col = n0 + wn0 + j * 16 + (lane & 15);
        if (g.nsplit > 1) {
          if (row < g.M && col < g.N)
            ((float2*)g.ws)[((long long)split * g.M + row) * g.N + col] = make_float2(cr[i][j][r], ci[i][j][r]);
        } else {
          epilogue_store<CplxOut>(g, row, col, cr[i][j][r], ci[i][j][r]);
        }
      }
}

// ---------------------------------------------------------------------------------------------
// Phi of a small system in one workgroup (n <= 32, FP64, eigen route): Xh = (V^H xi V) / (s_a +
// conj s_b), then -sum_j Lt_j Xh Lt_j^H with each Lt_j staged in LDS in turn.  At this size the
// matrix work is a few microseconds of FP64 arithmetic and the general path's chain of launches
// would be all of the cost.  Thread t holds the entries t + 256 u (u < 4) of the 32 x 32 tile.
// ---------------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_phi_small(const zd* __restrict__ xi, const zd* __restrict__ V,
                                                   const zd* __restrict__ Lt, const zd* __restrict__ s,
                                                   const zd* __restrict__ sbar, int n, int d, zd* __restrict__ out) {
  __shared__ zd A[32][33], B[32][33], X[32][33];
  const int t = threadIdx.x;
  int er[4], eq[4];
  bool ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int e = t + 256 * u;
    er[u] = e >> 5;
    eq[u] = e & 31;
    ok[u] = er[u] < n && eq[u] < n;
    A[er[u]][eq[u]] = ok[u] ? xi[er[u] * n + eq[u]] : zmk(0, 0);
    B[er[u]][eq[u]] = ok[u] ? V[er[u] * n + eq[u]] : zmk(0, 0);
  }
  __syncthreads();
  // V^H xi
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    zd acc = zmk(0, 0);
    for (int k = 0; k < n; ++k) acc = zadd(acc, zcmul(B[k][er[u]], A[k][eq[u]]));
    X[er[u]][eq[u]] = acc;
  }
  __syncthreads();
  // Xh = (V^H xi V) / (s_a + conj s_b), into A
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    zd acc = zmk(0, 0);
    for (int k = 0; k < n; ++k) acc = zadd(acc, zmul(X[er[u]][k], B[k][eq[u]]));
    A[er[u]][eq[u]] = ok[u] ? zdiv(acc, zadd(s[er[u]], sbar[eq[u]])) : zmk(0, 0);
  }
  zd o[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) o[u] = zmk(0, 0);
  for (int j = 0; j < d; ++j) {
    __syncthreads();
    const zd* L = Lt + (long long)j * n * n;
#pragma unroll
    for (int u = 0; u < 4; ++u) B[er[u]][eq[u]] = ok[u] ? L[er[u] * n + eq[u]] : zmk(0, 0);
    __syncthreads();
    // Y = Lt_j Xh
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      zd acc = zmk(0, 0);
      for (int k = 0; k < n; ++k) acc = zadd(acc, zmul(B[er[u]][k], A[k][eq[u]]));
      X[er[u]][eq[u]] = acc;
    }
    __syncthreads();
    // += Y Lt_j^H
#pragma unroll
    for (int u = 0; u < 4; ++u)
      for (int k = 0; k < n; ++k) o[u] = zadd(o[u], zmul(X[er[u]][k], zconj(B[eq[u]][k])));
  }
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (ok[u]) out[er[u] * n + eq[u]] = zmk(-o[u].x, -o[u].y);
}

int phi_small(const zd* xi, const zd* V, const zd* Lt, const zd* s, const zd* sbar, int n, int d, zd* out,
              hipStream_t st) {
  if (n < 1 || n > 32 || d < 1) return -1;
  hipLaunchKernelGGL(k_phi_small, dim3(1), dim3(256), 0, st, xi, V, Lt, s, sbar, n, d, out);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// bytes an operand spans (batches included), or -1 past the reach of a 32-bit buffer offset
static long long z64_extent(long long rows, long long cols, long long ld, long long bstride, int nbatch) {
  if (rows <= 0 || cols <= 0) return 0;
  long long e = ((long long)(nbatch - 1) * bstride + (rows - 1) * ld + cols) * 16;
  return e < 0x7ff00000LL ? e : -1;
}

// sum the split-K partials and apply the epilogue
template <typename CplxAcc, typename CplxOut>
__global__ __launch_bounds__(256) void k_splitk_reduce(GemmDesc g) {
  const long long tot = (long long)g.M * g.N;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    const int row = (int)(t / g.N), col = (int)(t - (long long)row * g.N);
    // Hermitian result: below the diagonal tiles, the partials of the mirrored entry, conjugated
    const bool low = g.tri && (row / 128) > (col / 128);
    const long long src = low ? (long long)col * g.N + row : t;
    double re = 0, im = 0;
    for (int s = 0; s < g.nsplit; ++s) {
      CplxAcc v = ((const CplxAcc*)g.ws)[(long long)s * tot + src];
      re += v.x;
      im += v.y;
    }
    epilogue_store<CplxOut>(g, row, col, re, low ? -im : im);
  }
}

// ---------------------------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------------------------
template <typename K>
static int launch(K kern, int BM, int BN, const GemmDesc& g, hipStream_t st) {
  int tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  if (tm <= 0 || tn <= 0) return 0;
  hipLaunchKernelGGL(kern, dim3(tm * tn * g.nsplit), dim3(256), 0, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <int BM, int BN, typename Out>
static int launch_bf16(const GemmDesc& g, hipStream_t st) {
  const bool akc = g.opA == OP_N, bkc = g.opB != OP_N;
  if (akc && bkc) return launch(zgemm_bf16x3_kernel<BM, BN, true, true, Out>, BM, BN, g, st);
  if (akc && !bkc) return launch(zgemm_bf16x3_kernel<BM, BN, true, false, Out>, BM, BN, g, st);
  if (!akc && bkc) return launch(zgemm_bf16x3_kernel<BM, BN, false, true, Out>, BM, BN, g, st);
  return launch(zgemm_bf16x3_kernel<BM, BN, false, false, Out>, BM, BN, g, st);
}

template <typename Acc, typename Out>
static int launch_reduce(const GemmDesc& g, hipStream_t st) {
  long long tot = (long long)g.M * g.N;
  long long nb = (tot + 255) / 256;
  if (nb > 16384) nb = 16384;
  hipLaunchKernelGGL((k_splitk_reduce<Acc, Out>), dim3((int)nb), dim3(256), 0, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

// split count for a batch-reduction product: enough blocks to cover the chip twice
static int choose_split(int prec, int M, int N, int nbatch) {
  if (nbatch < 2) return 1;
  const int bm = 128, bn = (prec == PREC_F64) ? 64 : 128;
  long long tiles = (long long)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
  int s = 1;
  while (s * 2 <= nbatch && (nbatch % (s * 2)) == 0 && tiles * s < 1024) s *= 2;
  return s;
}

// tiles of the register-staged FP64 kernel for a product too small for 128 x 128 tiles: 64 x 64 when
// they reach half the chip, else 32 x 32
static int small_tile64(int M, int N, int nbatch) {
  return ((long long)((M + 63) / 64) * ((N + 63) / 64) * nbatch >= 128) ? 64 : 32;
}
static long long small_tiles(int M, int N, int bt) { return (long long)((M + bt - 1) / bt) * ((N + bt - 1) / bt); }
static bool f64_small(int M, int N, int nbatch) {
  return (long long)((M + 127) / 128) * ((N + 127) / 128) * nbatch < 96;
}
// chunks of K for a single small product whose tiles leave half the chip or more idle: the chunks
// become the batches of a reduction (partials in the workspace), up to 8, each at least 32 deep
static constexpr int kMaxKSplit = 8;
static int ksplit_for(int M, int N, int K, long long tiles, long long ws_avail, int elem) {
  int ks = 1;
  while (ks * 2 <= kMaxKSplit && tiles * ks * 2 <= 256 && K % (ks * 2) == 0 && K / (ks * 2) >= 32 &&
         (long long)(ks * 2) * M * N * elem <= ws_avail)
    ks *= 2;
  return ks;
}
// the FP32 products of this size run on 32 x 32 tiles of the register-staged kernel
static bool f32_small32(int M, int N) {
  return !(M >= 1024 && N >= 1024) && small_tiles(M, N, 64) < 96 && small_tiles(M, N, 32) <= 128;
}
// a single product described as ks batches of K / ks (the reduction sums them)
static void split_k_as_batches(GemmDesc& g, int ks) {
  const int kc = g.K / ks;
  g.K = kc;
  g.nbatch = ks;
  g.sA = g.opA == OP_N ? (long long)kc : (long long)kc * g.lda;
  g.sB = g.opB == OP_N ? (long long)kc * g.ldb : (long long)kc;
  g.nsplit = ks;
}

int gemm_small_ksplit(int prec, int M, int N, int K, long long ws_avail) {
  if (M <= 0 || N <= 0 || K <= 0) return 1;
  if (prec == PREC_F64) {
    if (!f64_small(M, N, 1)) return 1;
    const long long tiles = small_tiles(M, N, small_tile64(M, N, 1));
    return tiles <= 128 ? ksplit_for(M, N, K, tiles, ws_avail, 16) : 1;
  }
  if (prec == PREC_F32) return f32_small32(M, N) ? ksplit_for(M, N, K, small_tiles(M, N, 32), ws_avail, 8) : 1;
  return 1;
}

long long gemm_ws_bytes(int prec, int M, int N, int nbatch) {
  int s = choose_split(prec, M, N, nbatch);
  long long b = s > 1 ? (long long)s * M * N * (prec == PREC_F64 ? 16 : 8) : 0;
  if (prec == PREC_F64 && nbatch == 1 && f64_small(M, N, 1) && small_tiles(M, N, small_tile64(M, N, 1)) <= 128)
    b = std::max(b, (long long)kMaxKSplit * M * N * 16);
  if (prec == PREC_F32 && nbatch == 1 && f32_small32(M, N)) b = std::max(b, (long long)kMaxKSplit * M * N * 8);
  return b;
}

int gemm(int prec, const GemmDesc& g0, hipStream_t st) {
  if (g0.M <= 0 || g0.N <= 0) return 0;
  if (g0.K <= 0 || g0.nbatch <= 0) return -1;  // callers never ask for an empty reduction
  GemmDesc g = g0;
  if (prec != PREC_F64) g.tri = 0;
  g.nsplit = 1;
  if (g0.ws) {
    int s = choose_split(prec, g.M, g.N, g.nbatch);
    if (s > 1) g.nsplit = s;
  }
  int rc = 0;
  if (prec == PREC_F64) {
    const bool an = g.opA == OP_N, bn = g.opB == OP_N;
    const long long ea = an ? z64_extent(g.M, g.K, g.lda, g.sA, g.nbatch) : z64_extent(g.K, g.M, g.lda, g.sA, g.nbatch);
    const long long eb = bn ? z64_extent(g.K, g.N, g.ldb, g.sB, g.nbatch) : z64_extent(g.N, g.K, g.ldb, g.sB, g.nbatch);
    const bool aligned = (((unsigned long long)g.A | (unsigned long long)g.B) & 15) == 0;
    const long long ws_avail = g0.ws ? (g0.ws_bytes > 0 ? g0.ws_bytes : gemm_ws_bytes(PREC_F64, g.M, g.N, g.nbatch)) : 0;
    const long long t128 = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.nbatch;
    if (t128 < 96) {
      // too few 128 x 128 tiles (even split over every batch) to occupy the chip: 64 x 64 or
      // 32 x 32 tiles of the register-staged kernel, split-K over the batches
      g.tri = 0;
      const int bt = small_tile64(g.M, g.N, g.nbatch);
      const long long tiles = small_tiles(g.M, g.N, bt);
      int s = 1;
      if (g0.ws)
        while (s * 2 <= g.nbatch && (g.nbatch % (s * 2)) == 0 && tiles * s < 512 &&
               (long long)(s * 2) * g.M * g.N * 16 <= ws_avail)
          s *= 2;
      g.nsplit = s;
      if (g0.ws && g.nbatch == 1) {
        // one product on a few dozen tiles: its K chunks as the batches of a reduction
        const int ks = gemm_small_ksplit(PREC_F64, g.M, g.N, g.K, ws_avail);
        if (ks > 1) split_k_as_batches(g, ks);
      }
      rc = bt == 64 ? launch(zgemm_kernel<double, 64, 64, 16, double2>, 64, 64, g, st)
                    : launch(zgemm_kernel<double, 32, 32, 16, double2>, 32, 32, g, st);
      if (!rc && g.nsplit > 1) rc = launch_reduce<double2, double2>(g, st);
      return rc;
    }
    if (ea > 0 && eb > 0 && aligned) {
      // direct-to-LDS kernel; the split-K count is re-derived for its 128 x 128 tiles
      g.tri = (g0.tri && g.M == g.N && g.ai == 0.0) ? 1 : 0;
      if (g0.ws) {
        int s = 1;
        const long long tm0 = (g.M + 127) / 128;
        const long long t = g.tri ? tm0 * (tm0 + 1) / 2 : tm0 * ((g.N + 127) / 128);
        while (s * 2 <= g.nbatch && (g.nbatch % (s * 2)) == 0 && t * s < 1024 && (long long)(s * 2) * g.M * g.N * 16 <= ws_avail) s *= 2;
        g.nsplit = s;
      }
      const int tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
      const dim3 grid((g.tri ? tm * (tm + 1) / 2 : tm * tn) * g.nsplit), blk(512);
      if (an && bn) hipLaunchKernelGGL((zgemm64_dma<true, true>), grid, blk, 0, st, g, (int)ea, (int)eb);
      else if (an) hipLaunchKernelGGL((zgemm64_dma<true, false>), grid, blk, 0, st, g, (int)ea, (int)eb);
      else if (bn) hipLaunchKernelGGL((zgemm64_dma<false, true>), grid, blk, 0, st, g, (int)ea, (int)eb);
      else hipLaunchKernelGGL((zgemm64_dma<false, false>), grid, blk, 0, st, g, (int)ea, (int)eb);
      rc = hipGetLastError() == hipSuccess ? 0 : -4;
      if (!rc && g.nsplit > 1) rc = launch_reduce<double2, double2>(g, st);
      return rc;
    }
    g.tri = 0;  // the register-staged kernel computes every tile
    if (g.nsplit > 1 || (g.M >= 1024 && g.N >= 1024)) rc = launch(zgemm_kernel<double, 128, 64, 16, double2>, 128, 64, g, st);
    else rc = launch(zgemm_kernel<double, 64, 64, 16, double2>, 64, 64, g, st);
    if (!rc && g.nsplit > 1) rc = launch_reduce<double2, double2>(g, st);
    return rc;
  }
  if (prec == PREC_F32) {
    // direct-to-LDS kernel when the operands allow it and 128 x 128 tiles fill the chip
    {
      const bool an = g.opA == OP_N, bn = g.opB == OP_N;
      auto ext = [](long long rows, long long cols, long long ld, long long bs, int nb) -> long long {
        if (rows <= 0 || cols <= 0) return 0;
        const long long e = ((long long)(nb - 1) * bs + (rows - 1) * ld + cols) * 8;
        return e < 0x7ff00000LL ? e : -1;
      };
      const long long ea = an ? ext(g.M, g.K, g.lda, g.sA, g.nbatch) : ext(g.K, g.M, g.lda, g.sA, g.nbatch);
      const long long eb = bn ? ext(g.K, g.N, g.ldb, g.sB, g.nbatch) : ext(g.N, g.K, g.ldb, g.sB, g.nbatch);
      // a 16-byte chunk holds two k (row-k tile) or two m / n (k-row tile): those counts even, so
      // that no chunk reaches past its row or the operand
      const bool even = (g.K % 2 == 0) && (g.lda % 2 == 0) && (g.ldb % 2 == 0) && (g.sA % 2 == 0) &&
                        (g.sB % 2 == 0) && (an || g.M % 2 == 0) && (!bn || g.N % 2 == 0);
      const bool aligned = (((unsigned long long)g.A | (unsigned long long)g.B) & 15) == 0;
      const long long t128 = (long long)((g.M + 127) / 128) * ((g.N + 127) / 128) * g.nsplit;
      if (ea > 0 && eb > 0 && even && aligned && t128 >= 128) {
        const int tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
        const dim3 grid(tm * tn * g.nsplit), blk(512);
#define Z32_LAUNCH(OUT)                                                                                           \
  do {                                                                                                           \
    if (an && bn) hipLaunchKernelGGL((zgemm32_dma<true, true, OUT>), grid, blk, 0, st, g, (int)ea, (int)eb);       \
    else if (an) hipLaunchKernelGGL((zgemm32_dma<true, false, OUT>), grid, blk, 0, st, g, (int)ea, (int)eb);      \
    else if (bn) hipLaunchKernelGGL((zgemm32_dma<false, true, OUT>), grid, blk, 0, st, g, (int)ea, (int)eb);      \
    else hipLaunchKernelGGL((zgemm32_dma<false, false, OUT>), grid, blk, 0, st, g, (int)ea, (int)eb);             \
  } while (0)
        if (g.out64 && g.nsplit == 1) Z32_LAUNCH(double2);
        else Z32_LAUNCH(float2);
#undef Z32_LAUNCH
        rc = hipGetLastError() == hipSuccess ? 0 : -4;
        if (!rc && g.nsplit > 1) rc = g.out64 ? launch_reduce<float2, double2>(g, st) : launch_reduce<float2, float2>(g, st);
        return rc;
      }
    }
    if (g0.ws && g.nbatch == 1 && g.nsplit == 1) {
      // one product on a few dozen 32 x 32 tiles: its K chunks as the batches of a reduction
      const long long ws_avail = g0.ws_bytes > 0 ? g0.ws_bytes : gemm_ws_bytes(PREC_F32, g.M, g.N, 1);
      const int ks = gemm_small_ksplit(PREC_F32, g.M, g.N, g.K, ws_avail);
      if (ks > 1) split_k_as_batches(g, ks);
    }
    // 128 x 128 tiles for split or large products, else 64 x 64; 32 x 32 when the larger tiles
    // would leave most of the chip idle
    int bt = (g.nsplit > 1 || (g.M >= 1024 && g.N >= 1024)) ? 128 : 64;
    auto tiles = [&](int b) { return (long long)((g.M + b - 1) / b) * ((g.N + b - 1) / b) * g.nsplit; };
    if (tiles(bt) < 96 && tiles(32) > tiles(bt)) bt = 32;
    if (g.nsplit > 1) {
      rc = bt == 128 ? launch(zgemm_kernel<float, 128, 128, 16, float2>, 128, 128, g, st)
                     : launch(zgemm_kernel<float, 32, 32, 16, float2>, 32, 32, g, st);
      if (!rc) rc = g.out64 ? launch_reduce<float2, double2>(g, st) : launch_reduce<float2, float2>(g, st);
      return rc;
    }
    if (g.out64) {
      if (bt == 128) return launch(zgemm_kernel<float, 128, 128, 16, double2>, 128, 128, g, st);
      if (bt == 64) return launch(zgemm_kernel<float, 64, 64, 16, double2>, 64, 64, g, st);
      return launch(zgemm_kernel<float, 32, 32, 16, double2>, 32, 32, g, st);
    }
    if (bt == 128) return launch(zgemm_kernel<float, 128, 128, 16, float2>, 128, 128, g, st);
    if (bt == 64) return launch(zgemm_kernel<float, 64, 64, 16, float2>, 64, 64, g, st);
    return launch(zgemm_kernel<float, 32, 32, 16, float2>, 32, 32, g, st);
  }

  if (prec == PREC_BF16X3) {
    if (g.nsplit > 1) {
      rc = launch_bf16<128, 128, float2>(g, st);
      if (!rc) rc = g.out64 ? launch_reduce<float2, double2>(g, st) : launch_reduce<float2, float2>(g, st);
      return rc;
    }
    const bool big = g.M >= 1024 && g.N >= 1024;
    if (g.out64) return big ? launch_bf16<128, 128, double2>(g, st) : launch_bf16<64, 64, double2>(g, st);
    return big ? launch_bf16<128, 128, float2>(g, st) : launch_bf16<64, 64, float2>(g, st);
  }
  return -1;
}

}  // namespace lindx
