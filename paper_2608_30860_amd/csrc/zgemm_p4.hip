// Complex products on pre-split BF16 operands (BF16x3 mode of the map Phi).
//
// An FP32-accurate complex operand Z is kept in HBM as four bf16 planes
//   [re_hi, re_lo, im_hi, im_lo],  hi = bf16(x), lo = bf16(x - hi)   (round to nearest even),
// each a rows x ld matrix with the reduction index k contiguous, rows and k zero-padded to the
// tile sizes.  Splitting once (constants at set-up, the Krylov vector once per Phi, every
// intermediate in the epilogue of the product that makes it) removes the per-tile conversion work
// of an on-the-fly split, and makes each stage a plain byte copy: global_load_lds_dwordx4 moves
// 16 bytes per lane straight into LDS, double-buffered, so the next stage streams in while the
// matrix cores work on the current one.
//
// Every real product is hi*hi + hi*lo + lo*hi with FP32 accumulation (v_mfma_f32_16x16x32_bf16):
// twelve MFMAs per complex 16 x 16 x 32 step.  Block tile 128 x 128, 8 waves of 64 x 32.
//
// Outputs: planes (the next product's A operand, row-major), transposed planes (the next
// product's B operand), or FP32 split-K partials reduced to complex128 by a second kernel.
#include "kernels.hpp"

namespace lindx {

typedef float v4f_p __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf_p __attribute__((ext_vector_type(8)));
typedef __bf16 v4bf_p __attribute__((ext_vector_type(4)));
typedef unsigned int v4u_p __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void;

namespace {

constexpr int TB = 128;  // block tile (both dimensions)
constexpr int KS = 32;   // k per stage

__device__ inline v8bf_p neg8(v8bf_p v) {
  v4u_p u = __builtin_bit_cast(v4u_p, v);
  u ^= 0x80008000u;
  return __builtin_bit_cast(v8bf_p, u);
}

__device__ inline v4f_p mfma16(v8bf_p a, v8bf_p b, v4f_p c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// 16-byte k chunk q of local row r sits in slot q ^ ((r >> 1) & 3) of the 64-byte LDS row.  An
// operand read takes 16 consecutive rows at one q (lane = row + 16 q); with this placement the
// read raises no LDS bank conflict on gfx950 (checked with the SQ_LDS_BANK_CONFLICT counter
// against the unswizzled and other XOR placements, which all conflict).
__device__ inline int slot_of(int r, int q) { return q ^ ((r >> 1) & 3); }

// s_waitcnt immediates (gfx9 encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8) that
// wait until at most 4 (0) LDS operations are outstanding and leave the other counters alone
constexpr int kLgkm4 = 0xC000 | 0x000F | 0x0070 | (4 << 8);
constexpr int kLgkm0 = 0xC000 | 0x000F | 0x0070;

// XCD-aware tile order: consecutive workgroup ids go to different XCDs (round robin over 8), so
// ids congruent mod 8 get a contiguous run of tiles.  When that run is whole tile rows, it is
// walked in column-major groups of 4 tile rows: the 32 workgroups an XCD runs at once then cover
// 4 x 8 tiles and share 4 A panels and 8 B panels in that XCD's L2 (2 x 16 for row-major order).
__device__ inline void tile_xcd(int bid, int tm, int tn, int& bm, int& bn) {
  const int T = tm * tn;
  int t = bid;
  if ((T & 7) == 0) {
    const int run = T >> 3;
    const int local = bid >> 3;
    t = (bid & 7) * run + local;
    constexpr int GH = 4;
    if (run % (GH * tn) == 0) {
      const int r0 = (bid & 7) * (run / tn);
      const int g = local / (GH * tn), w = local - g * GH * tn;
      bm = r0 + g * GH + w % GH;
      bn = w / GH;
      return;
    }
  }
  bm = t / tn;
  bn = t - bm * tn;
}

// tile t of the upper triangle (bm <= bn) of a tm x tm tile grid, row-major, after the same
// round robin over the 8 XCDs as tile_xcd
__device__ inline void tile_upper(int bid, int tm, int& bm, int& bn) {
  const int T = tm * (tm + 1) / 2;
  int t = ((T & 7) == 0) ? (bid & 7) * (T >> 3) + (bid >> 3) : bid;
  int r = 0;
  while (t >= tm - r) { t -= tm - r; ++r; }
  bm = r;
  bn = r + t;
}

__device__ inline void split_bf16(float x, __bf16& h, __bf16& l) {
  h = (__bf16)x;
  l = (__bf16)(x - (float)h);
}

// NW waves per block: 4 (2 x 2 waves of 64 x 64) or 8 (2 x 4 waves of 64 x 32, two waves per SIMD)
template <int NW, bool SWAP, bool CONJ_A, bool CONJ_B, int OUT>
__global__ __launch_bounds__(64 * NW) void k_p4_gemm(P4Desc g) {
  constexpr int TNW = NW == 4 ? 4 : 2;   // 16-wide n fragments per wave
  constexpr int LPW = 64 / NW;           // wave-loads (1 KB) per wave per stage
  // [stage][operand][plane][row][k]
  __shared__ __attribute__((aligned(1024))) __bf16 S[2][2][4][TB][KS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // wave-uniform values live in scalar registers: the stage loader's selections and addresses do
  // not go through vector memory (whose waits would also wait for the loads in flight)
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wm0 = (wave / (NW / 2)) * 64;
  const int wn0 = (wave % (NW / 2)) * (16 * TNW);
  const int tm = (g.M + TB - 1) / TB, tn = (g.N + TB - 1) / TB;
  const int tiles = g.tri ? tm * (tm + 1) / 2 : tm * tn;
  const int split = blockIdx.x / tiles;
  int bm, bn;
  if (g.tri) tile_upper(blockIdx.x - split * tiles, tm, bm, bn);
  else tile_xcd(blockIdx.x - split * tiles, tm, tn, bm, bn);
  const int m0 = bm * TB, n0 = bn * TB;
  const int ktiles = (g.K + KS - 1) / KS;
  // this workgroup's run of the (batch, k-chunk) steps
  const long long nit = (long long)g.nbatch * ktiles;
  const int it_begin = (int)(split * nit / g.nsplit);
  const int total = (int)((split + 1) * nit / g.nsplit) - it_begin;

  // stage loader: 64 wave-loads of 1 KB (operand, plane, 16-row group), LPW per wave: the first
  // half of the waves stage A, the second half B.  Lane l of a wave-load writes LDS
  // bytes [16 l, 16 l + 16) of the group: row l / 4, slot l % 4, i.e. k chunk slot_of(row, l % 4).
  const int lrow = lane >> 2;
  const int lslot = lane & 3;
  const int lop = wave / (NW / 2);
  const int pl0 = ((wave * LPW) >> 3) & 3;
  const __bf16* Xs = lop ? g.B : g.A;
  const long long xld = lop ? g.ldb : g.lda;
  const long long xp = lop ? g.pB : g.pA;
  const long long xs = lop ? g.sB : g.sA;
  const long long lane_off = (long long)((lop ? n0 : m0) + lrow) * xld + slot_of(lrow, lslot) * 8;
  auto issue = [&](int itl, int buf) {
    const int it = it_begin + itl;
    const int b = it / ktiles;
    const int k0 = (it - b * ktiles) * KS;
    const __bf16* base = Xs + (long long)b * xs + k0 + lane_off;
#pragma unroll
    for (int u = 0; u < LPW; ++u) {
      const int pl = pl0 + (u >> 3);
      const int q = u & 7;
      const __bf16* src = base + (long long)pl * xp + (long long)q * 16 * xld;
      __builtin_amdgcn_global_load_lds((const void*)src, (lds_void*)&S[buf][lop][pl][q * 16][0], 16, 0, 0);
    }
  };

  v4f_p cr[4][TNW], ci[4][TNW];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TNW; ++j) {
      cr[i][j] = v4f_p{0, 0, 0, 0};
      ci[i][j] = v4f_p{0, 0, 0, 0};
    }

  const int kq = lane >> 4;
  // operand fragments: A rows wm0 + 16 i (one 16-row block, all four planes), B rows wn0 + 16 j
  auto readA = [&](int buf, int i, v8bf_p (&ai)[4]) {
    const int r = wm0 + i * 16 + (lane & 15);
#pragma unroll
    for (int p = 0; p < 4; ++p) ai[p] = *(const v8bf_p*)&S[buf][0][p][r][slot_of(r, kq) * 8];
  };
  auto readB = [&](int buf, v8bf_p (&bb)[TNW][4]) {
#pragma unroll
    for (int j = 0; j < TNW; ++j) {
      const int r = wn0 + j * 16 + (lane & 15);
#pragma unroll
      for (int p = 0; p < 4; ++p) bb[j][p] = *(const v8bf_p*)&S[buf][1][p][r][slot_of(r, kq) * 8];
    }
  };
  // row block i of the wave tile, 12 TNW MFMAs: re += Ar Br - Ai Bi, im += Ar Bi + Ai Br.  The
  // conjugations change signs only: with conj(A) re += Ar Br + Ai Bi, im += Ar Bi - Ai Br; with
  // conj(B) the same pattern gives -im; with both, the plain pattern gives -im.  So the Ai planes
  // go with the plain signs into one accumulator and, negated in place (the fragment dies with
  // the block), into the other (XA picks which), and conj(B) negates im in the epilogue: no
  // operand is negated when it is read.  SWAP computes the transposed tile (B fragment as the MFMA
  // row operand), so that a lane's four accumulator entries run along n instead of m.
  constexpr bool XA = CONJ_A != CONJ_B;
  auto block = [&](int i, v8bf_p (&ai)[4], v8bf_p (&bb)[TNW][4]) {
#define P4_GROUP(ACC, AP, BP)                                                                  \
  _Pragma("unroll") for (int j = 0; j < TNW; ++j) ACC[i][j] =                                  \
      SWAP ? mfma16(bb[j][BP], ai[AP], ACC[i][j]) : mfma16(ai[AP], bb[j][BP], ACC[i][j]);
    P4_GROUP(cr, 0, 0)
    P4_GROUP(ci, 0, 2)
    P4_GROUP(cr, 0, 1)
    P4_GROUP(ci, 0, 3)
    P4_GROUP(cr, 1, 0)
    P4_GROUP(ci, 1, 2)
    if (XA) {
      P4_GROUP(cr, 2, 2)
      P4_GROUP(cr, 2, 3)
      P4_GROUP(cr, 3, 2)
    } else {
      P4_GROUP(ci, 2, 0)
      P4_GROUP(ci, 2, 1)
      P4_GROUP(ci, 3, 0)
    }
    ai[2] = neg8(ai[2]);
    ai[3] = neg8(ai[3]);
    if (XA) {
      P4_GROUP(ci, 2, 0)
      P4_GROUP(ci, 2, 1)
      P4_GROUP(ci, 3, 0)
    } else {
      P4_GROUP(cr, 2, 2)
      P4_GROUP(cr, 2, 3)
      P4_GROUP(cr, 3, 2)
    }
#undef P4_GROUP
  };
  // One stage s, with its B fragments and A blocks 0-2 already in registers.  The only barrier
  // comes after row block 0: by then every wave has read all of stage s (block 3 is read first)
  // and the DMA of stage s + 1 has landed, so stage s + 2 goes into this stage's buffer and the
  // fragments of stage s + 1 are read while blocks 1-3 keep the matrix cores busy.  All 24
  // fragment reads of a stage thus overlap MFMA work instead of stalling every wave at once.
  // The scheduling fences keep each read group where it stands: left alone, the compiler sinks the
  // reads next to their first use and waits for them there.
  auto step = [&](int s, v8bf_p (&A)[4][4], v8bf_p (&Bc)[TNW][4], v8bf_p (&An)[4][4], v8bf_p (&Bn)[TNW][4]) {
    const int buf = s & 1, nbuf = buf ^ 1;
    readA(buf, 3, A[3]);
    __builtin_amdgcn_sched_barrier(0);
    block(0, A[0], Bc);
    __builtin_amdgcn_sched_barrier(0);
    __syncthreads();
    if (s + 2 < total) issue(s + 2, buf);
    // on the last stage these read a buffer no DMA wrote: the values are never used
    readB(nbuf, Bn);
    readA(nbuf, 0, An[0]);
    __builtin_amdgcn_sched_barrier(0);
    block(1, A[1], Bc);
    __builtin_amdgcn_sched_barrier(0);
    readA(nbuf, 1, An[1]);
    __builtin_amdgcn_sched_barrier(0);
    block(2, A[2], Bc);
    __builtin_amdgcn_sched_barrier(0);
    // the 12 reads issued after the barrier have had two blocks to land.  Waiting for them here
    // (at most the 4 of block 1 still pending) keeps the LDS counter below its 4-bit limit: with
    // more reads in flight the compiler can only wait for all of them before the next block.
    __builtin_amdgcn_s_waitcnt(kLgkm4);
    readA(nbuf, 2, An[2]);
    __builtin_amdgcn_sched_barrier(0);
    block(3, A[3], Bc);
    __builtin_amdgcn_sched_barrier(0);
  };
  if (total > 0) {
    v8bf_p A0[4][4], A1[4][4], B0[TNW][4], B1[TNW][4];
    issue(0, 0);
    __syncthreads();
    if (total > 1) issue(1, 1);
    readB(0, B0);
    readA(0, 0, A0[0]);
    readA(0, 1, A0[1]);
    readA(0, 2, A0[2]);
    // nothing pending on entry to the loop, so that its first block waits for no more than the
    // loop's own back edge requires
    __builtin_amdgcn_s_waitcnt(kLgkm0);
    // unrolled by two so that the register sets alternate without copies
    int s = 0;
    for (; s + 1 < total; s += 2) {
      step(s, A0, B0, A1, B1);
      step(s + 1, A1, B1, A0, B0);
    }
    if (s < total) step(s, A0, B0, A1, B1);
  }

  // epilogue.  Normal: lane holds rows m = ..+4*(lane>>4)+r at column n = ..+(lane&15).
  // SWAP: lane holds columns n = ..+4*(lane>>4)+r at row m = ..+(lane&15).
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < TNW; ++j) {
      const int mb = m0 + wm0 + i * 16, nb = n0 + wn0 + j * 16;
      const int m_l = SWAP ? mb + (lane & 15) : mb + 4 * (lane >> 4);
      const int n_l = SWAP ? nb + 4 * (lane >> 4) : nb + (lane & 15);
      float re[4], im[4];
      int mm[4], nn[4];
      bool ok[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        mm[r] = SWAP ? m_l : m_l + r;
        nn[r] = SWAP ? n_l + r : n_l;
        ok[r] = mm[r] < g.M && nn[r] < g.N;
        re[r] = cr[i][j][r];
        im[r] = CONJ_B ? -ci[i][j][r] : ci[i][j][r];
      }
      if (OUT == P4OUT_WS) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (ok[r]) g.ws[((long long)split * g.M + mm[r]) * g.N + nn[r]] = make_float2(re[r], im[r]);
        continue;
      }
      if (g.dr) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!ok[r]) continue;
          const zd den = zmk(g.dr[mm[r]].x + g.dc[nn[r]].x, g.dr[mm[r]].y + g.dc[nn[r]].y);
          const zd q = zdiv(zmk(re[r], im[r]), den);
          re[r] = (float)q.x;
          im[r] = (float)q.y;
        }
      }
      v4bf_p h0, l0, h1, l1;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        __bf16 h, l;
        split_bf16(re[r], h, l);
        h0[r] = h; l0[r] = l;
        split_bf16(im[r], h, l);
        h1[r] = h; l1[r] = l;
      }
      // planes row-major [m][n] (P4OUT_PLANES, SWAP: four consecutive n) or transposed [n][m]
      // (P4OUT_PLANES_T, normal: four consecutive m)
      const long long base = (OUT == P4OUT_PLANES) ? (long long)m_l * g.ldc + n_l : (long long)n_l * g.ldc + m_l;
      const bool all = ok[0] && ok[1] && ok[2] && ok[3];
      if (g.tri && bm < bn) {
        // the conjugate of entry (mm, nn) is entry (nn, mm) of the Hermitian result
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!ok[r]) continue;
          const long long o = (OUT == P4OUT_PLANES) ? (long long)nn[r] * g.ldc + mm[r] : (long long)mm[r] * g.ldc + nn[r];
          g.C[o] = h0[r];
          g.C[g.pC + o] = l0[r];
          g.C[2 * g.pC + o] = -h1[r];
          g.C[3 * g.pC + o] = -l1[r];
        }
      }
      if (all) {
        *(v4bf_p*)(g.C + base) = h0;
        *(v4bf_p*)(g.C + g.pC + base) = l0;
        *(v4bf_p*)(g.C + 2 * g.pC + base) = h1;
        *(v4bf_p*)(g.C + 3 * g.pC + base) = l1;
      } else {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (!ok[r]) continue;
          g.C[base + r] = h0[r];
          g.C[g.pC + base + r] = l0[r];
          g.C[2 * g.pC + base + r] = h1[r];
          g.C[3 * g.pC + base + r] = l1[r];
        }
      }
    }
}

// sum of the FP32 split-K partials, scaled by alpha, into complex128 (row-major, ldo), in 32 x 32
// tiles: every partial row is read once, contiguously.  Hermitian result (tri): only the tiles on
// and above the diagonal are summed; each is written in place and, through an LDS transpose (so
// the stores stay contiguous too), as the conjugate of the tile below the diagonal.
__global__ __launch_bounds__(256) void k_p4_reduce(const float2* __restrict__ ws, int nsplit, int M, int N,
                                                   double alpha, zd* __restrict__ out, long long ldo, int tri) {
  __shared__ zd sh[32][33];
  const long long tot = (long long)M * N;
  const int tn = (N + 31) / 32;
  int bm, bn;
  if (tri) {
    int t = blockIdx.x, r = 0;
    while (t >= tn - r) { t -= tn - r; ++r; }
    bm = r;
    bn = r + t;
  } else {
    bm = blockIdx.x / tn;
    bn = blockIdx.x - bm * tn;
  }
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int yy = ty; yy < 32; yy += 8) {
    const int row = bm * 32 + yy, col = bn * 32 + tx;
    zd v = zmk(0, 0);
    if (row < M && col < N) {
      const long long o = (long long)row * N + col;
      double re = 0, im = 0;
      for (int sp = 0; sp < nsplit; ++sp) {
        const float2 p = ws[(long long)sp * tot + o];
        re += p.x;
        im += p.y;
      }
      v = zmk(alpha * re, alpha * im);
      if (tri && row == col) v.y = 0.0;
      // on a diagonal tile the entries below the diagonal come from the mirror below
      if (!tri || bm < bn || row <= col) out[(long long)row * ldo + col] = v;
    }
    sh[yy][tx] = v;
  }
  if (!tri) return;
  __syncthreads();
  for (int yy = ty; yy < 32; yy += 8) {
    // entry (bn*32 + yy, bm*32 + tx) of the lower tile is the conjugate of (bm*32 + tx, bn*32 + yy)
    const int row = bn * 32 + yy, col = bm * 32 + tx;
    if (row < M && col < N && (bm < bn || row > col)) {
      const zd v = sh[tx][yy];
      out[(long long)row * ldo + col] = zmk(v.x, -v.y);
    }
  }
}

// planes of op(X): out[r][k] = X[r][k] (or X[k][r] when transposed), conjugated on request;
// complex128 or complex64 input.  32 x 32 tiles through LDS so both sides stay coalesced.
template <typename Cplx, bool TRANS, bool CONJ>
__global__ __launch_bounds__(256) void k_p4_split(const Cplx* __restrict__ X, long long ldx, int rows, int cols,
                                                  __bf16* __restrict__ P, long long ld, long long pstride) {
  __shared__ float2 tile[32][33];
  // output extent: R rows x C k-columns
  const int R = TRANS ? cols : rows, C = TRANS ? rows : cols;
  const int tr = (R + 31) / 32;
  const int br = blockIdx.x % tr, bc = blockIdx.x / tr;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int r0 = br * 32, c0 = bc * 32;
  if (TRANS) {
    // X rows c0.., columns r0..: read X[c][r] coalesced along r, write out[r][c] along c
    for (int yy = ty; yy < 32; yy += 8) {
      const int c = c0 + yy, r = r0 + tx;
      float2 v = make_float2(0.f, 0.f);
      if (c < C && r < R) {
        const Cplx x = X[(long long)c * ldx + r];
        v = make_float2((float)x.x, (float)x.y);
      }
      tile[yy][tx] = v;
    }
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
      const int r = r0 + yy, c = c0 + tx;
      if (r < R && c < C) {
        float2 v = tile[tx][yy];
        if (CONJ) v.y = -v.y;
        __bf16 h, l;
        const long long o = (long long)r * ld + c;
        split_bf16(v.x, h, l);
        P[o] = h;
        P[pstride + o] = l;
        split_bf16(v.y, h, l);
        P[2 * pstride + o] = h;
        P[3 * pstride + o] = l;
      }
    }
  } else {
    for (int yy = ty; yy < 32; yy += 8) {
      const int r = r0 + yy, c = c0 + tx;
      if (r < R && c < C) {
        const Cplx x = X[(long long)r * ldx + c];
        float2 v = make_float2((float)x.x, (float)x.y);
        if (CONJ) v.y = -v.y;
        __bf16 h, l;
        const long long o = (long long)r * ld + c;
        split_bf16(v.x, h, l);
        P[o] = h;
        P[pstride + o] = l;
        split_bf16(v.y, h, l);
        P[2 * pstride + o] = h;
        P[3 * pstride + o] = l;
      }
    }
  }
}

// complex128 value of planes: X[r][c] = (re_hi + re_lo, im_hi + im_lo) of P[r][c] (or of P[c][r])
__global__ __launch_bounds__(256) void k_p4_join(const __bf16* __restrict__ P, long long ld, long long pstride,
                                                 int rows, int cols, int trans, zd* __restrict__ X, long long ldx) {
  const long long tot = (long long)rows * cols;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    const int r = (int)(t / cols), c = (int)(t - (long long)r * cols);
    const long long o = trans ? (long long)c * ld + r : (long long)r * ld + c;
    const double re = (double)(float)P[o] + (double)(float)P[pstride + o];
    const double im = (double)(float)P[2 * pstride + o] + (double)(float)P[3 * pstride + o];
    X[(long long)r * ldx + c] = zmk(re, im);
  }
}

template <int NW, bool SWAP, int OUT>
int launch_p4_nw(const P4Desc& g, int blocks, hipStream_t st) {
  if (g.conjA && g.conjB) hipLaunchKernelGGL((k_p4_gemm<NW, SWAP, true, true, OUT>), dim3(blocks), dim3(64 * NW), 0, st, g);
  else if (g.conjA) hipLaunchKernelGGL((k_p4_gemm<NW, SWAP, true, false, OUT>), dim3(blocks), dim3(64 * NW), 0, st, g);
  else if (g.conjB) hipLaunchKernelGGL((k_p4_gemm<NW, SWAP, false, true, OUT>), dim3(blocks), dim3(64 * NW), 0, st, g);
  else hipLaunchKernelGGL((k_p4_gemm<NW, SWAP, false, false, OUT>), dim3(blocks), dim3(64 * NW), 0, st, g);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

template <bool SWAP, int OUT>
int launch_p4_out(const P4Desc& g, int blocks, hipStream_t st) {
  // 8 waves per block (two per SIMD) hide the LDS-read latency of one wave behind the other's
  // matrix-core work
  return launch_p4_nw<8, SWAP, OUT>(g, blocks, st);
}

}  // namespace

long long p4_rows_alloc(long long rows) { return (rows + TB - 1) / TB * TB + TB; }
long long p4_ld(long long k) { return (k + KS - 1) / KS * KS; }

int p4_alloc(P4& p, long long rows, long long k) {
  p.rows = p4_rows_alloc(rows);
  p.ld = p4_ld(k);
  p.pstride = p.rows * p.ld;
  const size_t bytes = (size_t)(4 * p.pstride) * sizeof(__bf16);
  if (hipMalloc((void**)&p.p, bytes) != hipSuccess) { p.p = nullptr; return -5; }
  if (hipMemset(p.p, 0, bytes) != hipSuccess) return -4;  // zero padding in rows and k
  return 0;
}

int p4_split(const void* X, int is64, long long ldx, int rows, int cols, int trans, int conj, const P4& out,
             hipStream_t st) {
  const int R = trans ? cols : rows, C = trans ? rows : cols;
  if (R > out.rows || C > out.ld || rows <= 0 || cols <= 0) return -1;
  const int blocks = ((R + 31) / 32) * ((C + 31) / 32);
#define P4_SPLIT(T, TR, CJ) \
  hipLaunchKernelGGL((k_p4_split<T, TR, CJ>), dim3(blocks), dim3(256), 0, st, (const T*)X, ldx, rows, cols, out.p, out.ld, out.pstride)
  if (is64) {
    if (trans) { if (conj) P4_SPLIT(zd, true, true); else P4_SPLIT(zd, true, false); }
    else { if (conj) P4_SPLIT(zd, false, true); else P4_SPLIT(zd, false, false); }
  } else {
    if (trans) { if (conj) P4_SPLIT(zf, true, true); else P4_SPLIT(zf, true, false); }
    else { if (conj) P4_SPLIT(zf, false, true); else P4_SPLIT(zf, false, false); }
  }
#undef P4_SPLIT
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

int p4_join(const P4& P, int rows, int cols, int trans, zd* X, long long ldx, hipStream_t st) {
  long long tot = (long long)rows * cols;
  long long nb = (tot + 255) / 256;
  if (nb > 16384) nb = 16384;
  if (nb < 1) return 0;
  hipLaunchKernelGGL(k_p4_join, dim3((int)nb), dim3(256), 0, st, P.p, P.ld, P.pstride, rows, cols, trans, X, ldx);
  return hipGetLastError() == hipSuccess ? 0 : -4;
}

long long p4_ws_elems(int M, int N, int nsplit) { return (long long)nsplit * M * N; }

int device_cus(int dev) {
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 256;
  return cus;
}

// One workgroup per compute unit at a time (the double-buffered stages take 128 KB of LDS), so a
// grid of B workgroups runs in ceil(B / cus) rounds, each as long as the longest run of k-chunk
// steps.  Each split also writes, and the reduction reads, one more FP32 partial per tile (256 KB):
// at the few TB/s those passes reach, about a 64th of a k-chunk step's time per tile, the weight
// it gets below.  Smallest modelled time; ties go to fewer splits.
int p4_pick_split(long long tiles, int nbatch, int k_len, int cus) {
  const long long nit = (long long)nbatch * ((k_len + KS - 1) / KS);
  if (tiles < 1 || nit < 1 || cus < 1) return 1;
  long long best = -1;
  int best_s = 1;
  for (long long s = 1; s <= nit && s <= 64; ++s) {
    const long long rounds = (tiles * s + cus - 1) / cus;
    const long long steps = (nit + s - 1) / s;
    const long long cost = 64 * rounds * steps + s * tiles;
    if (best < 0 || cost < best) { best = cost; best_s = (int)s; }
  }
  return best_s;
}

int p4_gemm(const P4Desc& g0, hipStream_t st) {
  P4Desc g = g0;
  if (g.M <= 0 || g.N <= 0) return 0;
  if (g.K <= 0 || g.nbatch <= 0 || g.nsplit <= 0) return -1;
  if ((long long)g.nsplit > (long long)g.nbatch * ((g.K + KS - 1) / KS)) return -1;
  if (g.nsplit > 1 && g.out != P4OUT_WS) return -1;
  // every stage reads whole 128-row tiles and 32-wide k chunks: the planes must hold them
  const long long kpad = p4_ld(g.K);
  if (g.lda < kpad || g.ldb < kpad) return -1;
  const long long mt = (g.M + TB - 1) / TB * TB, nt = (g.N + TB - 1) / TB * TB;
  if ((g.nbatch - 1) * g.sA + (mt - 1) * g.lda + kpad > g.pA) return -1;
  if ((g.nbatch - 1) * g.sB + (nt - 1) * g.ldb + kpad > g.pB) return -1;
  if ((g.lda % 8) || (g.ldb % 8) || (g.sA % 8) || (g.sB % 8) || (g.pA % 8) || (g.pB % 8)) return -1;
  if ((((unsigned long long)g.A) & 15) || (((unsigned long long)g.B) & 15)) return -1;
  if (g.tri && g.M != g.N) return -1;
  const int tiles = g.tri ? (int)((mt / TB) * (mt / TB + 1) / 2) : (int)((mt / TB) * (nt / TB));
  const int blocks = tiles * g.nsplit;
  if (g.out == P4OUT_WS) {
    if (!g.ws) return -1;
    int rc = launch_p4_out<true, P4OUT_WS>(g, blocks, st);
    if (rc) return rc;
    const long long t32m = (g.M + 31) / 32, t32n = (g.N + 31) / 32;
    const long long nbk = g.tri ? t32n * (t32n + 1) / 2 : t32m * t32n;
    hipLaunchKernelGGL(k_p4_reduce, dim3((int)nbk), dim3(256), 0, st, (const float2*)g.ws, g.nsplit, g.M, g.N,
                       g.alpha, (zd*)g.out64, g.ldo, g.tri);
    return hipGetLastError() == hipSuccess ? 0 : -4;
  }
  if (!g.C || (g.ldc % 4) || (g.pC % 4)) return -1;
  if (g.out == P4OUT_PLANES) return launch_p4_out<true, P4OUT_PLANES>(g, blocks, st);
  if (g.out == P4OUT_PLANES_T) return launch_p4_out<false, P4OUT_PLANES_T>(g, blocks, st);
  return -1;
}

}  // namespace lindx
