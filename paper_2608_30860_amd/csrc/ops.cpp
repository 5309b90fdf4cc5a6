// Operator layer: the Lyapunov solve S^{-1} (both routes, any shift, forward and adjoint), the
// map Phi = -K S^{-1}, the Lindbladian and its adjoint, and a right-preconditioned GMRES whose
// Krylov basis, Gram-Schmidt and norms run on the device (FP64) with the small least-squares
// problem on the host.
#include <chrono>
#include <cmath>
#include <cstdlib>
#include "ctx.hpp"

namespace lindx {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// progress lines on stderr when the environment sets LINDX_LOG (to a value other than 0)
bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("LINDX_LOG");
    return v && v[0] && !(v[0] == '0' && v[1] == 0);
  }();
  return on;
}

Ctx::~Ctx() {
  for (auto& sl : pending) { hipEventDestroy(sl.a); hipEventDestroy(sl.b); }
  for (auto e : evpool) hipEventDestroy(e);
  for (void* p : allocs) hipFree(p);
  if (hsc) hipHostFree(hsc);
}

int Ctx::prof_begin(int kind) {
  // the pending slots are read back at the end of every entry point that synchronises; the cap
  // bounds the events in flight (thousands of outstanding timing events slow the runtime's own
  // synchronisation) and launches past it go untimed
  if (!prof || pending.size() >= 1024) return -1;
  ProfSlot sl;
  sl.kind = kind;
  for (hipEvent_t* e : {&sl.a, &sl.b}) {
    if (!evpool.empty()) { *e = evpool.back(); evpool.pop_back(); }
    else if (hipEventCreate(e) != hipSuccess) return -1;
  }
  hipEventRecord(sl.a, st);
  pending.push_back(sl);
  return (int)pending.size() - 1;
}
void Ctx::prof_end(int slot) {
  if (slot < 0 || slot >= (int)pending.size()) return;
  hipEventRecord(pending[slot].b, st);
}
int Ctx::prof_collect() {
  if (pending.empty()) return 0;
  if (hipStreamSynchronize(st) != hipSuccess) return LIND_EDEVICE;
  for (auto& sl : pending) {
    float ms = 0;
    if (hipEventElapsedTime(&ms, sl.a, sl.b) == hipSuccess && sl.kind >= 0 && sl.kind < 8) {
      prof_ms[sl.kind] += ms;
      prof_cnt[sl.kind] += 1;
    }
    evpool.push_back(sl.a);
    evpool.push_back(sl.b);
  }
  pending.clear();
  return 0;
}

int Ctx::sync() { return hipStreamSynchronize(st) == hipSuccess ? 0 : LIND_EDEVICE; }

int Ctx::fetch(const void* dptr, size_t bytes) {
  if (hipMemcpyAsync(hsc, dptr, bytes, hipMemcpyDeviceToHost, st) != hipSuccess) return LIND_EDEVICE;
  return sync();
}

int Ctx::ensure_krylov(int which, int slots) {
  zd** p = which == 1 ? &K1 : &K2;
  int* cap = which == 1 ? &K1cap : &K2cap;
  if (*cap >= slots) return 0;
  if (*p) {
    for (auto it = allocs.begin(); it != allocs.end(); ++it)
      if (*it == (void*)*p) { allocs.erase(it); break; }
    hipFree(*p);
    *p = nullptr;
    *cap = 0;
  }
  if (alloc(p, (size_t)slots * n2)) return LIND_ENOMEM;
  *cap = slots;
  return 0;
}

int op_gemm(Ctx& c, int prec, int M, int N, int K, const void* A, long long lda, int opA, const void* B,
            long long ldb, int opB, void* C, long long ldc, cplx alpha, int beta) {
  GemmDesc g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.lda = lda; g.opA = opA;
  g.B = B; g.ldb = ldb; g.opB = opB;
  g.C = C; g.ldc = ldc;
  g.ar = alpha.real(); g.ai = alpha.imag();
  g.beta = beta;
  g.ws = c.gws; g.ws_bytes = c.gws_bytes;  // split-K room for small products
  return gemm(prec, g, c.st) ? LIND_EDEVICE : 0;
}

#define TRY(x)                       \
  do {                               \
    int rc__ = (x);                  \
    if (rc__) return rc__ < 0 ? rc__ : LIND_EDEVICE; \
  } while (0)

// C (complex128, n x n) = A op(B) with complex64 operands in the working precision
static int basis_to64(Ctx& c, int prec, const zf* A, int opA, const zf* B, int opB, zd* C) {
  GemmDesc g;
  g.M = c.n; g.N = c.n; g.K = c.n;
  g.A = A; g.lda = c.n; g.opA = opA;
  g.B = B; g.ldb = c.n; g.opB = opB;
  g.C = C; g.ldc = c.n; g.out64 = 1;
  return gemm(prec, g, c.st) ? LIND_EDEVICE : 0;
}

// ---------------------------------------------------------------------------------------------
// (S - mu)^{-1}.  Eigenbasis route (eq. lyapu_eig_solution):
//   X = U [ (V^H Y V)_ij / (s_i + conj(s_j) - mu) ] U^H            (V = U^{-H})
// adjoint (S* - conj(mu))^{-1}, S*(X) = G^H X + X G:
//   X = V [ (U^H Y U)_ij / (conj(s_i) + s_j - conj(mu)) ] V^H
// Schur route (Bartels-Stewart, Section A.1): X = Z Xt Z^H with T Xt + Xt T^H - mu Xt = Z^H Y Z;
// adjoint through the flipped factor J T^H J.
// ---------------------------------------------------------------------------------------------
int op_sinv(Ctx& c, const zd* Y, zd* X, cplx mu, int prec, bool adjoint) {
  const int n = c.n;
  const long long n2 = c.n2;
  const cplx one(1, 0);
  if (c.route == LIND_ROUTE_EIG) {
    if (prec == PREC_F64) {
      const zd* P = adjoint ? c.U : c.V;  // inner basis
      const zd* Q = adjoint ? c.V : c.U;  // outer basis
      TRY(op_gemm(c, PREC_F64, n, n, n, P, n, OP_C, Y, n, OP_N, c.w1, n, one, 0));
      GemmDesc g;
      g.M = n; g.N = n; g.K = n;
      g.A = c.w1; g.lda = n; g.opA = OP_N;
      g.B = P; g.ldb = n; g.opB = OP_N;
      g.C = c.w2; g.ldc = n;
      g.epi = EPI_DIV;
      g.dr = adjoint ? c.sbar : c.s;
      g.dc = adjoint ? c.s : c.sbar;
      cplx m = adjoint ? std::conj(mu) : mu;
      g.dzr = -m.real(); g.dzi = -m.imag();
      g.ws = c.gws; g.ws_bytes = c.gws_bytes;  // split-K room for small systems
      TRY(gemm(PREC_F64, g, c.st));
      TRY(op_gemm(c, PREC_F64, n, n, n, Q, n, OP_N, c.w2, n, OP_N, c.w1, n, one, 0));
      TRY(op_gemm(c, PREC_F64, n, n, n, c.w1, n, OP_N, Q, n, OP_C, X, n, one, 0));
      return 0;
    }
    const zf* P = adjoint ? c.U32 : c.V32;
    const zf* Q = adjoint ? c.V32 : c.U32;
    TRY(to_c64(Y, c.a32, n2, c.st));
    TRY(op_gemm(c, prec, n, n, n, P, n, OP_C, c.a32, n, OP_N, c.b32, n, one, 0));
    GemmDesc g;
    g.M = n; g.N = n; g.K = n;
    g.A = c.b32; g.lda = n; g.opA = OP_N;
    g.B = P; g.ldb = n; g.opB = OP_N;
    g.C = c.a32; g.ldc = n;
    g.epi = EPI_DIV;
    g.dr = adjoint ? c.sbar : c.s;
    g.dc = adjoint ? c.s : c.sbar;
    cplx m = adjoint ? std::conj(mu) : mu;
    g.dzr = -m.real(); g.dzi = -m.imag();
    g.ws = c.gws; g.ws_bytes = c.gws_bytes;  // split-K room for small systems
    TRY(gemm(prec, g, c.st));
    TRY(op_gemm(c, prec, n, n, n, Q, n, OP_N, c.a32, n, OP_N, c.b32, n, one, 0));
    GemmDesc h;
    h.M = n; h.N = n; h.K = n;
    h.A = c.b32; h.lda = n; h.opA = OP_N;
    h.B = Q; h.ldb = n; h.opB = OP_C;
    h.C = X; h.ldc = n; h.out64 = 1;
    TRY(gemm(prec, h, c.st));
    return 0;
  }
  // Schur route: the triangular solve always in FP64; the basis changes in the working precision
  // (FP64, or FP32 / BF16x3 products of the FP32 copy of Z with FP32 accumulation)
  const bool lowp = prec != PREC_F64 && c.Z32;
  if (lowp) {
    TRY(to_c64(Y, c.a32, n2, c.st));
    TRY(op_gemm(c, prec, n, n, n, c.Z32, n, OP_C, c.a32, n, OP_N, c.b32, n, one, 0));
    TRY(basis_to64(c, prec, c.b32, OP_N, c.Z32, OP_N, c.w2));
  } else {
    TRY(op_gemm(c, PREC_F64, n, n, n, c.Z, n, OP_C, Y, n, OP_N, c.w1, n, one, 0));
    TRY(op_gemm(c, PREC_F64, n, n, n, c.w1, n, OP_N, c.Z, n, OP_N, c.w2, n, one, 0));
  }
  if (!adjoint) {
    TRY(trisylv(c.T, c.w2, n, zmk(-mu.real(), -mu.imag()), c.tsws, c.st, lowp ? &c.tsb : nullptr));
  } else {
    // T^H Xt + Xt T - conj(mu) Xt = Yt  <=>  T' X' + X' T'^H - conj(mu) X' = Y'  with
    // T' = J T^H J (upper triangular, precomputed), X' = J Xt J, Y' = J Yt J (J = exchange)
    TRY(flip_rev(c.w2, c.w1, n, c.st));
    TRY(trisylv(c.Tadj, c.w1, n, zmk(-mu.real(), mu.imag()), c.tsws, c.st, lowp ? &c.tsb_adj : nullptr));
    TRY(flip_rev(c.w1, c.w2, n, c.st));
  }
  if (lowp) {
    TRY(to_c64(c.w2, c.a32, n2, c.st));
    TRY(op_gemm(c, prec, n, n, n, c.Z32, n, OP_N, c.a32, n, OP_N, c.b32, n, one, 0));
    TRY(basis_to64(c, prec, c.b32, OP_N, c.Z32, OP_C, X));
    return 0;
  }
  TRY(op_gemm(c, PREC_F64, n, n, n, c.Z, n, OP_N, c.w2, n, OP_N, c.w1, n, one, 0));
  TRY(op_gemm(c, PREC_F64, n, n, n, c.w1, n, OP_N, c.Z, n, OP_C, X, n, one, 0));
  return 0;
}

// ---------------------------------------------------------------------------------------------
// Phi(xi) = -K(S^{-1} xi) = -sum_j Lt_j Xh Lt_j^H with Xh the solution in the factor basis and
// Lt_j = L_j U (eigen route) or L_j Z (Schur route): 2 basis-change products + the stacked jump
// product [Lt_1; ..; Lt_d] Xh (one launch, M = d n) + the reduction product sum_j Y_j Lt_j^H
// (one launch, K loop over (j, k)).
// ---------------------------------------------------------------------------------------------
int op_phi(Ctx& c, const zd* xi, zd* out, int prec, bool hermitian) {
  const int n = c.n, d = c.d;
  const long long n2 = c.n2;
  const cplx one(1, 0), mone(-1, 0);
  if (d == 0) return fill_zero(out, n2 * (long long)sizeof(zd), c.st) ? LIND_EDEVICE : 0;
  if (c.route == LIND_ROUTE_SCHUR && prec == PREC_BF16X3 && c.p4_ready) {
    // pre-split BF16 products around the FP64 triangular solve: C1 = Z^H xi (planes), W = C1 Z
    // (complex128 through the split-K path), T Xh + Xh T^H = W, Xh^T into planes, then the jump
    // products of the eigen route with Lt_j = L_j Z
    const int sp = c.prof_begin(PROF_PHI);
    int s0 = c.prof_begin(PROF_BASIS_IN);
    TRY(p4_split(xi, 1, n, n, n, 1, 0, c.p4_xiT, c.st));
    P4Desc g;
    g.M = n; g.N = n; g.K = n;
    g.A = c.p4_VH.p; g.lda = c.p4_VH.ld; g.pA = c.p4_VH.pstride;
    g.B = c.p4_xiT.p; g.ldb = c.p4_xiT.ld; g.pB = c.p4_xiT.pstride;
    g.out = P4OUT_PLANES; g.C = c.p4_C1.p; g.ldc = c.p4_C1.ld; g.pC = c.p4_C1.pstride;
    TRY(p4_gemm(g, c.st));
    P4Desc h;
    h.M = n; h.N = n; h.K = n;
    h.A = c.p4_C1.p; h.lda = c.p4_C1.ld; h.pA = c.p4_C1.pstride;
    h.B = c.p4_VT.p; h.ldb = c.p4_VT.ld; h.pB = c.p4_VT.pstride;
    h.tri = hermitian;  // Hermitian xi: Z^H xi Z is Hermitian
    const long long tm = (n + 127) / 128;
    h.nsplit = std::min(c.p4_nsplit, p4_pick_split(hermitian ? tm * (tm + 1) / 2 : tm * tm, 1, n, device_cus(c.dev)));
    h.out = P4OUT_WS; h.ws = c.p4_ws; h.out64 = c.w2; h.ldo = n; h.alpha = 1.0;
    TRY(p4_gemm(h, c.st));
    c.prof_end(s0);
    TRY(trisylv(c.T, c.w2, n, zmk(0, 0), c.tsws, c.st, &c.tsb));
    TRY(p4_split(c.w2, 1, n, n, n, 1, 0, c.p4_XhT, c.st));
    int s1 = c.prof_begin(PROF_JUMP_STACK);
    P4Desc y;
    y.M = d * n; y.N = n; y.K = n;
    y.A = c.p4_Lt.p; y.lda = c.p4_Lt.ld; y.pA = c.p4_Lt.pstride;
    y.B = c.p4_XhT.p; y.ldb = c.p4_XhT.ld; y.pB = c.p4_XhT.pstride;
    y.out = P4OUT_PLANES; y.C = c.p4_Y.p; y.ldc = c.p4_Y.ld; y.pC = c.p4_Y.pstride;
    TRY(p4_gemm(y, c.st));
    c.prof_end(s1);
    P4Desc r;
    r.M = n; r.N = n; r.K = n; r.nbatch = d; r.nsplit = c.p4_nsplit;
    r.A = c.p4_Y.p; r.lda = c.p4_Y.ld; r.pA = c.p4_Y.pstride; r.sA = (long long)n * c.p4_Y.ld;
    r.B = c.p4_Lt.p; r.ldb = c.p4_Lt.ld; r.pB = c.p4_Lt.pstride; r.sB = (long long)n * c.p4_Lt.ld;
    r.conjB = 1;
    r.out = P4OUT_WS; r.ws = c.p4_ws; r.out64 = out; r.ldo = n; r.alpha = -1.0;
    r.tri = hermitian;
    int s2 = c.prof_begin(PROF_JUMP_REDUCE);
    TRY(p4_gemm(r, c.st));
    c.prof_end(s2);
    c.prof_end(sp);
    return 0;
  }
  if (c.route == LIND_ROUTE_SCHUR) {
    // FP64 triangular solve between basis changes and jump products in the working precision
    const bool lowp = prec != PREC_F64 && c.Z32;
    if (lowp) {
      TRY(to_c64(xi, c.a32, n2, c.st));
      TRY(op_gemm(c, prec, n, n, n, c.Z32, n, OP_C, c.a32, n, OP_N, c.b32, n, one, 0));
      TRY(basis_to64(c, prec, c.b32, OP_N, c.Z32, OP_N, c.w2));
    } else {
      TRY(op_gemm(c, PREC_F64, n, n, n, c.Z, n, OP_C, xi, n, OP_N, c.w1, n, one, 0));
      TRY(op_gemm(c, PREC_F64, n, n, n, c.w1, n, OP_N, c.Z, n, OP_N, c.w2, n, one, 0));
    }
    TRY(trisylv(c.T, c.w2, n, zmk(0, 0), c.tsws, c.st, lowp ? &c.tsb : nullptr));
    if (prec == PREC_F64) {
      TRY(op_gemm(c, PREC_F64, d * n, n, n, c.Lt, n, OP_N, c.w2, n, OP_N, c.Ys, n, one, 0));
      GemmDesc g;
      g.M = n; g.N = n; g.K = n; g.nbatch = d; g.ws = c.gws; g.ws_bytes = c.gws_bytes;
      g.A = c.Ys; g.lda = n; g.sA = n2; g.opA = OP_N;
      g.B = c.Lt; g.ldb = n; g.sB = n2; g.opB = OP_C;
      g.C = out; g.ldc = n; g.ar = -1.0;
      TRY(gemm(PREC_F64, g, c.st));
      return 0;
    }
    TRY(to_c64(c.w2, c.a32, n2, c.st));
    TRY(op_gemm(c, prec, d * n, n, n, c.Lt32, n, OP_N, c.a32, n, OP_N, c.Y32, n, one, 0));
    GemmDesc g;
    g.M = n; g.N = n; g.K = n; g.nbatch = d; g.ws = c.gws; g.ws_bytes = c.gws_bytes;
    g.A = c.Y32; g.lda = n; g.sA = n2; g.opA = OP_N;
    g.B = c.Lt32; g.ldb = n; g.sB = n2; g.opB = OP_C;
    g.C = out; g.ldc = n; g.ar = -1.0; g.out64 = 1;
    TRY(gemm(prec, g, c.st));
    return 0;
  }
  const int sp = c.prof_begin(PROF_PHI);
  if (prec == PREC_F64 && n <= 32) {
    // small system: one workgroup instead of the chain of product launches
    TRY(phi_small(xi, c.V, c.Lt, c.s, c.sbar, n, d, out, c.st));
    c.prof_end(sp);
    return 0;
  }
  if (prec == PREC_F64) {
    int s0 = c.prof_begin(PROF_BASIS_IN);
    TRY(op_gemm(c, PREC_F64, n, n, n, c.V, n, OP_C, xi, n, OP_N, c.w1, n, one, 0));
    GemmDesc g;
    g.M = n; g.N = n; g.K = n;
    g.A = c.w1; g.lda = n; g.opA = OP_N;
    g.B = c.V; g.ldb = n; g.opB = OP_N;
    g.C = c.w2; g.ldc = n;
    g.epi = EPI_DIV; g.dr = c.s; g.dc = c.sbar;
    g.tri = hermitian;  // Hermitian xi: Xh = (V^H xi V) / (s_i + conj s_j) is Hermitian
    g.ws = c.gws; g.ws_bytes = c.gws_bytes;  // split-K room for small systems
    TRY(gemm(PREC_F64, g, c.st));
    c.prof_end(s0);
    int s1 = c.prof_begin(PROF_JUMP_STACK);
    TRY(op_gemm(c, PREC_F64, d * n, n, n, c.Lt, n, OP_N, c.w2, n, OP_N, c.Ys, n, one, 0));
    c.prof_end(s1);
    GemmDesc h;
    h.M = n; h.N = n; h.K = n; h.nbatch = d; h.ws = c.gws; h.ws_bytes = c.gws_bytes;
    h.A = c.Ys; h.lda = n; h.sA = n2; h.opA = OP_N;
    h.B = c.Lt; h.ldb = n; h.sB = n2; h.opB = OP_C;
    h.C = out; h.ldc = n; h.ar = -1.0;
    h.tri = hermitian;
    int s2 = c.prof_begin(PROF_JUMP_REDUCE);
    TRY(gemm(PREC_F64, h, c.st));
    c.prof_end(s2);
    c.prof_end(sp);
    (void)mone;
    return 0;
  }
  if (prec == PREC_BF16X3 && c.p4_ready) {
    // pre-split BF16 products: xi^T planes, C1 = V^H xi, Xh^T = ((C1 V) / (s_i + conj s_j))^T,
    // Y = [Lt_1; ..; Lt_d] Xh, Phi = -sum_j Y_j Lt_j^H (split-K partials, complex128 result)
    int s0 = c.prof_begin(PROF_BASIS_IN);
    TRY(p4_split(xi, 1, n, n, n, 1, 0, c.p4_xiT, c.st));
    P4Desc g;
    g.M = n; g.N = n; g.K = n;
    g.A = c.p4_VH.p; g.lda = c.p4_VH.ld; g.pA = c.p4_VH.pstride;
    g.B = c.p4_xiT.p; g.ldb = c.p4_xiT.ld; g.pB = c.p4_xiT.pstride;
    g.out = P4OUT_PLANES; g.C = c.p4_C1.p; g.ldc = c.p4_C1.ld; g.pC = c.p4_C1.pstride;
    TRY(p4_gemm(g, c.st));
    P4Desc h;
    h.M = n; h.N = n; h.K = n;
    h.A = c.p4_C1.p; h.lda = c.p4_C1.ld; h.pA = c.p4_C1.pstride;
    h.B = c.p4_VT.p; h.ldb = c.p4_VT.ld; h.pB = c.p4_VT.pstride;
    h.dr = c.s; h.dc = c.sbar;
    h.out = P4OUT_PLANES_T; h.C = c.p4_XhT.p; h.ldc = c.p4_XhT.ld; h.pC = c.p4_XhT.pstride;
    h.tri = hermitian;  // Hermitian xi: V^H xi V and the divisors are Hermitian, so is Xh
    TRY(p4_gemm(h, c.st));
    c.prof_end(s0);
    int s1 = c.prof_begin(PROF_JUMP_STACK);
    P4Desc y;
    y.M = d * n; y.N = n; y.K = n;
    y.A = c.p4_Lt.p; y.lda = c.p4_Lt.ld; y.pA = c.p4_Lt.pstride;
    y.B = c.p4_XhT.p; y.ldb = c.p4_XhT.ld; y.pB = c.p4_XhT.pstride;
    y.out = P4OUT_PLANES; y.C = c.p4_Y.p; y.ldc = c.p4_Y.ld; y.pC = c.p4_Y.pstride;
    TRY(p4_gemm(y, c.st));
    c.prof_end(s1);
    P4Desc r;
    r.M = n; r.N = n; r.K = n; r.nbatch = d; r.nsplit = c.p4_nsplit;
    r.A = c.p4_Y.p; r.lda = c.p4_Y.ld; r.pA = c.p4_Y.pstride; r.sA = (long long)n * c.p4_Y.ld;
    r.B = c.p4_Lt.p; r.ldb = c.p4_Lt.ld; r.pB = c.p4_Lt.pstride; r.sB = (long long)n * c.p4_Lt.ld;
    r.conjB = 1;
    r.out = P4OUT_WS; r.ws = c.p4_ws; r.out64 = out; r.ldo = n; r.alpha = -1.0;
    r.tri = hermitian;  // sum_j L_j X L_j^+ of a Hermitian X
    int s2 = c.prof_begin(PROF_JUMP_REDUCE);
    TRY(p4_gemm(r, c.st));
    c.prof_end(s2);
    c.prof_end(sp);
    return 0;
  }
  int s0 = c.prof_begin(PROF_BASIS_IN);
  TRY(to_c64(xi, c.a32, n2, c.st));
  TRY(op_gemm(c, prec, n, n, n, c.V32, n, OP_C, c.a32, n, OP_N, c.b32, n, one, 0));
  GemmDesc g;
  g.M = n; g.N = n; g.K = n;
  g.A = c.b32; g.lda = n; g.opA = OP_N;
  g.B = c.V32; g.ldb = n; g.opB = OP_N;
  g.C = c.a32; g.ldc = n;
  g.epi = EPI_DIV; g.dr = c.s; g.dc = c.sbar;
  g.ws = c.gws; g.ws_bytes = c.gws_bytes;  // split-K room for small systems
  TRY(gemm(prec, g, c.st));
  c.prof_end(s0);
  int s1 = c.prof_begin(PROF_JUMP_STACK);
  TRY(op_gemm(c, prec, d * n, n, n, c.Lt32, n, OP_N, c.a32, n, OP_N, c.Y32, n, one, 0));
  c.prof_end(s1);
  GemmDesc h;
  h.M = n; h.N = n; h.K = n; h.nbatch = d; h.ws = c.gws; h.ws_bytes = c.gws_bytes;
  h.A = c.Y32; h.lda = n; h.sA = n2; h.opA = OP_N;
  h.B = c.Lt32; h.ldb = n; h.sB = n2; h.opB = OP_C;
  h.C = out; h.ldc = n; h.ar = -1.0; h.out64 = 1;
  int s2 = c.prof_begin(PROF_JUMP_REDUCE);
  TRY(gemm(prec, h, c.st));
  c.prof_end(s2);
  c.prof_end(sp);
  return 0;
}

// ---------------------------------------------------------------------------------------------
// L(rho) = G rho + rho G^H + sum_j L_j rho L_j^H (eq. lindblad_decomposition), FP64.
// Hermitian rho: P = G rho, out = sum_j (L_j rho) L_j^H + P + P^H (fused epilogue).
// ---------------------------------------------------------------------------------------------
int op_apply(Ctx& c, const zd* rho, zd* out, bool hermitian_in) {
  const int n = c.n, d = c.d;
  const long long n2 = c.n2;
  const cplx one(1, 0);
  if (hermitian_in && d > 0) {
    TRY(op_gemm(c, PREC_F64, n, n, n, c.G, n, OP_N, rho, n, OP_N, c.w4, n, one, 0));
    TRY(op_gemm(c, PREC_F64, d * n, n, n, c.L, n, OP_N, rho, n, OP_N, c.Ys, n, one, 0));
    GemmDesc g;
    g.M = n; g.N = n; g.K = n; g.nbatch = d; g.ws = c.gws; g.ws_bytes = c.gws_bytes;
    g.A = c.Ys; g.lda = n; g.sA = n2; g.opA = OP_N;
    g.B = c.L; g.ldb = n; g.sB = n2; g.opB = OP_C;
    g.C = out; g.ldc = n;
    g.epi = EPI_HERM_ADD; g.E = c.w4; g.lde = n;
    g.tri = 1;  // the result is Hermitian: tiles on and above the diagonal only
    TRY(gemm(PREC_F64, g, c.st));
    return 0;
  }
  TRY(op_gemm(c, PREC_F64, n, n, n, c.G, n, OP_N, rho, n, OP_N, out, n, one, 0));
  TRY(op_gemm(c, PREC_F64, n, n, n, rho, n, OP_N, c.G, n, OP_C, out, n, one, 1));
  if (d > 0) {
    TRY(op_gemm(c, PREC_F64, d * n, n, n, c.L, n, OP_N, rho, n, OP_N, c.Ys, n, one, 0));
    GemmDesc g;
    g.M = n; g.N = n; g.K = n; g.nbatch = d; g.ws = c.gws; g.ws_bytes = c.gws_bytes;
    g.A = c.Ys; g.lda = n; g.sA = n2; g.opA = OP_N;
    g.B = c.L; g.ldb = n; g.sB = n2; g.opB = OP_C;
    g.C = out; g.ldc = n; g.beta = 1;
    TRY(gemm(PREC_F64, g, c.st));
  }
  return 0;
}

// BF16x3 Lindbladian.  One stacked product Y = [L_1; ..; L_d] X (planes out), then one batched
// reduction over d + 2 pairs with split-K partials:
//   sum_{j<d} Y_j L_j^H  +  G (conj(X^T))^H  +  X G^H  =  L(X)   (eq. lindblad_decomposition)
// The constant planes (L_j, G in both operand arrays) are split once; X is split three ways per call.
static P4 p4_rows_view(const P4& P, long long row0) {
  P4 v = P;
  v.p = P.p + row0 * P.ld;
  v.rows = P.rows - row0;
  return v;
}
static int setup_p4L(Ctx& c) {
  const int n = c.n, d = c.d;
  const long long rows = (long long)(d + 2) * n;
  for (P4* b : {&c.p4L_A, &c.p4L_B}) {
    if (p4_alloc(*b, rows, n)) return c.fail(LIND_ENOMEM, "out of device memory (bf16 Lindbladian planes)");
    c.allocs.push_back(b->p);
  }
  if (p4_alloc(c.p4L_xT, n, n)) return c.fail(LIND_ENOMEM, "out of device memory (bf16 Lindbladian planes)");
  c.allocs.push_back(c.p4L_xT.p);
  // the Lindbladian is the same for every gauge: the (possibly shifted) pair the context holds
  for (int j = 0; j < d; ++j)
    if (p4_split(c.L + (long long)j * c.n2, 1, n, n, n, 0, 0, p4_rows_view(c.p4L_B, (long long)j * n), c.st))
      return LIND_EDEVICE;
  if (p4_split(c.G, 1, n, n, n, 0, 0, p4_rows_view(c.p4L_B, (long long)(d + 1) * n), c.st)) return LIND_EDEVICE;
  if (p4_split(c.G, 1, n, n, n, 0, 0, p4_rows_view(c.p4L_A, (long long)d * n), c.st)) return LIND_EDEVICE;
  // split-K over the d + 2 products summed, in runs that fill whole rounds of the chip
  const long long tm = (n + 127) / 128;
  const int s = p4_pick_split(tm * tm, d + 2, n, device_cus(c.dev));
  c.p4L_nsplit = s;
  if (c.alloc(&c.p4L_ws, (size_t)s * c.n2)) return c.fail(LIND_ENOMEM, "out of device memory (split-K)");
  c.p4L_ready = true;
  return 0;
}

int op_apply_p4(Ctx& c, const zd* X, zd* out) {
  const int n = c.n, d = c.d;
  if (c.route != LIND_ROUTE_EIG || d < 1) return LIND_EINVAL;
  if (!c.p4L_ready) TRY(setup_p4L(c));
  TRY(p4_split(X, 1, n, n, n, 0, 0, p4_rows_view(c.p4L_A, (long long)(d + 1) * n), c.st));  // X
  TRY(p4_split(X, 1, n, n, n, 1, 1, p4_rows_view(c.p4L_B, (long long)d * n), c.st));        // conj(X^T)
  TRY(p4_split(X, 1, n, n, n, 1, 0, c.p4L_xT, c.st));                                        // X^T
  P4Desc y;
  y.M = d * n; y.N = n; y.K = n;
  y.A = c.p4L_B.p; y.lda = c.p4L_B.ld; y.pA = c.p4L_B.pstride;
  y.B = c.p4L_xT.p; y.ldb = c.p4L_xT.ld; y.pB = c.p4L_xT.pstride;
  y.out = P4OUT_PLANES; y.C = c.p4L_A.p; y.ldc = c.p4L_A.ld; y.pC = c.p4L_A.pstride;
  TRY(p4_gemm(y, c.st));
  P4Desc r;
  r.M = n; r.N = n; r.K = n; r.nbatch = d + 2; r.nsplit = c.p4L_nsplit;
  r.A = c.p4L_A.p; r.lda = c.p4L_A.ld; r.pA = c.p4L_A.pstride; r.sA = (long long)n * c.p4L_A.ld;
  r.B = c.p4L_B.p; r.ldb = c.p4L_B.ld; r.pB = c.p4L_B.pstride; r.sB = (long long)n * c.p4L_B.ld;
  r.conjB = 1;
  r.out = P4OUT_WS; r.ws = c.p4L_ws; r.out64 = out; r.ldo = n; r.alpha = 1.0;
  TRY(p4_gemm(r, c.st));
  return 0;
}

// L*(X) = G^H X + X G + sum_j L_j^H X L_j
int op_apply_adj(Ctx& c, const zd* X, zd* out) {
  const int n = c.n, d = c.d;
  const long long n2 = c.n2;
  const cplx one(1, 0);
  TRY(op_gemm(c, PREC_F64, n, n, n, c.G, n, OP_C, X, n, OP_N, out, n, one, 0));
  TRY(op_gemm(c, PREC_F64, n, n, n, X, n, OP_N, c.G, n, OP_N, out, n, one, 1));
  for (int j = 0; j < d; ++j)
    TRY(op_gemm(c, PREC_F64, n, n, n, c.L + j * n2, n, OP_C, X, n, OP_N, c.Ys + j * n2, n, one, 0));
  if (d > 0) {
    GemmDesc g;
    g.M = n; g.N = n; g.K = n; g.nbatch = d; g.ws = c.gws; g.ws_bytes = c.gws_bytes;
    g.A = c.Ys; g.lda = n; g.sA = n2; g.opA = OP_N;
    g.B = c.L; g.ldb = n; g.sB = n2; g.opB = OP_N;
    g.C = out; g.ldc = n; g.beta = 1;
    TRY(gemm(PREC_F64, g, c.st));
  }
  return 0;
}

int op_norms(Ctx& c, const zd* X, double out[4]) {
  TRY(mat_norms(X, c.n, (double*)c.dsc, c.dscr, c.st));
  TRY(c.fetch(c.dsc, 4 * sizeof(double)));
  const double* h = (const double*)c.hsc;
  for (int i = 0; i < 4; ++i) out[i] = h[i];
  return 0;
}
int op_trace(Ctx& c, const zd* X, cplx* tr) {
  TRY(trace(X, c.n, c.dsc, c.dscr, c.st));
  TRY(c.fetch(c.dsc, sizeof(zd)));
  *tr = cplx(c.hsc[0].x, c.hsc[0].y);
  return 0;
}
int op_nrm(Ctx& c, const zd* x, double* out) {
  TRY(nrm2(x, c.n2, (double*)c.dsc, c.dscr, c.st));
  TRY(c.fetch(c.dsc, sizeof(double)));
  *out = ((const double*)c.hsc)[0];
  return 0;
}

// ---------------------------------------------------------------------------------------------
// Right-preconditioned restarted GMRES(m): solve A x = b with x = x0 + P(V y).  Classical
// Gram-Schmidt with one full re-orthogonalisation pass (CGS2) on the device; Givens QR of the
// (m+1) x m Hessenberg on the host.  Each restart recomputes the true residual b - A x.
// ---------------------------------------------------------------------------------------------
int gmres(Ctx& c, const std::function<int(const zd*, zd*)>& A, const std::function<int(const zd*, zd*)>* P,
          const zd* b, zd* x, bool x_zero, int m, int max_cycles, double rtol, double atol, GmresResult& res,
          double t_deadline) {
  const long long n2 = c.n2;
  if (m < 1) m = 1;
  if (m > 64) m = 64;
  TRY(c.ensure_krylov(2, m + 2));
  zd* Vb = c.K2;
  zd* r = Vb;  // slot 0 holds the residual / first basis vector
  zd* tmp = Vb + (long long)(m + 1) * n2;  // scratch slot
  double bnorm = 0;
  TRY(op_nrm(c, b, &bnorm));
  if (x_zero) TRY(fill_zero(x, n2 * (long long)sizeof(zd), c.st));
  res = GmresResult();
  std::vector<cplx> Hh((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1);
  bool first = true;
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    // r = b - A x
    if (first && x_zero) {
      TRY(copy(b, r, n2, c.st));
    } else {
      TRY(A(x, tmp));
      TRY(copy(b, r, n2, c.st));
      TRY(axpby(zmk(-1, 0), tmp, zmk(1, 0), r, n2, c.st));
    }
    double beta = 0;
    TRY(op_nrm(c, r, &beta));
    if (first) res.resid0 = beta;
    first = false;
    res.resid = beta;
    double target = std::max(rtol * bnorm, atol);
    if (beta <= target || beta == 0.0) { res.converged = true; break; }
    if (t_deadline > 0 && now_s() > t_deadline) break;
    TRY(scale_by_inv(r, n2, (const double*)c.dsc, c.st));  // dsc[0] holds beta
    std::fill(g.begin(), g.end(), cplx(0));
    g[0] = beta;
    int k = 0;
    double est = beta;
    for (int j = 0; j < m; ++j) {
      zd* vj = Vb + (long long)j * n2;
      zd* w = Vb + (long long)(j + 1) * n2;
      if (P) {
        TRY((*P)(vj, tmp));
        TRY(A(tmp, w));
      } else {
        TRY(A(vj, w));
      }
      zd* hdev = c.dsc + 8;
      zd* h2dev = c.dsc + 8 + 72;
      TRY(multi_dot(Vb, n2, j + 1, w, n2, hdev, (zd*)c.dscr, c.st));
      TRY(multi_axpy(Vb, n2, j + 1, hdev, w, n2, 1, -1.0, c.st));
      TRY(multi_dot(Vb, n2, j + 1, w, n2, h2dev, (zd*)c.dscr, c.st));
      TRY(multi_axpy(Vb, n2, j + 1, h2dev, w, n2, 1, -1.0, c.st));
      TRY(nrm2(w, n2, (double*)(c.dsc + 4), c.dscr, c.st));
      TRY(c.fetch(c.dsc, sizeof(zd) * (8 + 72 + 72)));
      double hn = ((const double*)(c.hsc + 4))[0];
      for (int i = 0; i <= j; ++i) {
        cplx h1(c.hsc[8 + i].x, c.hsc[8 + i].y), h2(c.hsc[80 + i].x, c.hsc[80 + i].y);
        Hh[(size_t)i * m + j] = h1 + h2;
      }
      Hh[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0) TRY(scale_by_inv(w, n2, (const double*)(c.dsc + 4), c.st));
      // apply previous rotations
      for (int i = 0; i < j; ++i) {
        cplx a = Hh[(size_t)i * m + j], bb = Hh[(size_t)(i + 1) * m + j];
        Hh[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
        Hh[(size_t)(i + 1) * m + j] = -std::conj(sn[i]) * a + cs[i] * bb;
      }
      cplx f = Hh[(size_t)j * m + j], gg = Hh[(size_t)(j + 1) * m + j];
      double af = std::abs(f), ag = std::abs(gg);
      if (ag == 0) { cs[j] = 1; sn[j] = 0; }
      else if (af == 0) { cs[j] = 0; sn[j] = std::conj(gg) / ag; }
      else {
        double nr = std::hypot(af, ag);
        cplx ph = f / af;
        cs[j] = af / nr;
        sn[j] = ph * std::conj(gg) / nr;
      }
      Hh[(size_t)j * m + j] = cs[j] * f + sn[j] * gg;
      Hh[(size_t)(j + 1) * m + j] = 0;
      cplx gj = g[j];
      g[j] = cs[j] * gj;
      g[j + 1] = -std::conj(sn[j]) * gj;
      k = j + 1;
      est = std::abs(g[j + 1]);
      ++res.iters;
      if (est <= target || hn == 0.0) break;
      if (t_deadline > 0 && now_s() > t_deadline) break;
    }
    // back substitution R y = g
    std::vector<cplx> y(k);
    for (int i = k - 1; i >= 0; --i) {
      cplx acc = g[i];
      for (int l = i + 1; l < k; ++l) acc -= Hh[(size_t)i * m + l] * y[l];
      y[i] = acc / Hh[(size_t)i * m + i];
    }
    for (int i = 0; i < k; ++i) c.hsc[i] = zmk(y[i].real(), y[i].imag());
    zd* ydev = c.dsc + 160;
    if (hipMemcpyAsync(ydev, c.hsc, sizeof(zd) * k, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
    TRY(c.sync());  // the pinned buffer is reused right after
    zd* z = Vb + (long long)(m + 1) * n2;  // tmp slot
    TRY(multi_axpy(Vb, n2, k, ydev, z, n2, 0, 1.0, c.st));
    if (P) {
      // x += P(z): P writes into slot 1 (no longer needed)
      zd* pz = Vb + n2;
      TRY((*P)(z, pz));
      TRY(axpby(zmk(1, 0), pz, zmk(1, 0), x, n2, c.st));
    } else {
      TRY(axpby(zmk(1, 0), z, zmk(1, 0), x, n2, c.st));
    }
    res.cycles = cyc + 1;
    res.resid = est;
    if (est <= target) {
      res.converged = true;
      // one final true-residual check is left to the caller
      break;
    }
  }
  return 0;
}

}  // namespace lindx
