// Internal definition of the lindx context and the operator layer shared by the drivers.
#pragma once
#include <functional>
#include <string>
#include <vector>
#include <complex>
#include "kernels.hpp"
#include "../../include/lind.h"

namespace lindx {

typedef std::complex<double> cplx;

// profiled kernel kinds
enum { PROF_JUMP_STACK = 0, PROF_JUMP_REDUCE = 1, PROF_BASIS_IN = 2, PROF_PHI = 3, PROF_RESID = 4, PROF_CGS = 5 };

struct Ctx;
constexpr int kMaxLong = 6144;
// Largest condition number (infinity norm) of a diagonal block's eigenvector matrix for which the
// low-precision maps solve a block pair through block eigenbases: the FP64 rounding error of that
// solve grows like kappa_I kappa_J u <= 1e8 * 1.1e-16, two orders below FP32 rounding.
constexpr double kBlkKappaMax = 1e4;  // longest GMRES cycle (basis vectors kept in HBM)
constexpr int kHostScalars = 2 * kMaxLong + 4096;  // complex128 slots of the pinned host buffer
// recycled subspace of the GCRO-DR solver: (A P) U = C with orthonormal C, k vectors of n*n
struct Recycle {
  int k = 0, cap = 0;
  long long n2 = 0;
  zd *U = nullptr, *Un = nullptr, *C = nullptr;
  zd* coef = nullptr;  // device staging of the small coefficient matrices
  zd* hb = nullptr;    // device Gram-Schmidt coefficients and norm of the current step
  void* ws = nullptr;  // split-K workspace of the cross products
  long long ws_bytes = 0;
  void reset() { k = 0; }
  int ensure(Ctx& c, int kcap);
  int cross(Ctx& c, const zd* Urows, int M, const zd* Vrows, int N, zd* T);
};

struct Ctx {
  int n = 0, d = 0;
  int dev = 0;  // HIP device the context was created on
  long long n2 = 0;
  lind_opts opts;
  hipStream_t st = nullptr;
  std::string err;
  int route = LIND_ROUTE_EIG;
  int prec = PREC_F64;
  double kappa = 0.0;
  double t_factor = 0.0, t_hess = 0.0, t_qr = 0.0;
  double gnorm = 0.0;

  // FP64 operator data
  zd *H = nullptr, *L = nullptr, *G = nullptr, *T = nullptr, *Z = nullptr, *U = nullptr, *V = nullptr;
  // gauge-shifted split: H, L hold the shifted operators; L0 the given jump operators (gradients)
  zd* L0 = nullptr;
  std::vector<cplx> gauge;
  zd *s = nullptr, *sbar = nullptr;
  zd *Lt = nullptr;    // L_j U (eigen route) or L_j Z (Schur route), stacked d x n x n
  zd *Tadj = nullptr;  // J T^H J (upper triangular) for the adjoint Schur solve
  zd *tsws = nullptr;  // partial block products of the triangular Sylvester solve
  std::vector<cplx> s_host;
  // low-precision operands (complex64)
  zf *U32 = nullptr, *V32 = nullptr, *Z32 = nullptr, *Lt32 = nullptr;
  // Schur route, low-precision modes: eigenbases of the diagonal blocks of T and of T_adj
  TsBlk tsb, tsb_adj;
  // work
  zd *w1 = nullptr, *w2 = nullptr, *w3 = nullptr, *w4 = nullptr, *Ys = nullptr;
  zf *a32 = nullptr, *b32 = nullptr, *Y32 = nullptr;
  void* gws = nullptr;    // split-K workspace of the batch-reduction products
  long long gws_bytes = 0;
  // BF16x3 eigen route: pre-split bf16 planes of V^H, V^T, the stacked L_j U (constants) and of
  // the intermediates of Phi; FP32 split-K partials of the jump reduction
  bool p4_ready = false;
  P4 p4_VH, p4_VT, p4_Lt, p4_xiT, p4_C1, p4_XhT, p4_Y;
  float2* p4_ws = nullptr;
  int p4_nsplit = 1;
  // BF16x3 Lindbladian (inner solves of lind_eigs, allocated on first use): the batched operands of
  //   L(X) = sum_j Y_j L_j^H + G X + X G^H,  Y = [L_1; ..; L_d] X,
  // A rows [Y_1 .. Y_d | G | X], B rows [L_1 .. L_d | conj(X^T) | G] (each block n rows, read with
  // B conjugated), and X^T for the stacked product
  bool p4L_ready = false;
  P4 p4L_A, p4L_B, p4L_xT;
  float2* p4L_ws = nullptr;
  int p4L_nsplit = 1;
  zd* dsc = nullptr;      // device scalars
  double* dscr = nullptr; // reduction scratch
  long long dscr_len = 0;
  zd* hsc = nullptr;      // pinned host scalars
  // Krylov bases (lazily allocated): outer and inner
  zd* K1 = nullptr;
  int K1cap = 0;
  zd* K2 = nullptr;
  int K2cap = 0;
  // eigs: cached W = R_mu(I) and Tr W
  bool W_valid = false;
  cplx W_mu = 0.0, W_tr = 0.0;
  zd* Wmu = nullptr;
  Recycle rec;  // inner-solver recycle space (valid for one operator at a time)
  std::vector<void*> allocs;
  // event timing of named kernels (enabled by lindx_profile): kinds of PROF_*
  bool prof = false;
  struct ProfSlot { hipEvent_t a, b; int kind; };
  std::vector<hipEvent_t> evpool;
  std::vector<ProfSlot> pending;
  double prof_ms[8] = {0};
  long long prof_cnt[8] = {0};
  int prof_begin(int kind);
  void prof_end(int slot);
  int prof_collect();

  ~Ctx();
  int fail(int code, const std::string& msg) { err = msg; return code; }
  template <typename T> int alloc(T** p, size_t count) {
    void* q = nullptr;
    if (count == 0) { *p = nullptr; return 0; }
    if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) return LIND_ENOMEM;
    allocs.push_back(q);
    *p = (T*)q;
    return 0;
  }
  int ensure_krylov(int which, int slots);
  void release(void* p) {
    for (auto it = allocs.begin(); it != allocs.end(); ++it)
      if (*it == p) { allocs.erase(it); break; }
    hipFree(p);
  }
  int sync();
  // host scalar fetch: copies `count` zd from device pointer into the pinned buffer and syncs
  int fetch(const void* dptr, size_t bytes);
};

// operator layer (FP64 unless noted); all buffers are n x n complex128 on the device
int op_gemm(Ctx& c, int prec, int M, int N, int K, const void* A, long long lda, int opA, const void* B,
            long long ldb, int opB, void* C, long long ldc, cplx alpha, int beta);
// X = (S - mu)^{-1} Y in precision prec (route of the context); adjoint: (S* - conj(mu))^{-1}
int op_sinv(Ctx& c, const zd* Y, zd* X, cplx mu, int prec, bool adjoint);
// out = Phi(xi) in precision prec; hermitian: xi is Hermitian (Phi preserves it), so the Hermitian
// intermediate and result are formed from the tiles on and above the diagonal
int op_phi(Ctx& c, const zd* xi, zd* out, int prec, bool hermitian = false);
// out = L(rho) (FP64); hermitian_in: rho is Hermitian (fewer products)
int op_apply(Ctx& c, const zd* rho, zd* out, bool hermitian_in);
// out = L*(X) (FP64)
int op_apply_adj(Ctx& c, const zd* X, zd* out);
// out = L(X) with BF16x3 products (FP32 accumulation, complex128 result); sets up its constant
// operand planes on the first call (eigen route only: returns LIND_EINVAL when unavailable)
int op_apply_p4(Ctx& c, const zd* X, zd* out);
// norms of an n x n matrix to host: fro, max, colsum, max|Im diag|
int op_norms(Ctx& c, const zd* X, double out[4]);
int op_trace(Ctx& c, const zd* X, cplx* tr);
int op_nrm(Ctx& c, const zd* x, double* out);

// generic right-preconditioned restarted GMRES on n*n vectors, FP64 Krylov basis (K2)
struct GmresResult {
  int iters = 0;
  int cycles = 0;
  double resid = 0.0;      // final residual 2-norm (true residual at the last restart)
  double resid0 = 0.0;
  bool converged = false;
  bool stagnated = false;  // restarts stopped reducing the true residual
  bool est_hit = false;    // the last cycle's recurrence reached the target (the true residual may
                           // still miss it: a reduced-precision operator is linear only up to rounding)
};
int gmres(Ctx& c, const std::function<int(const zd*, zd*)>& A, const std::function<int(const zd*, zd*)>* P,
          const zd* b, zd* x, bool x_zero, int m, int max_cycles, double rtol, double atol, GmresResult& res,
          double t_deadline);

double now_s();
// progress lines on stderr requested by the environment (LINDX_LOG)
bool log_on();

// device address of the fixed scratch array of lind_apply_noalloc on device dev (resolved once
// per device; lind_create calls it with the device current)
int noalloc_setup(int dev);

#define TRY_RC(x)                                        \
  do {                                                   \
    int rc__ = (x);                                      \
    if (rc__) return rc__ < 0 ? rc__ : LIND_EDEVICE;     \
  } while (0)

}  // namespace lindx

// the C ABI handle: operator context plus solver buffers
struct lind_ctx {
  lindx::Ctx c;
  lindx::zd *rhoB = nullptr, *resB = nullptr, *xiB = nullptr, *zetaB = nullptr, *delB = nullptr;
  lindx::zd *hm = nullptr, *ev = nullptr, *Yv = nullptr, *yv = nullptr;
  lindx::zd* hd = nullptr;  // (m + 1) x m Hessenberg matrix of the steady-state Arnoldi cycle
  int* sinfo = nullptr;
};

namespace lindx {
// helpers shared by the drivers (lind.cpp)
int ensure_solver_bufs(lind_ctx* X);
int ritz_near_dev(lind_ctx* X, const zd* Hd, int ld, int& k, const double* sub, cplx& theta, std::vector<cplx>& y,
                  double& rin, double& hn);
int small_eig_host(lind_ctx* X, const std::vector<cplx>& Hh, int ld, int k, std::vector<cplx>& w,
                   std::vector<cplx>& Y);
int upload_vec(lind_ctx* X, const cplx* v, int k, zd* dst);
int steady_state_impl(lind_ctx* X, double tol, const zd* rho0, zd* rho_out, lind_info* info);
// Algorithm "Steady state via preconditioned GMRES" (method LIND_METHOD_GMRES)
int steady_state_gmres(lind_ctx* X, double tol, const zd* rho0, zd* rho_out, lind_info* info);
// rho <- herm(rho)/Tr; FP64 residual L(rho) into resB; its norms (colsum bound, max, Frobenius)
int finish_state(lind_ctx* X, zd* rho, double* colsum, double* mx, double* fro, cplx* tr_before);
// right-preconditioned flexible GMRES(m) with a recycled subspace of up to kdef vectors (GCRO-DR),
// carried in rec across cycles and across solves with the same operator A (P may be null: identity).
// m <= 64 for recycling; longer cycles (up to kMaxLong) run without it.  x_zero: start from x = 0.
int gmres_rec(lind_ctx* X, const std::function<int(const zd*, zd*)>& A, const std::function<int(const zd*, zd*)>* P,
              const zd* b, zd* x, bool x_zero, int m, int kdef, int max_cycles, double rtol, double atol,
              Recycle& rec, GmresResult& res, double t_deadline);
// longest cycle (<= want) whose basis fits the HBM budget; release a long basis after use
int long_cycle_len(Ctx& c, int want, bool flexible);
void release_long_basis(Ctx& c);
}  // namespace lindx
