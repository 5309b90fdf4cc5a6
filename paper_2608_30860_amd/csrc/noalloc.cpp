// lind_apply_noalloc: L(rho) with every intermediate in a fixed device array instead of the
// context's workspaces, for callers that cannot allocate device memory while they run (code
// under stream capture, serving loops, harnesses that forbid hipMalloc).  Same kernels as
// lind_apply: the stacked product [L_1; ..; L_d] rho and the batch reduction over j with its
// split-K partials, here placed in `scratch`.
#include <cmath>
#include <mutex>
#include "ctx.hpp"

namespace lindx {

// one copy per GPU, alive until the process ends; host code never passes the array's name to a
// kernel (in host code it is only a stand-in): it uses the device address resolved below
static __device__ __align__(256) unsigned char scratch[LIND_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices] = {nullptr};
int g_state[kMaxDevices] = {0};  // 0: not resolved, 1: resolved, -1: resolution failed
}  // namespace

// resolve the scratch array's device address on the current device (once per device); called by
// lind_create with the context's device current
int noalloc_setup(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return LIND_EINVAL;
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_state[dev] == 0) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e == hipSuccess && p) {
      g_ptr[dev] = p;
      g_state[dev] = 1;
    } else {
      g_state[dev] = -1;
    }
  }
  return g_state[dev] == 1 ? 0 : LIND_EDEVICE;
}

static void* scratch_ptr(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_mu);
  return g_state[dev] == 1 ? g_ptr[dev] : nullptr;
}

// bytes of scratch the variant needs: the stacked products L_j rho (d n^2 complex128) and the
// split-K partials of the reduction over j, each part 256-byte aligned
static long long noalloc_need(int n, int d, long long* ws_off) {
  const long long n2 = (long long)n * n;
  const long long ys = ((long long)d * n2 * 16 + 255) / 256 * 256;
  *ws_off = ys;
  return ys + (d > 0 ? gemm_ws_bytes(PREC_F64, n, n, d) : 0);
}

}  // namespace lindx

using namespace lindx;

extern "C" long long lind_apply_noalloc_bytes(int n, int d) {
  if (n < 1 || d < 0) return -1;
  long long off = 0;
  return noalloc_need(n, d, &off);
}

extern "C" int lind_apply_noalloc(lind_ctx* ctx, const void* rho, void* out) {
  if (!ctx || !rho || !out || rho == out) return LIND_EINVAL;
  Ctx& c = ctx->c;
  const int n = c.n, d = c.d;
  const long long n2 = c.n2;
  long long ws_off = 0;
  const long long need = noalloc_need(n, d, &ws_off);
  if (need > (long long)LIND_NOALLOC_SCRATCH_BYTES)
    return c.fail(LIND_EINVAL, "lind_apply_noalloc: the products need more than the fixed scratch of "
                               "LIND_NOALLOC_SCRATCH_BYTES (d n^2 complex128 plus split-K partials)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != c.dev)
    return c.fail(LIND_EINVAL, "lind_apply_noalloc: the context's device is not the current device");
  unsigned char* base = (unsigned char*)scratch_ptr(c.dev);
  if (!base) return c.fail(LIND_EDEVICE, "lind_apply_noalloc: the scratch array's device address is unavailable");
  zd* Ys = (zd*)base;
  const cplx one(1, 0);
  // G rho + rho G^H, then + sum_j (L_j rho) L_j^H as one batch reduction (as lind_apply)
  TRY_RC(op_gemm(c, PREC_F64, n, n, n, c.G, n, OP_N, (const zd*)rho, n, OP_N, out, n, one, 0));
  TRY_RC(op_gemm(c, PREC_F64, n, n, n, (const zd*)rho, n, OP_N, c.G, n, OP_C, out, n, one, 1));
  if (d > 0) {
    TRY_RC(op_gemm(c, PREC_F64, d * n, n, n, c.L, n, OP_N, (const zd*)rho, n, OP_N, Ys, n, one, 0));
    GemmDesc g;
    g.M = n; g.N = n; g.K = n; g.nbatch = d;
    const long long wsb = need - ws_off;
    g.ws = wsb > 0 ? (void*)(base + ws_off) : nullptr;
    g.ws_bytes = wsb;
    g.A = Ys; g.lda = n; g.sA = n2; g.opA = OP_N;
    g.B = c.L; g.ldb = n; g.sB = n2; g.opB = OP_C;
    g.C = out; g.ldc = n; g.beta = 1;
    if (gemm(PREC_F64, g, c.st)) return LIND_EDEVICE;
  }
  return c.sync();
}
