// C ABI entry points: context creation (G and its FP64 factorisation on the GPU), the operator
// calls, and the steady-state driver (Algorithm "Steady state as the fixed point of Phi" with
// FP64 iterative refinement).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include "ctx.hpp"

using namespace lindx;


static thread_local std::string g_create_err;

#define TRY(x)                                           \
  do {                                                   \
    int rc__ = (x);                                      \
    if (rc__) return rc__ < 0 ? rc__ : LIND_EDEVICE;     \
  } while (0)

// BF16x3: split the constant operands of Phi into bf16 planes once (the basis change by V on the
// eigen route, by Z on the Schur route, and the fused jump operators), and allocate the planes of
// its intermediates (all zero-padded to whole tiles)
static int setup_p4(Ctx& c) {
  const int n = c.n, d = c.d;
  P4* bufs[7] = {&c.p4_VH, &c.p4_VT, &c.p4_Lt, &c.p4_xiT, &c.p4_C1, &c.p4_XhT, &c.p4_Y};
  const long long rows[7] = {n, n, (long long)d * n, n, n, n, (long long)d * n};
  for (int i = 0; i < 7; ++i) {
    if (bufs[i]->p) continue;
    if (p4_alloc(*bufs[i], rows[i], n)) return c.fail(LIND_ENOMEM, "out of device memory (bf16 planes)");
    c.allocs.push_back(bufs[i]->p);
  }
  // B^H (rows m, k: conj B[k][m]), B^T (rows j, k: B[k][j]) for B = V or Z, L_j U or L_j Z stacked
  const zd* Bm = c.route == LIND_ROUTE_EIG ? c.V : c.Z;
  if (p4_split(Bm, 1, n, n, n, 1, 1, c.p4_VH, c.st)) return LIND_EDEVICE;
  if (p4_split(Bm, 1, n, n, n, 1, 0, c.p4_VT, c.st)) return LIND_EDEVICE;
  if (p4_split(c.Lt, 1, n, d * n, n, 0, 0, c.p4_Lt, c.st)) return LIND_EDEVICE;
  // split-K of the jump reduction (d n-long products summed; only the tiles on and above the
  // diagonal of its Hermitian result are computed) in runs that fill whole rounds of the chip
  const long long tm = (n + 127) / 128;
  const int s = p4_pick_split(tm * (tm + 1) / 2, d, n, device_cus(c.dev));
  c.p4_nsplit = s;
  if (!c.p4_ws && c.alloc(&c.p4_ws, (size_t)s * c.n2)) return c.fail(LIND_ENOMEM, "out of device memory (split-K)");
  c.p4_ready = true;
  return 0;
}

extern "C" void lind_default_opts(lind_opts* o) {
  if (!o) return;
  o->prec = LIND_PREC_FP64;
  o->route = LIND_ROUTE_AUTO;
  o->kappa_max = 1e3;
  o->m = 30;
  o->p = 0;
  o->max_restarts = 200;
  o->refine_max = 8;
  o->eta = 1.0;
  o->time_limit_s = 0.0;
  o->stream = nullptr;
  o->method = LIND_METHOD_PHI_ARNOLDI;
  o->gauge = nullptr;
}

static int prec_of(int p) {
  if (p == LIND_PREC_FP32) return PREC_F32;
  if (p == LIND_PREC_BF16X3) return PREC_BF16X3;
  return PREC_F64;
}

__global__ void k_nonfinite(const double* x, long long len, int* flag) {
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += stride)
    if (!isfinite(x[i])) flag[0] = 1;
}
// xi = -(G v + v G^H) for rho = v I: -v (G + G^H), elementwise
__global__ void k_minus_herm_part(const zd* G, int n, double v, zd* xi) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    const long long i = t / n, j = t - i * n;
    const zd a = G[t], b = G[j * n + i];
    xi[t] = zmk(-v * (a.x + b.x), -v * (a.y - b.y));
  }
}
__global__ void k_fill_identity_scaled(zd* X, int n, double v) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride)
    X[t] = (t / n == t % n) ? zmk(v, 0) : zmk(0, 0);
}

// eq. lindblad_gauge: with Lt_j = L_j + c_j I (already applied to L),
// H <- H + (1/2i) sum_j (conj(c_j) Lt_j - c_j Lt_j^+), elementwise
__global__ void k_gauge_H(zd* H, const zd* Lt, const zd* cs, int n, int d) {
  const long long tot = (long long)n * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    const long long a = t / n, b = t % n;
    double sr = 0, si = 0;
    for (int j = 0; j < d; ++j) {
      const zd cj = cs[j];
      const zd x = Lt[(long long)j * tot + a * n + b];   // Lt_j[a][b]
      const zd y = Lt[(long long)j * tot + b * n + a];   // Lt_j[b][a]; (Lt_j^+)[a][b] = conj(y)
      // conj(c) x - c conj(y)
      sr += (cj.x * x.x + cj.y * x.y) - (cj.x * y.x + cj.y * y.y);
      si += (cj.x * x.y - cj.y * x.x) - (cj.y * y.x - cj.x * y.y);
    }
    // (1/2i)(sr + i si) = si/2 - i sr/2
    H[t] = zmk(H[t].x + 0.5 * si, H[t].y - 0.5 * sr);
  }
}

static int count_nonfinite(Ctx& c, const zd* x, long long len, int* flag_dev, bool* bad) {
  if (fill_zero(flag_dev, sizeof(int), c.st)) return LIND_EDEVICE;
  long long nb = (2 * len + 255) / 256;
  if (nb > 8192) nb = 8192;
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL(k_nonfinite, dim3((int)nb), dim3(256), 0, c.st, (const double*)x, 2 * len, flag_dev);
  TRY(c.fetch(flag_dev, sizeof(int)));
  *bad = ((const int*)c.hsc)[0] != 0;
  return 0;
}

// kappa_2(M) estimate for n x n M: sqrt of the largest eigenvalue of M^H M by power iteration.
static int power_norm(Ctx& c, const zd* M, zd* x, zd* y, int iters, double* out) {
  const int n = c.n;
  double nrm = 0;
  if (iters < 1) return LIND_EINVAL;
  for (int it = 0; it < iters; ++it) {
    // y holds n entries of an n x n buffer; the rest is the scratch of the two-pass A^H x
    zd* scratch = gemv_scratch_elems(n) <= (long long)n * n - n ? y + n : nullptr;
    TRY(gemv(M, n, OP_N, x, y, nullptr, c.st));
    TRY(gemv(M, n, OP_C, y, x, scratch, c.st));
    TRY(nrm2(x, n, (double*)c.dsc, c.dscr, c.st));
    TRY(scale_by_inv(x, n, (const double*)c.dsc, c.st));
  }
  // only the last iterate's norm is used: one read-back after the loop
  TRY(c.fetch(c.dsc, sizeof(double)));
  nrm = ((const double*)c.hsc)[0];
  *out = std::sqrt(nrm);
  return 0;
}

static int ctx_factor(lind_ctx* X) {
  Ctx& c = X->c;
  const int n = c.n, d = c.d;
  const long long n2 = c.n2;
  const cplx one(1, 0);
  double t0 = now_s();
  // W = sum_j L_j^H L_j (one launch, reduction over j), G = -iH - W/2   (eq. G)
  if (d > 0) {
    GemmDesc g;
    g.M = n; g.N = n; g.K = n; g.nbatch = d; g.ws = c.gws; g.ws_bytes = c.gws_bytes;
    g.A = c.L; g.lda = n; g.sA = n2; g.opA = OP_C;
    g.B = c.L; g.ldb = n; g.sB = n2; g.opB = OP_N;
    g.C = c.w1; g.ldc = n;
    TRY(gemm(PREC_F64, g, c.st));
  } else {
    TRY(fill_zero(c.w1, n2 * (long long)sizeof(zd), c.st));
  }
  TRY(make_generator(c.H, c.w1, c.G, n, c.st));
  double gn[4];
  TRY(op_norms(c, c.G, gn));
  c.gnorm = gn[0];
  // Schur form G = Z T Z^H
  TRY(copy(c.G, c.T, n2, c.st));
  int rc = schur_factor(c.T, c.Z, n, c.st, &c.t_hess, &c.t_qr);
  if (rc == -3) return c.fail(LIND_ENOCONV, "QR iteration on G did not converge");
  if (rc == -5) return c.fail(LIND_ENOMEM, "out of device memory in the factorisation");
  if (rc) return c.fail(LIND_EDEVICE, "factorisation failed");
  TRY(diag_extract(c.T, c.s, n, c.st));
  TRY(conj_copy(c.s, c.sbar, n, c.st));
  c.s_host.resize(n);
  {
    std::vector<zd> hs(n);
    if (hipMemcpyAsync(hs.data(), c.s, sizeof(zd) * n, hipMemcpyDeviceToHost, c.st) != hipSuccess) return LIND_EDEVICE;
    TRY(c.sync());
    for (int i = 0; i < n; ++i) c.s_host[i] = cplx(hs[i].x, hs[i].y);
  }
  // Theorem 1: S invertible iff spec(G) avoids the imaginary axis
  double minre = 1e300, maxre = -1e300;
  for (auto& z : c.s_host) {
    minre = std::min(minre, std::fabs(z.real()));
    maxre = std::max(maxre, z.real());
  }
  if (!(minre > 1e-13 * std::max(c.gnorm, 1e-300)) || maxre >= 0)
    return c.fail(LIND_ESINGULAR, "spec(G) meets the imaginary axis: S is not invertible");
  // eigenvectors: Y (upper triangular), Y^{-1}; U = Z Y, V = Z Y^{-H}; unit columns of U
  // (U and V serve as the solves' workspaces before they receive their values)
  TRY(trevec(c.T, c.U, c.w2, n, c.st));
  TRY(triinv_unit(c.w2, c.V, c.w3, n, c.st));
  TRY(op_gemm(c, PREC_F64, n, n, n, c.Z, n, OP_N, c.w2, n, OP_N, c.U, n, one, 0));
  TRY(op_gemm(c, PREC_F64, n, n, n, c.Z, n, OP_N, c.w3, n, OP_C, c.V, n, one, 0));
  double* cn = (double*)c.dscr;  // n doubles
  TRY(col_norms(c.U, n, cn, c.st));
  TRY(scale_cols(c.U, n, cn, 1, c.st));
  TRY(scale_cols(c.V, n, cn, 0, c.st));
  // kappa_2(U) = ||U||_2 ||U^{-1}||_2 = ||U||_2 ||V||_2
  {
    std::vector<zd> x0(n);
    std::mt19937_64 rng(12345);
    std::normal_distribution<double> nd;
    for (auto& z : x0) z = zmk(nd(rng), nd(rng));
    if (hipMemcpyAsync(c.w1, x0.data(), sizeof(zd) * n, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
    TRY(c.sync());
    double su = 0, sv = 0;
    TRY(power_norm(c, c.U, c.w1, c.w2, 40, &su));
    if (hipMemcpyAsync(c.w1, x0.data(), sizeof(zd) * n, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
    TRY(c.sync());
    TRY(power_norm(c, c.V, c.w1, c.w2, 40, &sv));
    c.kappa = su * sv;
  }
  int route = c.opts.route;
  if (route == LIND_ROUTE_AUTO) route = (c.kappa <= c.opts.kappa_max) ? LIND_ROUTE_EIG : LIND_ROUTE_SCHUR;
  c.route = route;
  // fused jump operands Lt_j = L_j U (eigen route) or L_j Z (Schur route): one launch, M = d n
  const zd* B = (route == LIND_ROUTE_EIG) ? c.U : c.Z;
  if (d > 0) TRY(op_gemm(c, PREC_F64, d * n, n, n, c.L, n, OP_N, B, n, OP_N, c.Lt, n, one, 0));
  if (route == LIND_ROUTE_SCHUR) TRY(flip_conj_transpose(c.T, c.Tadj, n, c.st));
  if (route == LIND_ROUTE_SCHUR && c.prec != PREC_F64 && !c.tsb.kap) {
    // the low-precision maps solve well-conditioned diagonal block pairs through block eigenbases
    const long long be = trisylv_blk_elems(n), nbk = (n + 31) / 32;
    zd *y, *yi, *ya, *yia;
    double *k, *ka;
    if (c.alloc(&y, be) || c.alloc(&yi, be) || c.alloc(&ya, be) || c.alloc(&yia, be) ||
        c.alloc(&k, nbk) || c.alloc(&ka, nbk))
      return c.fail(LIND_ENOMEM, "out of device memory (block eigenbases)");
    TRY(trisylv_blk_setup(c.T, n, y, yi, k, c.st));
    TRY(trisylv_blk_setup(c.Tadj, n, ya, yia, ka, c.st));
    c.tsb.Y = y; c.tsb.Yi = yi; c.tsb.kap = k; c.tsb.thr = kBlkKappaMax;
    c.tsb_adj.Y = ya; c.tsb_adj.Yi = yia; c.tsb_adj.kap = ka; c.tsb_adj.thr = kBlkKappaMax;
  }
  if (c.prec != PREC_F64) {
    TRY(to_c64(c.U, c.U32, n2, c.st));
    TRY(to_c64(c.V, c.V32, n2, c.st));
    TRY(to_c64(c.Z, c.Z32, n2, c.st));
    if (d > 0) TRY(to_c64(c.Lt, c.Lt32, (long long)d * n2, c.st));
  }
  if (c.prec == PREC_BF16X3 && d > 0) TRY(setup_p4(c));
  TRY(c.sync());
  c.t_factor = now_s() - t0;
  return 0;
}

extern "C" int lind_create(lind_ctx** out, const void* H, const void* Ls, int n, int d, const lind_opts* opts) {
  g_create_err.clear();
  if (!out) { g_create_err = "out is NULL"; return LIND_EINVAL; }
  *out = nullptr;
  if (!H || n < 1 || d < 0 || d > 64 || (d > 0 && !Ls)) {
    g_create_err = "invalid arguments (need H, n >= 1, 0 <= d <= 64, L when d > 0)";
    return LIND_EINVAL;
  }
  if (n > LIND_NMAX) {
    g_create_err = "n > 10240: the eigenvector solves keep one column's right-hand sides in 160 KB of LDS";
    return LIND_EINVAL;
  }
  lind_opts o;
  lind_default_opts(&o);
  if (opts) o = *opts;
  if (o.m < 4 || o.m > 64 || !(o.eta > 0) || o.prec < 0 || o.prec > 2 || o.route < 0 || o.route > 2 ||
      o.max_restarts < 1 || o.refine_max < 0 || o.method < 0 || o.method > 1) {
    g_create_err = "invalid options (m in [4, 64], eta > 0, prec/route/method enums, max_restarts >= 1)";
    return LIND_EINVAL;
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess ||
      std::strstr(prop.gcnArchName, "gfx950") == nullptr) {
    g_create_err = "no gfx950 (MI355X) device available";
    return LIND_EDEVICE;
  }
  // the fixed scratch of lind_apply_noalloc is resolved here, once per device (failure only
  // disables that entry point)
  noalloc_setup(dev);
  lind_ctx* X = new lind_ctx();
  Ctx& c = X->c;
  c.dev = dev;
  c.n = n;
  c.d = d;
  c.n2 = (long long)n * n;
  c.opts = o;
  c.st = (hipStream_t)o.stream;
  c.prec = prec_of(o.prec);
  const long long n2 = c.n2;
  const size_t nd = (size_t)std::max(d, 1) * n2;
  c.dscr_len = std::max<long long>(2LL * 66 * 1024 + 64, 3LL * 32 * n + 4LL * n + 64);
  int rc = 0;
  rc |= c.alloc(&c.H, n2); rc |= c.alloc(&c.L, nd); rc |= c.alloc(&c.G, n2); rc |= c.alloc(&c.T, n2);
  rc |= c.alloc(&c.Z, n2); rc |= c.alloc(&c.U, n2); rc |= c.alloc(&c.V, n2); rc |= c.alloc(&c.s, n);
  rc |= c.alloc(&c.sbar, n); rc |= c.alloc(&c.Lt, nd); rc |= c.alloc(&c.Tadj, n2);
  rc |= c.alloc(&c.tsws, trisylv_ws_elems(n));
  rc |= c.alloc(&c.w1, n2); rc |= c.alloc(&c.w2, n2); rc |= c.alloc(&c.w3, n2); rc |= c.alloc(&c.w4, n2);
  rc |= c.alloc(&c.Ys, nd); rc |= c.alloc(&c.dsc, 1024); rc |= c.alloc(&c.dscr, (size_t)c.dscr_len);
  rc |= c.alloc(&X->hm, 64 * 64); rc |= c.alloc(&X->ev, 64); rc |= c.alloc(&X->Yv, 64 * 64);
  rc |= c.alloc(&X->yv, 64); rc |= c.alloc(&X->sinfo, 16); rc |= c.alloc(&X->hd, 65 * 64);
  if (c.prec != PREC_F64) {
    rc |= c.alloc(&c.U32, n2); rc |= c.alloc(&c.V32, n2); rc |= c.alloc(&c.Z32, n2);
    rc |= c.alloc(&c.Lt32, nd); rc |= c.alloc(&c.a32, n2); rc |= c.alloc(&c.b32, n2); rc |= c.alloc(&c.Y32, nd);
  }
  {
    long long wsb = std::max(gemm_ws_bytes(PREC_F64, n, n, std::max(d, 1)), gemm_ws_bytes(c.prec, n, n, std::max(d, 1)));
    // single products of small systems split along K
    wsb = std::max(wsb, gemm_ws_bytes(PREC_F64, n, n, 1));
    if (d >= 1) wsb = std::max(wsb, gemm_ws_bytes(PREC_F64, d * n, n, 1));
    // room for up to 8 FP64 split-K partials (the Hermitian residual runs on half the tiles)
    if (d >= 2) wsb = std::max(wsb, (long long)std::min(d, 8) * n2 * 16);
    if (wsb > 0) rc |= c.alloc((char**)&c.gws, (size_t)wsb);
    c.gws_bytes = wsb;
  }
  if (rc == 0 && hipHostMalloc((void**)&c.hsc, sizeof(zd) * kHostScalars) != hipSuccess) rc = LIND_ENOMEM;
  if (rc) {
    delete X;
    g_create_err = "out of device memory";
    return LIND_ENOMEM;
  }
  bool bad = false;
  int frc = 0;
  if (hipMemcpyAsync(c.H, H, sizeof(zd) * n2, hipMemcpyDeviceToDevice, c.st) != hipSuccess ||
      (d > 0 && hipMemcpyAsync(c.L, Ls, sizeof(zd) * (size_t)d * n2, hipMemcpyDeviceToDevice, c.st) != hipSuccess)) {
    delete X;
    g_create_err = "copy of H / L failed (are they device pointers?)";
    return LIND_EDEVICE;
  }
  frc = count_nonfinite(c, c.H, n2, X->sinfo, &bad);
  if (!frc && !bad && d > 0) frc = count_nonfinite(c, c.L, (long long)d * n2, X->sinfo, &bad);
  if (frc || bad) {
    delete X;
    g_create_err = frc ? "device error while checking inputs" : "non-finite entries in H or L";
    return frc ? LIND_EDEVICE : LIND_EINVAL;
  }
  if (o.gauge && d > 0) {
    // keep the given L for the gradients, factorise the shifted split
    std::vector<zd> cs(d);
    for (int j = 0; j < d; ++j) {
      cs[j] = zmk(o.gauge[2 * j], o.gauge[2 * j + 1]);
      if (!std::isfinite(cs[j].x) || !std::isfinite(cs[j].y)) {
        delete X;
        g_create_err = "non-finite gauge shift";
        return LIND_EINVAL;
      }
    }
    zd* cdev = nullptr;
    int grc = c.alloc(&c.L0, (size_t)d * n2) | c.alloc(&cdev, (size_t)d);
    if (!grc && hipMemcpyAsync(c.L0, c.L, sizeof(zd) * (size_t)d * n2, hipMemcpyDeviceToDevice, c.st) != hipSuccess) grc = 1;
    if (!grc && hipMemcpyAsync(cdev, cs.data(), sizeof(zd) * d, hipMemcpyHostToDevice, c.st) != hipSuccess) grc = 1;
    for (int j = 0; j < d && !grc; ++j) grc = add_identity(c.L + (long long)j * n2, n, cs[j], c.st);
    if (!grc) {
      hipLaunchKernelGGL(k_gauge_H, dim3(1024), dim3(256), 0, c.st, c.H, (const zd*)c.L, (const zd*)cdev, n, d);
      grc = hipGetLastError() != hipSuccess;
    }
    if (!grc) grc = c.sync();
    if (grc) {
      delete X;
      g_create_err = "gauge shift failed";
      return LIND_EDEVICE;
    }
    c.gauge.assign(d, cplx(0, 0));
    for (int j = 0; j < d; ++j) c.gauge[j] = cplx(cs[j].x, cs[j].y);
  }
  c.opts.gauge = nullptr;  // host memory of the caller: not kept
  rc = ctx_factor(X);
  if (rc) {
    g_create_err = c.err.empty() ? "factorisation failed" : c.err;
    delete X;
    return rc;
  }
  *out = X;
  return LIND_OK;
}

extern "C" void lind_destroy(lind_ctx* ctx) {
  if (!ctx) return;
  hipStreamSynchronize(ctx->c.st);
  delete ctx;
}

// kernel timing (include/lind_internal.h)
extern "C" int lindx_profile(lind_ctx* ctx, int enable) {
  if (!ctx) return LIND_EINVAL;
  Ctx& c = ctx->c;
  TRY(c.prof_collect());
  for (int i = 0; i < 8; ++i) { c.prof_ms[i] = 0; c.prof_cnt[i] = 0; }
  c.prof = enable != 0;
  return 0;
}
extern "C" int lindx_profile_read(lind_ctx* ctx, int kind, long long* count, double* total_ms) {
  if (!ctx || kind < 0 || kind >= 8 || !count || !total_ms) return LIND_EINVAL;
  Ctx& c = ctx->c;
  TRY(c.prof_collect());
  *count = c.prof_cnt[kind];
  *total_ms = c.prof_ms[kind];
  return 0;
}

extern "C" const char* lind_last_error(const lind_ctx* ctx) {
  if (!ctx) return g_create_err.c_str();
  return ctx->c.err.c_str();
}

extern "C" const void* lind_factor_ptr(const lind_ctx* ctx, int which) {
  if (!ctx) return nullptr;
  const Ctx& c = ctx->c;
  switch (which) {
    case 0: return c.G;
    case 1: return c.T;
    case 2: return c.Z;
    case 3: return c.U;
    case 4: return c.V;
    case 5: return c.s;
    default: return nullptr;
  }
}

extern "C" int lind_apply(lind_ctx* ctx, const void* rho, void* out) {
  if (!ctx || !rho || !out || rho == out) return LIND_EINVAL;
  Ctx& c = ctx->c;
  TRY(op_apply(c, (const zd*)rho, (zd*)out, false));
  return c.sync();
}

// out = L(X) with BF16x3 products (include/lind_internal.h; the operator of the inner solves of
// lind_eigs in BF16x3 contexts)
extern "C" int lindx_apply_bf16(lind_ctx* ctx, const void* X, void* out) {
  if (!ctx || !X || !out || X == out) return LIND_EINVAL;
  Ctx& c = ctx->c;
  TRY(op_apply_p4(c, (const zd*)X, (zd*)out));
  return c.sync();
}

extern "C" int lind_apply_adjoint(lind_ctx* ctx, const void* X, void* out) {
  if (!ctx || !X || !out || X == out) return LIND_EINVAL;
  Ctx& c = ctx->c;
  TRY(op_apply_adj(c, (const zd*)X, (zd*)out));
  return c.sync();
}

static bool divisor_vanishes(const Ctx& c, cplx mu) {
  // min_ij |s_i + conj(s_j) - mu| relative to ||G||
  double tol = 1e-14 * std::max(c.gnorm, 1e-300);
  for (int i = 0; i < c.n; ++i) {
    double re = c.s_host[i].real() - mu.real();
    double im = c.s_host[i].imag() - mu.imag();
    for (int j = 0; j < c.n; ++j) {
      double a = re + c.s_host[j].real();
      if (std::fabs(a) > tol) continue;
      double b = im - c.s_host[j].imag();
      if (std::hypot(a, b) <= tol) return true;
    }
  }
  return false;
}

extern "C" int lind_sinv(lind_ctx* ctx, const void* Y, void* Xo, double mu_re, double mu_im) {
  if (!ctx || !Y || !Xo || !std::isfinite(mu_re) || !std::isfinite(mu_im)) return LIND_EINVAL;
  Ctx& c = ctx->c;
  cplx mu(mu_re, mu_im);
  if (divisor_vanishes(c, mu)) return c.fail(LIND_ESINGULAR, "mu - s_i - conj(s_j) vanishes");
  TRY(op_sinv(c, (const zd*)Y, (zd*)Xo, mu, PREC_F64, false));
  return c.sync();
}

extern "C" int lind_phi(lind_ctx* ctx, const void* xi, void* out) {
  if (!ctx || !xi || !out || xi == out) return LIND_EINVAL;
  Ctx& c = ctx->c;
  TRY(op_phi(c, (const zd*)xi, (zd*)out, c.prec));
  TRY(c.sync());
  return c.prof_collect();
}

// ---------------------------------------------------------------------------------------------
// steady state
// ---------------------------------------------------------------------------------------------
int lindx::ensure_solver_bufs(lind_ctx* X) {
  Ctx& c = X->c;
  if (X->rhoB) return 0;
  int rc = 0;
  rc |= c.alloc(&X->rhoB, c.n2); rc |= c.alloc(&X->resB, c.n2); rc |= c.alloc(&X->xiB, c.n2);
  rc |= c.alloc(&X->zetaB, c.n2); rc |= c.alloc(&X->delB, c.n2);
  return rc ? LIND_ENOMEM : 0;
}

// small eigenproblem of the k x k leading block of the host matrix Hh (row stride ld)
int lindx::small_eig_host(lind_ctx* X, const std::vector<cplx>& Hh, int ld, int k, std::vector<cplx>& w,
                          std::vector<cplx>& Y) {
  Ctx& c = X->c;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) c.hsc[i * k + j] = zmk(Hh[(size_t)i * ld + j].real(), Hh[(size_t)i * ld + j].imag());
  if (hipMemcpyAsync(X->hm, c.hsc, sizeof(zd) * k * k, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
  TRY(small_eig(X->hm, k, k, X->ev, X->Yv, X->sinfo, c.st));
  if (hipMemcpyAsync(c.hsc, X->ev, sizeof(zd) * k, hipMemcpyDeviceToHost, c.st) != hipSuccess) return LIND_EDEVICE;
  if (hipMemcpyAsync(c.hsc + 64, X->Yv, sizeof(zd) * k * k, hipMemcpyDeviceToHost, c.st) != hipSuccess)
    return LIND_EDEVICE;
  if (hipMemcpyAsync(c.hsc + 8000, X->sinfo, sizeof(int), hipMemcpyDeviceToHost, c.st) != hipSuccess)
    return LIND_EDEVICE;
  TRY(c.sync());
  w.resize(k);
  Y.resize((size_t)k * k);
  for (int i = 0; i < k; ++i) w[i] = cplx(c.hsc[i].x, c.hsc[i].y);
  for (int i = 0; i < k * k; ++i) Y[i] = cplx(c.hsc[64 + i].x, c.hsc[64 + i].y);
  int info = *(const int*)(c.hsc + 8000);
  return info ? LIND_ENOCONV : 0;
}

// Ritz pair of the k x k leading block of the device Hessenberg matrix Hd (row stride ld) whose
// value is nearest 1: theta, the unit-norm vector y (largest entry real positive; it also stays on
// the device at Yv + 1) and the residual ||H y - theta y|| inside the Krylov space.  The
// subdiagonal entries sub[0 .. k) come back in the same synchronisation: an exact zero among the
// first k - 1 (an invariant Krylov space) cuts k to the first such column and the pair is taken
// again there.  hn = sub[k - 1] for the k finally used.
int lindx::ritz_near_dev(lind_ctx* X, const zd* Hd, int ld, int& k, const double* sub, cplx& theta,
                         std::vector<cplx>& y, double& rin, double& hn) {
  Ctx& c = X->c;
  for (int pass = 0; pass < 2; ++pass) {
    TRY(ritz_near(Hd, ld, k, zmk(1.0, 0.0), X->Yv, X->sinfo, c.st));
    if (hipMemcpyAsync(c.hsc, X->Yv, sizeof(zd) * (k + 2), hipMemcpyDeviceToHost, c.st) != hipSuccess)
      return LIND_EDEVICE;
    if (hipMemcpyAsync(c.hsc + 80, sub, sizeof(double) * k, hipMemcpyDeviceToHost, c.st) != hipSuccess)
      return LIND_EDEVICE;
    TRY(c.sync());
    const double* hs = (const double*)(c.hsc + 80);
    int kb = k;
    for (int i = 0; i + 1 < k; ++i)
      if (hs[i] == 0.0) { kb = i + 1; break; }
    if (kb < k && pass == 0) { k = kb; continue; }
    hn = hs[k - 1];
    theta = cplx(c.hsc[0].x, c.hsc[0].y);
    y.resize(k);
    for (int i = 0; i < k; ++i) y[i] = cplx(c.hsc[1 + i].x, c.hsc[1 + i].y);
    rin = c.hsc[k + 1].x;
    break;
  }
  return std::isfinite(rin) && std::isfinite(theta.real()) ? 0 : LIND_ENOCONV;
}

int lindx::upload_vec(lind_ctx* X, const cplx* v, int k, zd* dst) {
  Ctx& c = X->c;
  for (int i = 0; i < k; ++i) c.hsc[i] = zmk(v[i].real(), v[i].imag());
  if (hipMemcpyAsync(dst, c.hsc, sizeof(zd) * k, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
  return c.sync();
}

// rho <- hermitise, normalise (trace 1); res = L(rho); norms (colsum bound, max) to host
int lindx::finish_state(lind_ctx* X, zd* rho, double* colsum, double* mx, double* fro, cplx* tr_before) {
  Ctx& c = X->c;
  TRY(hermitize(rho, c.n, 1, c.dsc + 900, c.dscr, c.st));
  if (tr_before) {
    TRY(c.fetch(c.dsc + 900, sizeof(zd)));
    *tr_before = cplx(c.hsc[0].x, c.hsc[0].y);
  }
  TRY(op_apply(c, rho, X->resB, true));
  double nr[4];
  TRY(op_norms(c, X->resB, nr));
  *fro = nr[0];
  *mx = nr[1];
  *colsum = nr[2];
  return 0;
}

extern "C" int lind_steady_state(lind_ctx* ctx, double tol, const void* rho0, void* rho_out, lind_info* info) {
  if (!ctx || !rho_out || !(tol > 0) || !std::isfinite(tol)) return LIND_EINVAL;
  const int rc = steady_state_impl(ctx, tol, (const zd*)rho0, (zd*)rho_out, info);
  const int prc = ctx->c.prof_collect();
  return rc ? rc : prc;
}

int lindx::steady_state_impl(lind_ctx* ctx, double tol, const zd* rho0, zd* rho_out, lind_info* info) {
  lind_ctx* X = ctx;
  Ctx& c = X->c;
  if (c.opts.method == LIND_METHOD_GMRES) return steady_state_gmres(X, tol, rho0, rho_out, info);
  const int n = c.n;
  const long long n2 = c.n2;
  const int m = c.opts.m;
  const int p = c.prec;
  const double t0 = now_s();
  const double deadline = c.opts.time_limit_s > 0 ? t0 + c.opts.time_limit_s : 0.0;
  TRY(ensure_solver_bufs(X));
  TRY(c.ensure_krylov(1, m + 2));
  zd* K = c.K1;
  const cplx one(1, 0), mone(-1, 0);
  lind_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.kappa_U = c.kappa;
  inf.t_factor_s = c.t_factor;
  inf.route_used = c.route;
  // start state and xi_0 = -S(rho_0)
  if (rho0) {
    // the Hermitian part of the start state (the steady state is Hermitian), so that every Krylov
    // vector is Hermitian
    TRY(copy((const zd*)rho0, X->rhoB, n2, c.st));
    TRY(hermitize(X->rhoB, n, 0, nullptr, c.dscr, c.st));
  } else {
    hipLaunchKernelGGL(k_fill_identity_scaled, dim3(1024), dim3(256), 0, c.st, X->rhoB, n, 1.0 / n);
  }
  // first Krylov vector xi = -S(rho) / ||.|| from the state in rhoB; c_scale converts the Ritz
  // residual estimate into a bound on the state's residual
  double c_scale = 1.0;
  bool rho_is_identity = !rho0;  // rhoB = I/n: -S(I/n) = -(G + G^H)/n needs no product
  auto start_from_rho = [&]() -> int {
    if (rho_is_identity) {
      hipLaunchKernelGGL(k_minus_herm_part, dim3(1024), dim3(256), 0, c.st, (const zd*)c.G, n, 1.0 / n, X->xiB);
      if (hipGetLastError() != hipSuccess) return LIND_EDEVICE;
    } else {
      TRY(op_gemm(c, PREC_F64, n, n, n, c.G, n, OP_N, X->rhoB, n, OP_N, X->xiB, n, mone, 0));
      TRY(op_gemm(c, PREC_F64, n, n, n, X->rhoB, n, OP_N, c.G, n, OP_C, X->xiB, n, mone, 1));
    }
    double xin = 0;
    TRY(op_nrm(c, X->xiB, &xin));
    if (!(xin > 0) || !std::isfinite(xin)) return c.fail(LIND_EINVAL, "start state gives xi_0 = 0 or non-finite");
    cplx tr0;
    TRY(op_trace(c, X->rhoB, &tr0));
    c_scale = std::sqrt((double)n) * xin / std::max(std::abs(tr0), 1e-300);
    TRY(copy(X->xiB, K, n2, c.st));
    TRY(op_nrm(c, K, &xin));
    TRY(scale_by_inv(K, n2, (const double*)c.dsc, c.st));
    return 0;
  };
  TRY(start_from_rho());

  const double eps_floor = (p == PREC_F64) ? 0.0 : (p == PREC_F32 ? 1e-6 : 3e-3);
  double best = 1e300, best_max = 0;
  bool converged = false;
  double colsum = 0, mx = 0, fro = 0;
  bool floor_hit = false;
  bool best_is_last = false;  // rhoB / resB hold the best state and its FP64 residual
  int restarts_left = c.opts.max_restarts;
  // pass 0: restarted Arnoldi until the tolerance, its estimate's floor, or (FP64) a residual that
  // oscillates without progress, then refinement on the FP64 residual.  If refinement stalls
  // short of the tolerance after an oscillation stop, pass 1 resumes the restarted Arnoldi from
  // the best state with the oscillation stop switched off.
  for (int pass = 0; pass < 2 && !converged; ++pass) {
    bool oscillation_stop = false;
    double gain_ref = 1e300, prev_colsum = 1e300;
    int restart_stall = 0;
    floor_hit = false;
    for (int rs = 0; restarts_left > 0 && !converged; ++rs) {
      --restarts_left;
      int k = 0, k_ritz = 0;  // k_ritz: the Krylov dimension the Ritz pair (theta, ysel) belongs to
      double est = 1e300;
      cplx theta(0.0, 0.0);
      double rin = 0.0;
      std::vector<cplx> ysel;
      // The Hessenberg matrix is built on the device (row stride m; the entries below the
      // subdiagonal stay zero) and read back only when a Ritz pair is evaluated, so that the steps
      // in between queue without a host round trip.  A breakdown (zero norm) leaves the next
      // vectors zero until that evaluation finds it and cuts the space there.
      if (hipMemsetAsync(X->hd, 0, sizeof(zd) * (size_t)(m + 1) * m, c.st) != hipSuccess) return LIND_EDEVICE;
      double* subd = (double*)(c.dsc + 400);
      double hn = 0.0;
      for (int j = 0; j < m; ++j) {
        zd* vj = K + (long long)j * n2;
        zd* wv = K + (long long)(j + 1) * n2;
        TRY(op_phi(c, vj, wv, p, true));  // Krylov vectors of a Hermitian start stay Hermitian
        ++inf.n_phi;
        if (n2 <= 4096) {
          // small systems: the whole CGS2 step in one workgroup (launch latency dominates here)
          TRY(cgs2_small(K, n2, j + 1, wv, n2, X->hd, m, subd, c.st));
        } else {
          zd* h1 = c.dsc + 8;
          zd* h2 = c.dsc + 80;
          TRY(multi_dot(K, n2, j + 1, wv, n2, h1, (zd*)c.dscr, c.st));
          TRY(multi_axpy(K, n2, j + 1, h1, wv, n2, 1, -1.0, c.st));
          TRY(multi_dot(K, n2, j + 1, wv, n2, h2, (zd*)c.dscr, c.st));
          TRY(multi_axpy(K, n2, j + 1, h2, wv, n2, 1, -1.0, c.st));
          TRY(nrm2(wv, n2, (double*)(c.dsc + 4), c.dscr, c.st));
          TRY(scale_by_inv_hcol(wv, n2, (const double*)(c.dsc + 4), h1, h2, X->hd, m, j, subd, c.st));
        }
        k = j + 1;
        bool check = (k >= 3 && (k % 2 == 1)) || k == m;
        if (check) {
          // Ritz pair nearest 1; the estimate also carries the pair's residual inside the
          // Krylov space, which is zero for an exact eigenpair of H
          TRY(ritz_near_dev(X, X->hd, m, k, subd, theta, ysel, rin, hn));
          k_ritz = k;
          est = std::sqrt(std::norm(theta - 1.0) + rin * rin + hn * hn * std::norm(ysel[k - 1]));
          if (c_scale * est <= std::max(0.25 * tol, eps_floor) || hn == 0.0) break;
        }
        if (deadline > 0 && now_s() > deadline) break;
      }
      // the cycle may end (time limit) at a step without a Ritz evaluation: evaluate it for this k
      if (k_ritz != k) TRY(ritz_near_dev(X, X->hd, m, k, subd, theta, ysel, rin, hn));
      // Ritz vector xi = V_k y (y left on the device by the last evaluation)
      TRY(multi_axpy(K, n2, k, X->Yv + 1, X->xiB, n2, 0, 1.0, c.st));
      // the fixed point xi = -S(rho_inf) is Hermitian: keep the restart vector Hermitian
      TRY(hermitize(X->xiB, n, 0, nullptr, c.dscr, c.st));
      // rho = -S^{-1} xi, hermitised and normalised (the sign cancels in the normalisation)
      TRY(op_sinv(c, X->xiB, X->rhoB, cplx(0, 0), p, false));
      cplx trb;
      TRY(finish_state(X, X->rhoB, &colsum, &mx, &fro, &trb));
      ++inf.n_restarts;
      if (log_on())
        std::fprintf(stderr, "[lindx] steady state restart %d: residual bound %.3e after %d Phi\n", inf.n_restarts,
                     colsum, inf.n_phi);
      double xn = 0;
      TRY(op_nrm(c, X->xiB, &xn));
      if (std::abs(trb) > 0) c_scale = std::sqrt((double)n) * xn / std::abs(trb);
      best_is_last = colsum < best;
      if (colsum < best) {
        best = colsum;
        best_max = mx;
        TRY(copy(X->rhoB, (zd*)rho_out, n2, c.st));
      }
      if (colsum <= tol) { converged = true; break; }
      if (c_scale * est <= std::max(0.25 * tol, eps_floor) || p != PREC_F64) { floor_hit = true; break; }
      // a residual that goes up again three times before the best one halves marks the rounding
      // floor of the restarted iteration (slow convergence keeps decreasing): refinement on the FP64
      // residual takes over
      if (colsum < 0.5 * gain_ref) {
        gain_ref = colsum;
        restart_stall = 0;
      } else if (pass == 0 && p == PREC_F64 && colsum >= 0.95 * prev_colsum && ++restart_stall >= 3) {
        floor_hit = true;
        oscillation_stop = true;
        break;
      }
      prev_colsum = colsum;
      if (deadline > 0 && now_s() > deadline) break;
      // restart from xi
      TRY(copy(X->xiB, K, n2, c.st));
      TRY(op_nrm(c, K, &xn));
      TRY(scale_by_inv(K, n2, (const double*)c.dsc, c.st));
    }
    // FP64 iterative refinement: (I - Phi_p) zeta = L rho, rho <- rho - S_p^{-1} zeta
    if (!converged && (floor_hit || true)) {
      // continue from the best state; when it is the last one evaluated, rhoB and its residual in
      // resB are already in place
      if (!best_is_last) {
        TRY(copy((const zd*)rho_out, X->rhoB, n2, c.st));
        TRY(finish_state(X, X->rhoB, &colsum, &mx, &fro, nullptr));
      } else {
        colsum = best;
      }
      double prev = colsum;
      int stagn = 0;
      const double floor_inner = (p == PREC_F64) ? 1e-13 : (p == PREC_F32 ? 3e-6 : 1e-4);
      std::function<int(const zd*, zd*)> Aop = [&](const zd* in, zd* out) -> int {
        int rc = op_phi(c, in, out, p, true);  // GMRES on a Hermitian right-hand side
        if (rc) return rc;
        ++inf.n_phi;
        return axpby(zmk(1, 0), in, zmk(-1, 0), out, n2, c.st) ? LIND_EDEVICE : 0;
      };
      // inner solves: GMRES(m) first; once one misses its tolerance the map is treated as strongly
      // non-normal and the remaining solves use one long cycle (basis in HBM)
      int m_ref = m;
      bool long_mode = false;
      for (int it = 0; it < c.opts.refine_max && !converged; ++it) {
        if (deadline > 0 && now_s() > deadline) break;
        double rtol = std::min(0.1, std::max(floor_inner, 0.05 * tol / std::max(colsum, 1e-300)));
        GmresResult gr;
        int grc = gmres_rec(X, Aop, nullptr, X->resB, X->zetaB, true, m_ref, 0, 2, rtol, 0.0, c.rec, gr, deadline);
        if (grc) {
          if (long_mode) release_long_basis(c);
          return grc;
        }
        inf.n_inner += gr.iters;
        // a long cycle only when the recurrence itself missed the target (a strongly non-normal
        // map); a recurrence that met it with the true residual short of it has reached the
        // rounding floor of the reduced-precision map, which more steps do not lower
        if (!gr.converged && !gr.stagnated && !gr.est_hit && !long_mode) {
          long_mode = true;
          m_ref = long_cycle_len(c, 256, false);
        }
        TRY(op_sinv(c, X->zetaB, X->delB, cplx(0, 0), p, false));
        TRY(axpby(zmk(-1, 0), X->delB, zmk(1, 0), X->rhoB, n2, c.st));
        TRY(finish_state(X, X->rhoB, &colsum, &mx, &fro, nullptr));
        ++inf.n_refine;
        if (colsum < best) {
          best = colsum;
          best_max = mx;
          TRY(copy(X->rhoB, (zd*)rho_out, n2, c.st));
        }
        if (colsum <= tol) { converged = true; break; }
        if (colsum > 0.5 * prev) { if (++stagn >= 2) break; } else stagn = 0;
        prev = colsum;
      }
      if (long_mode) release_long_basis(c);
    }
    if (converged || !oscillation_stop || restarts_left <= 0) break;
    if (deadline > 0 && now_s() > deadline) break;
    TRY(copy((const zd*)rho_out, X->rhoB, n2, c.st));
    rho_is_identity = false;
    TRY(start_from_rho());
    best_is_last = false;
  }
  TRY(c.sync());
  inf.resid_trace = best;
  inf.resid_max = best_max;
  inf.err_est = best;
  inf.t_solve_s = now_s() - t0;
  if (info) *info = inf;
  if (!converged) return c.fail(LIND_ENOCONV, "steady state: tolerance not reached (best iterate returned)");
  return LIND_OK;
}
