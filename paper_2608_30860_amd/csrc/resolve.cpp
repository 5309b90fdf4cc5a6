// Resolvent of the Lindbladian and the implicit Euler step.
//
// resolve: (lambda - L) X = B for Re(lambda) > 0 by GMRES right-preconditioned with the no-jump
// resolvent R^S_lambda = (lambda - S)^{-1} (eq. right-precond-identity: (lambda - L) R^S_lambda =
// Id - K R^S_lambda, whose norm the contraction theorem keeps below 1, so the inner iteration
// converges geometrically, Remark "Geometric convergence of the preconditioned GMRES").  The
// operator is applied in FP64; the preconditioner in the context precision.
//
// ie: rho_{k+1} = (I - dt L)^{-1} rho_k = lambda (lambda - L)^{-1} rho_k with lambda = 1/dt
// (eq. resolvent of the implicit-solver section), each step warm-started from rho_k, the recycled
// GMRES subspace threaded through all steps (one operator throughout).
#include <cmath>
#include <cstdio>
#include <cstring>
#include "ctx.hpp"

using namespace lindx;

#define TRY(x)                                           \
  do {                                                   \
    int rc__ = (x);                                      \
    if (rc__) return rc__ < 0 ? rc__ : LIND_EDEVICE;     \
  } while (0)

namespace {

constexpr int kResM = 40;  // GMRES cycle length
constexpr int kResK = 20;  // recycled harmonic Ritz vectors

struct ResolveOps {
  Ctx* c;
  cplx lam;
  long long n_prec = 0;
  // out = lambda x - L(x)
  int A(const zd* x, zd* out) {
    TRY(op_apply(*c, x, out, false));
    return axpby(zmk(lam.real(), lam.imag()), x, zmk(-1, 0), out, c->n2, c->st) ? LIND_EDEVICE : 0;
  }
  // out = R^S_lambda(x) = -(S - lambda)^{-1} x
  int P(const zd* x, zd* out) {
    ++n_prec;
    TRY(op_sinv(*c, x, out, lam, c->prec, false));
    return axpby(zmk(0, 0), out, zmk(-1, 0), out, c->n2, c->st) ? LIND_EDEVICE : 0;
  }
};

// one solve (lambda - L) x = b to relative residual tol; x holds the start guess when warm.
// Reports the true final residual (relative to ||b||) in *rel and its max-norm in *rmax.
int solve(lind_ctx* X, ResolveOps& ops, const zd* b, zd* x, bool warm, double tol, double deadline,
          GmresResult& gr, double* rel, double* rmax) {
  Ctx& c = X->c;
  std::function<int(const zd*, zd*)> Aop = [&](const zd* in, zd* out) { return ops.A(in, out); };
  std::function<int(const zd*, zd*)> Pop = [&](const zd* in, zd* out) { return ops.P(in, out); };
  TRY(gmres_rec(X, Aop, &Pop, b, x, !warm, kResM, kResK, 100, tol, 0.0, c.rec, gr, deadline));
  // true residual
  TRY(ops.A(x, X->resB));
  TRY(axpby(zmk(1, 0), b, zmk(-1, 0), X->resB, c.n2, c.st));
  double nr[4], nb = 0;
  TRY(op_norms(c, X->resB, nr));
  TRY(op_nrm(c, b, &nb));
  *rel = nr[0] / std::max(nb, 1e-300);
  *rmax = nr[1];
  return 0;
}

}  // namespace

extern "C" int lind_resolve(lind_ctx* ctx, double lam_re, double lam_im, const void* B, void* Xout, double tol,
                            lind_info* info) {
  if (!ctx || !B || !Xout || !(tol > 0) || !std::isfinite(lam_re) || !std::isfinite(lam_im)) return LIND_EINVAL;
  lind_ctx* X = ctx;
  Ctx& c = X->c;
  if (!(lam_re > 0)) return c.fail(LIND_EINVAL, "resolve: Re(lambda) must be positive");
  if (B == Xout) return c.fail(LIND_EINVAL, "resolve: B and X may not alias");
  const double t0 = now_s();
  const double deadline = c.opts.time_limit_s > 0 ? t0 + c.opts.time_limit_s : 0.0;
  TRY(ensure_solver_bufs(X));
  lind_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.kappa_U = c.kappa;
  inf.t_factor_s = c.t_factor;
  inf.route_used = c.route;
  ResolveOps ops;
  ops.c = &c;
  ops.lam = cplx(lam_re, lam_im);
  c.rec.reset();
  GmresResult gr;
  double rel = 0, rmax = 0;
  int rc = solve(X, ops, (const zd*)B, (zd*)Xout, false, tol, deadline, gr, &rel, &rmax);
  c.rec.reset();
  TRY(rc);
  TRY(c.sync());
  inf.n_inner = gr.iters;
  inf.n_phi = (int)ops.n_prec;
  inf.n_restarts = gr.cycles;
  inf.err_est = rel;
  inf.resid_max = rmax;
  inf.t_solve_s = now_s() - t0;
  if (info) *info = inf;
  if (!(rel <= tol)) {
    char msg[128];
    std::snprintf(msg, sizeof msg, "resolve: relative residual %.2e above tol after %d iterations", rel, gr.iters);
    return c.fail(LIND_ENOCONV, msg);
  }
  return LIND_OK;
}

extern "C" int lind_ie(lind_ctx* ctx, double dt, int steps, const void* rho0, void* rho_out, double tol,
                       lind_info* info) {
  if (!ctx || !rho0 || !rho_out || !(tol > 0) || !(dt > 0) || !std::isfinite(dt) || steps < 0) return LIND_EINVAL;
  lind_ctx* X = ctx;
  Ctx& c = X->c;
  const long long n2 = c.n2;
  const double t0 = now_s();
  const double deadline = c.opts.time_limit_s > 0 ? t0 + c.opts.time_limit_s : 0.0;
  TRY(ensure_solver_bufs(X));
  lind_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.kappa_U = c.kappa;
  inf.t_factor_s = c.t_factor;
  inf.route_used = c.route;
  ResolveOps ops;
  ops.c = &c;
  ops.lam = cplx(1.0 / dt, 0.0);
  zd* state = (zd*)rho_out;
  if (rho0 != rho_out) TRY(copy((const zd*)rho0, state, n2, c.st));
  c.rec.reset();
  double worst = 0, worst_max = 0;
  int status = LIND_OK;
  for (int k = 0; k < steps; ++k) {
    // b = lambda rho_k; x starts at rho_k
    TRY(copy(state, X->zetaB, n2, c.st));
    TRY(axpby(zmk(0, 0), X->zetaB, zmk(1.0 / dt, 0), X->zetaB, n2, c.st));
    GmresResult gr;
    double rel = 0, rmax = 0;
    int rc = solve(X, ops, X->zetaB, state, true, tol, deadline, gr, &rel, &rmax);
    if (rc) { c.rec.reset(); return rc; }
    inf.n_inner += gr.iters;
    ++inf.n_restarts;
    worst = std::max(worst, rel);
    worst_max = std::max(worst_max, rmax);
    if (!(rel <= tol)) { status = LIND_ENOCONV; break; }
    if (deadline > 0 && now_s() > deadline && k + 1 < steps) { status = LIND_ENOCONV; break; }
  }
  c.rec.reset();
  TRY(c.sync());
  inf.n_phi = (int)ops.n_prec;
  inf.err_est = worst;
  inf.resid_max = worst_max;
  inf.t_solve_s = now_s() - t0;
  if (info) *info = inf;
  if (status) return c.fail(status, "ie: a step missed the tolerance or the time limit was hit");
  return LIND_OK;
}
