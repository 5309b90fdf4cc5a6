// Low-lying spectrum (Algorithm "Low-lying spectrum via shift-invert Arnoldi") and steady-state
// gradients (Remark "Differentiating the steady state").
//
// eigs: Krylov-Schur Arnoldi on OP = (mu - L~_eta)^{-1}, L~_eta = L + eta |I><I|.  Each OP
// application is a right-preconditioned recycled GMRES solve of (mu - L~_eta) x = b with the deflated
// no-jump preconditioner P_mu (Algorithm "Precond": Z = R^S_mu(X), W = R^S_mu(I) precomputed,
// P = Z + eta Tr(Z) / (1 - eta Tr W) W, eq. ShermanMorr).  Thick restart keeps an orthonormal basis
// of the invariant subspace of the p dominant Ritz values; eigenvalues of L are mu - 1/nu.
//
// grad: steady state rho, then the adjoint system (L~_eta)^* w = O - <O> I solved by GMRES with
// the adjoint preconditioner (same factorisation: (S^*)^{-1} swaps U and V and conjugates the
// eigenvalues), then g_H = i[rho, w], g_Lj = L_j {rho, w} - 2 w L_j rho.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include "ctx.hpp"

using namespace lindx;

#define TRY(x)                                           \
  do {                                                   \
    int rc__ = (x);                                      \
    if (rc__) return rc__ < 0 ? rc__ : LIND_EDEVICE;     \
  } while (0)

namespace {

constexpr int kInnerM = 40;  // inner GMRES cycle length
constexpr int kInnerK = 20;  // recycled harmonic Ritz vectors

// A(x) = mu x - L(x) - eta Tr(x) I   (or the adjoint: conj(mu) x - L*(x) - eta Tr(x) I)
int apply_shifted_deflated(Ctx& c, const zd* x, zd* out, cplx mu, double eta, bool adjoint) {
  if (adjoint) TRY(op_apply_adj(c, x, out));
  else TRY(op_apply(c, x, out, false));
  cplx m = adjoint ? std::conj(mu) : mu;
  TRY(axpby(zmk(m.real(), m.imag()), x, zmk(-1, 0), out, c.n2, c.st));
  // - eta Tr(x) I with the trace kept on the device (no host round trip per Krylov step)
  TRY(add_identity_trace(out, c.n, x, zmk(-eta, 0), c.dsc + 980, c.st));
  return 0;
}

struct Precond {
  cplx mu;
  double eta;
  bool adjoint;
  zd* W = nullptr;  // R^S_mu(I) (or its adjoint)
  cplx trW;
};

// Z = R_mu(X) = -(S - mu)^{-1} X (adjoint: -(S* - conj(mu))^{-1} X), then the rank-one correction
int apply_precond(Ctx& c, const Precond& P, const zd* x, zd* out, int prec) {
  TRY(op_sinv(c, x, out, P.mu, prec, P.adjoint));
  TRY(axpby(zmk(0, 0), out, zmk(-1, 0), out, c.n2, c.st));
  // Z + eta Tr(Z) / (1 - eta Tr W) W with Tr(Z) and the coefficient on the device
  TRY(sherman_morrison(out, P.W, c.n, zmk(P.eta, 0), zmk(P.trW.real(), P.trW.imag()), c.dsc + 984, c.dscr, c.st));
  return 0;
}

int make_precond(lind_ctx* X, Precond& P, cplx mu, double eta, bool adjoint) {
  Ctx& c = X->c;
  P.mu = mu;
  P.eta = eta;
  P.adjoint = adjoint;
  if (!c.Wmu) TRY(c.alloc(&c.Wmu, c.n2));
  P.W = c.Wmu;
  TRY(fill_zero(X->delB, c.n2 * (long long)sizeof(zd), c.st));
  TRY(add_identity(X->delB, c.n, zmk(1, 0), c.st));
  TRY(op_sinv(c, X->delB, P.W, mu, PREC_F64, adjoint));
  TRY(axpby(zmk(0, 0), P.W, zmk(-1, 0), P.W, c.n2, c.st));
  TRY(op_trace(c, P.W, &P.trW));
  if (std::abs(1.0 - eta * P.trW) < 1e-12) return c.fail(LIND_ESINGULAR, "1 - eta Tr W vanishes (eq. ShermanMorr)");
  return 0;
}

// orthonormalise the columns of Y (m x p, row-major ld = p) in place (modified Gram-Schmidt, twice)
void mgs(std::vector<cplx>& Y, int m, int p) {
  for (int j = 0; j < p; ++j) {
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        cplx h = 0;
        for (int r = 0; r < m; ++r) h += std::conj(Y[(size_t)r * p + i]) * Y[(size_t)r * p + j];
        for (int r = 0; r < m; ++r) Y[(size_t)r * p + j] -= h * Y[(size_t)r * p + i];
      }
    double nrm = 0;
    for (int r = 0; r < m; ++r) nrm += std::norm(Y[(size_t)r * p + j]);
    nrm = std::sqrt(nrm);
    for (int r = 0; r < m; ++r) Y[(size_t)r * p + j] /= nrm;
  }
}

__global__ void k_conj_transpose(const zd* X, zd* Y, int n) {
  long long tot = (long long)n * n;
  long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride) {
    long long i = t / n, j = t % n;
    Y[j * n + i] = zconj(X[t]);
  }
}

}  // namespace

// ---------------------------------------------------------------------------------------------
extern "C" int lind_eigs(lind_ctx* ctx, int k, double mu_re, double mu_im, double tol, void* evals_out, void* evecs_out,
                         lind_info* info) {
  if (!ctx || !evals_out || !(tol > 0) || !std::isfinite(mu_re) || !std::isfinite(mu_im)) return LIND_EINVAL;
  lind_ctx* X = ctx;
  Ctx& c = X->c;
  const int m = c.opts.m;
  if (k < 1 || k > m - 3) return c.fail(LIND_EINVAL, "need 1 <= k <= m - 3");
  const int n = c.n;
  const long long n2 = c.n2;
  const double t0 = now_s();
  const double deadline = c.opts.time_limit_s > 0 ? t0 + c.opts.time_limit_s : 0.0;
  const cplx mu(mu_re, mu_im);
  const double eta = c.opts.eta;
  int p = c.opts.p > 0 ? c.opts.p : std::max(k + 3, m / 2);
  p = std::min(p, m - 2);
  TRY(ensure_solver_bufs(X));
  TRY(c.ensure_krylov(1, m + 1 + p));
  zd* Q = c.K1;
  lind_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.kappa_U = c.kappa;
  inf.t_factor_s = c.t_factor;
  inf.route_used = c.route;

  Precond P;
  TRY(make_precond(X, P, mu, eta, false));
  std::function<int(const zd*, zd*)> Aop = [&](const zd* in, zd* out) -> int {
    return apply_shifted_deflated(c, in, out, mu, eta, false);
  };
  std::function<int(const zd*, zd*)> Pop = [&](const zd* in, zd* out) -> int {
    ++inf.n_phi;
    return apply_precond(c, P, in, out, c.prec);
  };
  // inner solves: recycled GMRES(40) keeping 20 harmonic Ritz vectors, threaded through every
  // application of OP (same operator and preconditioner throughout); the inner tolerance follows
  // the outer one (the eigen-residual of a Ritz pair is about |lambda| times the inner residual)
  const double rtol_in = std::min(1e-8, std::max(1e-12, 0.1 * tol));
  c.rec.reset();
  // reduced-precision contexts (eigen route): each solve is iterative refinement on the FP64
  // residual, the corrections from recycled GMRES on the operator with BF16x3 products and the
  // context's preconditioner, a consistent low-precision pair; the FP64 operator is applied once per
  // refinement step instead of once per Krylov step
  // The low-precision operator must be accurate on the scale of the shifted spectrum: a truncated
  // Fock ladder with ||L|| ~ n^2 and wanted eigenvalues near 1e-3 is not (BF16x3 errors of
  // ~1e-5 ||L|| exceed |mu - lambda|).  A first refinement step that does not halve the residual
  // switches the call back to the FP64 operator in every Krylov step.
  bool mixed = c.prec != PREC_F64 && c.route == LIND_ROUTE_EIG && c.d > 0;
  std::function<int(const zd*, zd*)> Alow = [&](const zd* in, zd* out) -> int {
    TRY(op_apply_p4(c, in, out));
    TRY(axpby(zmk(mu.real(), mu.imag()), in, zmk(-1, 0), out, c.n2, c.st));
    TRY(add_identity_trace(out, c.n, in, zmk(-eta, 0), c.dsc + 980, c.st));
    return 0;
  };
  auto OP = [&](const zd* b, zd* x) -> int {
    GmresResult gr;
    if (!mixed) {
      TRY(gmres_rec(X, Aop, &Pop, b, x, true, kInnerM, kInnerK, 60, rtol_in, 0.0, c.rec, gr, deadline));
      inf.n_inner += gr.iters;
      return 0;
    }
    double bn = 0;
    TRY(op_nrm(c, b, &bn));
    TRY(fill_zero(x, c.n2 * (long long)sizeof(zd), c.st));
    TRY(copy(b, X->resB, c.n2, c.st));  // r = b - A x with x = 0
    double rn = bn, prev = 1e300;
    for (int it = 0; it < 8 && rn > rtol_in * bn; ++it) {
      // correction to 1e-3 of the current residual (the BF16x3 operator is accurate to ~1e-5)
      TRY(gmres_rec(X, Alow, &Pop, X->resB, X->delB, true, kInnerM, kInnerK, 60, 1e-3, 0.0, c.rec, gr, deadline));
      inf.n_inner += gr.iters;
      TRY(axpby(zmk(1, 0), X->delB, zmk(1, 0), x, c.n2, c.st));
      TRY(Aop(x, X->resB));
      TRY(axpby(zmk(1, 0), b, zmk(-1, 0), X->resB, c.n2, c.st));
      TRY(op_nrm(c, X->resB, &rn));
      if (it == 0 && !(rn <= 0.5 * bn)) {
        // the low-precision operator is too coarse for this shift: FP64 operator from here on
        mixed = false;
        c.rec.reset();  // the recycle space belonged to the low-precision operator
        TRY(gmres_rec(X, Aop, &Pop, b, x, true, kInnerM, kInnerK, 60, rtol_in, 0.0, c.rec, gr, deadline));
        inf.n_inner += gr.iters;
        return 0;
      }
      if (rn > 0.5 * prev) break;  // refinement no longer converging: keep the best so far
      prev = rn;
    }
    return 0;
  };

  // start vector: seeded random complex (non-Hermitian) matrix
  {
    std::vector<zd> v0((size_t)n2);
    std::mt19937_64 rng(20260801ULL);
    std::normal_distribution<double> nd;
    for (auto& z : v0) z = zmk(nd(rng), nd(rng));
    if (hipMemcpyAsync(Q, v0.data(), sizeof(zd) * n2, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
    TRY(c.sync());
    double nr;
    TRY(op_nrm(c, Q, &nr));
    TRY(scale_by_inv(Q, n2, (const double*)c.dsc, c.st));
  }
  std::vector<cplx> Hk((size_t)(m + 1) * m, cplx(0));
  int j0 = 0;
  bool converged = false;
  std::vector<cplx> lam_out;
  std::vector<int> idx_out;
  std::vector<cplx> w, Y;
  double worst = 0;
  for (int rs = 0; rs < c.opts.max_restarts; ++rs) {
    ++inf.n_restarts;
    for (int j = j0; j < m; ++j) {
      zd* qj = Q + (long long)j * n2;
      zd* wv = Q + (long long)(j + 1) * n2;
      TRY(OP(qj, wv));
      zd* h1 = c.dsc + 8;
      zd* h2 = c.dsc + 80;
      TRY(multi_dot(Q, n2, j + 1, wv, n2, h1, (zd*)c.dscr, c.st));
      TRY(multi_axpy(Q, n2, j + 1, h1, wv, n2, 1, -1.0, c.st));
      TRY(multi_dot(Q, n2, j + 1, wv, n2, h2, (zd*)c.dscr, c.st));
      TRY(multi_axpy(Q, n2, j + 1, h2, wv, n2, 1, -1.0, c.st));
      TRY(nrm2(wv, n2, (double*)(c.dsc + 4), c.dscr, c.st));
      TRY(c.fetch(c.dsc, sizeof(zd) * 160));
      double hn = ((const double*)(c.hsc + 4))[0];
      for (int i = 0; i <= j; ++i)
        Hk[(size_t)i * m + j] += cplx(c.hsc[8 + i].x + c.hsc[80 + i].x, c.hsc[8 + i].y + c.hsc[80 + i].y);
      Hk[(size_t)(j + 1) * m + j] = hn;
      if (hn > 0) TRY(scale_by_inv(wv, n2, (const double*)(c.dsc + 4), c.st));
      // (the time limit is checked between restarts: a thick restart needs the whole m-step basis)
    }
    // Ritz pairs of the m x m projected matrix
    int rc = small_eig_host(X, Hk, m, m, w, Y);
    if (rc && rc != LIND_ENOCONV) return rc;
    std::vector<int> order(m);
    for (int i = 0; i < m; ++i) order[i] = i;
    std::sort(order.begin(), order.end(), [&](int a, int b) { return std::abs(w[a]) > std::abs(w[b]); });
    // verify the k dominant pairs on the true Lindbladian
    worst = 0;
    lam_out.clear();
    idx_out.clear();
    int nconv = 0;
    for (int t = 0; t < k; ++t) {
      int i = order[t];
      cplx nu = w[i];
      cplx lam = mu - 1.0 / nu;
      // Ritz vector v = Q_m y into xiB
      std::vector<cplx> y(m);
      for (int r = 0; r < m; ++r) y[r] = Y[(size_t)r * m + i];
      TRY(upload_vec(X, y.data(), m, X->yv));
      TRY(multi_axpy(Q, n2, m, X->yv, X->xiB, n2, 0, 1.0, c.st));
      TRY(op_apply(c, X->xiB, X->resB, false));
      TRY(axpby(zmk(-lam.real(), -lam.imag()), X->xiB, zmk(1, 0), X->resB, n2, c.st));
      double nr[4], nv[4];
      TRY(op_norms(c, X->resB, nr));
      TRY(op_norms(c, X->xiB, nv));
      double res = nr[1] / std::max(nv[0], 1e-300);  // max-norm residual of the unit-norm vector
      double rel = res / std::max(1.0, std::abs(lam));
      worst = std::max(worst, rel);
      if (rel <= tol) ++nconv;
      lam_out.push_back(lam);
      idx_out.push_back(i);
    }
    if (log_on())
      std::fprintf(stderr, "[lindx] eigs restart %d: %d of %d pairs converged, worst %.2e, %d inner steps, %.1f s\n",
                   inf.n_restarts, nconv, k, worst, inf.n_inner, now_s() - t0);
    if (nconv == k) { converged = true; break; }
    if (deadline > 0 && now_s() > deadline) break;
    if (rs + 1 >= c.opts.max_restarts) break;
    // thick restart: orthonormal basis of the p dominant Ritz vectors
    std::vector<cplx> Yp((size_t)m * p);
    for (int r = 0; r < m; ++r)
      for (int t = 0; t < p; ++t) Yp[(size_t)r * p + t] = Y[(size_t)r * m + order[t]];
    mgs(Yp, m, p);
    // new basis vectors into the spare slots m+1 .. m+p, then move to 0 .. p-1; q_m -> slot p
    for (int t = 0; t < p; ++t) {
      std::vector<cplx> y(m);
      for (int r = 0; r < m; ++r) y[r] = Yp[(size_t)r * p + t];
      TRY(upload_vec(X, y.data(), m, X->yv));
      TRY(multi_axpy(Q, n2, m, X->yv, Q + (long long)(m + 1 + t) * n2, n2, 0, 1.0, c.st));
    }
    TRY(copy(Q + (long long)m * n2, Q + (long long)p * n2, n2, c.st));
    for (int t = 0; t < p; ++t) TRY(copy(Q + (long long)(m + 1 + t) * n2, Q + (long long)t * n2, n2, c.st));
    // projected matrix: S = Yp^H H Yp, last row b^T Yp
    std::vector<cplx> HY((size_t)m * p, cplx(0)), Hn((size_t)(m + 1) * m, cplx(0));
    for (int r = 0; r < m; ++r)
      for (int t = 0; t < p; ++t) {
        cplx s = 0;
        for (int q = 0; q < m; ++q) s += Hk[(size_t)r * m + q] * Yp[(size_t)q * p + t];
        HY[(size_t)r * p + t] = s;
      }
    for (int a = 0; a < p; ++a)
      for (int t = 0; t < p; ++t) {
        cplx s = 0;
        for (int r = 0; r < m; ++r) s += std::conj(Yp[(size_t)r * p + a]) * HY[(size_t)r * p + t];
        Hn[(size_t)a * m + t] = s;
      }
    for (int t = 0; t < p; ++t) {
      cplx s = 0;
      for (int q = 0; q < m; ++q) s += Hk[(size_t)m * m + q] * Yp[(size_t)q * p + t];
      Hn[(size_t)p * m + t] = s;
    }
    Hk.swap(Hn);
    j0 = p;
  }
  // pack the k pairs, sorted by |lambda| ascending (ties: Im ascending); conjugate partners
  // (L(X^H) = L(X)^H) are added for non-real eigenvalues whose partner is missing
  struct Pair { cplx lam; int ritz; bool conj_of; };
  std::vector<Pair> pairs;
  for (size_t t = 0; t < lam_out.size(); ++t) pairs.push_back({lam_out[t], idx_out[t], false});
  for (size_t t = 0; t < lam_out.size(); ++t) {
    cplx l = lam_out[t];
    if (std::fabs(l.imag()) <= 1e-10 * std::max(1.0, std::abs(l))) {
      // real eigenvalue: X^H is an eigenvector too; if it is independent of X the eigenvalue is
      // (at least) double and a single Krylov sequence only holds one copy -- add the partner
      std::vector<cplx> y(m);
      for (int r = 0; r < m; ++r) y[r] = Y[(size_t)r * m + idx_out[t]];
      TRY(upload_vec(X, y.data(), m, X->yv));
      TRY(multi_axpy(Q, n2, m, X->yv, X->xiB, n2, 0, 1.0, c.st));
      double nx;
      TRY(op_nrm(c, X->xiB, &nx));
      TRY(scale_by_inv(X->xiB, n2, (const double*)c.dsc, c.st));
      hipLaunchKernelGGL(k_conj_transpose, dim3(1024), dim3(256), 0, c.st, X->xiB, X->zetaB, n);
      TRY(multi_dot(X->xiB, n2, 1, X->zetaB, n2, c.dsc + 200, (zd*)c.dscr, c.st));
      TRY(c.fetch(c.dsc + 200, sizeof(zd)));
      double ov = std::hypot(c.hsc[0].x, c.hsc[0].y);
      int same = 0;
      for (auto& q : pairs) same += std::abs(q.lam - l) <= 1e-8 * std::max(1.0, std::abs(l));
      if (ov < 1.0 - 1e-6 && same < 2) pairs.push_back({l, idx_out[t], true});
      continue;
    }
    bool have = false;
    for (auto& q : pairs) have |= std::abs(q.lam - std::conj(l)) <= 1e-8 * std::max(1.0, std::abs(l));
    if (!have) pairs.push_back({std::conj(l), idx_out[t], true});
  }
  std::stable_sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
    double da = std::abs(a.lam), db = std::abs(b.lam);
    if (std::fabs(da - db) > 1e-12 * std::max(1.0, da)) return da < db;
    return a.lam.imag() < b.lam.imag();
  });
  double* ev = (double*)evals_out;
  for (int t = 0; t < k; ++t) {
    ev[2 * t] = pairs[t].lam.real();
    ev[2 * t + 1] = pairs[t].lam.imag();
    if (evecs_out) {
      zd* dst = (zd*)evecs_out + (long long)t * n2;
      std::vector<cplx> y(m);
      for (int r = 0; r < m; ++r) y[r] = Y[(size_t)r * m + pairs[t].ritz];
      TRY(upload_vec(X, y.data(), m, X->yv));
      TRY(multi_axpy(Q, n2, m, X->yv, X->xiB, n2, 0, 1.0, c.st));
      if (pairs[t].conj_of) {
        hipLaunchKernelGGL(k_conj_transpose, dim3(1024), dim3(256), 0, c.st, X->xiB, dst, n);
      } else {
        TRY(copy(X->xiB, dst, n2, c.st));
      }
      // unit Frobenius norm, largest-modulus entry real positive
      std::vector<zd> hv((size_t)n2);
      if (hipMemcpyAsync(hv.data(), dst, sizeof(zd) * n2, hipMemcpyDeviceToHost, c.st) != hipSuccess) return LIND_EDEVICE;
      TRY(c.sync());
      double nrm = 0, amax = -1;
      long long imax = 0;
      for (long long q = 0; q < n2; ++q) {
        double a = zabs2(hv[q]);
        nrm += a;
        if (a > amax) { amax = a; imax = q; }
      }
      nrm = std::sqrt(nrm);
      cplx ph(hv[imax].x, hv[imax].y);
      cplx f = std::conj(ph) / (std::abs(ph) * nrm);
      TRY(axpby(zmk(0, 0), dst, zmk(f.real(), f.imag()), dst, n2, c.st));
    }
  }
  TRY(c.sync());
  inf.err_est = worst;
  inf.resid_max = worst;
  inf.t_solve_s = now_s() - t0;
  if (info) *info = inf;
  if (!converged) return c.fail(LIND_ENOCONV, "eigs: tolerance not reached");
  return LIND_OK;
}

// ---------------------------------------------------------------------------------------------
extern "C" int lind_steady_grad(lind_ctx* ctx, const void* O, double tol, double* expval, void* grad_H, void* grad_L,
                                void* rho_out, lind_info* info) {
  if (!ctx || !O || !expval || !(tol > 0)) return LIND_EINVAL;
  lind_ctx* X = ctx;
  Ctx& c = X->c;
  const int n = c.n, d = c.d;
  const long long n2 = c.n2;
  const cplx one(1, 0);
  const double t0 = now_s();
  TRY(ensure_solver_bufs(X));
  zd* rho = nullptr;
  zd* wadj = nullptr;
  zd* rhs = nullptr;
  if (!c.Wmu) TRY(c.alloc(&c.Wmu, n2));
  // dedicated buffers (allocated once per context)
  static_assert(sizeof(zd) == 16, "complex128");
  TRY(c.alloc(&rho, n2));
  TRY(c.alloc(&wadj, n2));
  TRY(c.alloc(&rhs, n2));
  lind_info inf;
  std::memset(&inf, 0, sizeof(inf));
  int rc = steady_state_impl(X, tol, nullptr, rho, &inf);
  int status = LIND_OK;
  if (rc == LIND_ENOCONV) {
    if (inf.resid_trace > 100 * tol) status = LIND_ENOCONV;
  } else if (rc) {
    return rc;
  }
  // <O> = Re Tr(O rho) = Re sum_ij conj(O_ij) rho_ij for Hermitian rho
  TRY(multi_dot((const zd*)O, n2, 1, rho, n2, c.dsc + 200, (zd*)c.dscr, c.st));
  TRY(c.fetch(c.dsc + 200, sizeof(zd)));
  const double J = c.hsc[0].x;
  *expval = J;
  // adjoint system: -(L~_eta)^* w = -(O - J I), right preconditioner for the adjoint no-jump part
  TRY(copy((const zd*)O, rhs, n2, c.st));
  TRY(add_identity(rhs, n, zmk(-J, 0), c.st));
  TRY(axpby(zmk(0, 0), rhs, zmk(-1, 0), rhs, n2, c.st));
  const double eta = c.opts.eta;
  Precond P;
  TRY(make_precond(X, P, cplx(0, 0), eta, true));
  std::function<int(const zd*, zd*)> Aop = [&](const zd* in, zd* out) -> int {
    return apply_shifted_deflated(c, in, out, cplx(0, 0), eta, true);
  };
  std::function<int(const zd*, zd*)> Pop = [&](const zd* in, zd* out) -> int {
    ++inf.n_phi;
    return apply_precond(c, P, in, out, c.prec);
  };
  // recycled GMRES(40) first; if it has not converged after a dozen cycles the preconditioned adjoint
  // is strongly non-normal (long chains of levels), and one long cycle (up to kMaxLong steps, basis in
  // HBM) continues from the current iterate
  const double rtol_adj = std::min(1e-9, std::max(1e-13, 0.01 * tol));
  GmresResult gr;
  c.rec.reset();
  TRY(gmres_rec(X, Aop, &Pop, rhs, wadj, true, kInnerM, kInnerK, 12, rtol_adj, 0.0, c.rec, gr, 0.0));
  c.rec.reset();
  inf.n_inner += gr.iters;
  // restarts that stopped reducing the residual mean either its rounding floor (the residual is
  // already what the gradient needs) or a plateau of the restarted method on a strongly non-normal
  // operator, which the long cycle is for
  const double adj_need = std::max(10.0 * rtol_adj, 1e-10);
  const bool at_floor = gr.stagnated && gr.resid <= adj_need * gr.resid0;
  if (!gr.converged && !at_floor) {
    const double r0 = gr.resid0;
    GmresResult g2;
    int rc2 = 0;
    if (c.prec == PREC_F64) {
      // FP64 preconditioner (linear to rounding): plain right preconditioning keeps one basis, half
      // the memory of the flexible form, so the cycle can be twice as long.  Solve (A P) y = r with
      // r = rhs - A w from the current iterate, then w += P y.  A truncated Fock ladder needs a
      // Krylov space of a few times n (about 4n for the dephased Kerr cavity at n = 128): one
      // cycle, restarted only to confirm the true residual.
      const int ml = long_cycle_len(c, kMaxLong, false);
      zd* r = X->zetaB;
      zd* y = X->rhoB;
      zd* t = X->delB;
      TRY(Aop(wadj, r));
      TRY(axpby(zmk(1, 0), rhs, zmk(-1, 0), r, n2, c.st));
      std::function<int(const zd*, zd*)> APop = [&](const zd* in, zd* out) -> int {
        int e = Pop(in, t);
        return e ? e : Aop(t, out);
      };
      rc2 = gmres_rec(X, APop, nullptr, r, y, true, ml, 0, 3, 0.0, rtol_adj * r0, c.rec, g2, 0.0);
      if (!rc2) rc2 = Pop(y, t);
      if (!rc2) rc2 = axpby(zmk(1, 0), t, zmk(1, 0), wadj, n2, c.st) ? LIND_EDEVICE : 0;
    } else {
      const int ml = long_cycle_len(c, kMaxLong, true);
      rc2 = gmres_rec(X, Aop, &Pop, rhs, wadj, false, ml, 0, 4, rtol_adj, 0.0, c.rec, g2, 0.0);
    }
    release_long_basis(c);
    TRY(rc2);
    inf.n_inner += g2.iters;
    g2.resid0 = r0;  // relative to ||rhs||, as for the first attempt
    gr = g2;
  }
  // hermitise w (exact adjoint state is Hermitian for Hermitian O), then its true relative residual
  TRY(hermitize(wadj, n, 0, nullptr, c.dscr, c.st));
  double adj_rel = 0.0;
  {
    TRY(Aop(wadj, X->zetaB));
    TRY(axpby(zmk(1, 0), rhs, zmk(-1, 0), X->zetaB, n2, c.st));
    double rn = 0;
    TRY(op_nrm(c, X->zetaB, &rn));
    adj_rel = rn / std::max(gr.resid0, 1e-300);
  }
  // g_H = i (rho w - w rho); M = rho w + w rho
  if (grad_H) {
    TRY(op_gemm(c, PREC_F64, n, n, n, rho, n, OP_N, wadj, n, OP_N, grad_H, n, cplx(0, 1), 0));
    TRY(op_gemm(c, PREC_F64, n, n, n, wadj, n, OP_N, rho, n, OP_N, grad_H, n, cplx(0, -1), 1));
  }
  if (grad_L && d > 0) {
    // derivatives with respect to the jump operators as given (a gauge shift leaves L unchanged)
    const zd* Lg = c.L0 ? c.L0 : c.L;
    zd* M = X->xiB;
    TRY(op_gemm(c, PREC_F64, n, n, n, rho, n, OP_N, wadj, n, OP_N, M, n, one, 0));
    TRY(op_gemm(c, PREC_F64, n, n, n, wadj, n, OP_N, rho, n, OP_N, M, n, one, 1));
    // grad_L = L M (stacked), then grad_L_j -= 2 w (L_j rho)
    TRY(op_gemm(c, PREC_F64, d * n, n, n, Lg, n, OP_N, M, n, OP_N, grad_L, n, one, 0));
    TRY(op_gemm(c, PREC_F64, d * n, n, n, Lg, n, OP_N, rho, n, OP_N, c.Ys, n, one, 0));
    for (int j = 0; j < d; ++j)
      TRY(op_gemm(c, PREC_F64, n, n, n, wadj, n, OP_N, c.Ys + (long long)j * n2, n, OP_N,
                  (zd*)grad_L + (long long)j * n2, n, cplx(-2, 0), 1));
  }
  if (rho_out) TRY(copy(rho, (zd*)rho_out, n2, c.st));
  TRY(c.sync());
  // release the per-call buffers
  for (zd* p : {rho, wadj, rhs}) {
    for (auto it = c.allocs.begin(); it != c.allocs.end(); ++it)
      if (*it == (void*)p) { c.allocs.erase(it); break; }
    hipFree(p);
  }
  inf.err_est = adj_rel;
  inf.t_solve_s = now_s() - t0;
  if (info) *info = inf;
  if (status) return c.fail(status, "steady state for the gradient did not reach the tolerance");
  // a solve that stops at its rounding floor short of rtol_adj is accepted when the true relative
  // residual is far below what the gradient needs (1e-10; the FP64 floor of the long chains of a
  // truncated Fock ladder sits near 1e-13)
  const bool adj_ok = adj_rel <= adj_need;
  if (!adj_ok) {
    char msg[160];
    std::snprintf(msg, sizeof msg, "adjoint GMRES did not converge (relative residual %.2e after %d iterations)",
                  adj_rel, inf.n_inner);
    return c.fail(LIND_ENOCONV, msg);
  }
  return LIND_OK;
}

// ---------------------------------------------------------------------------------------------
// Algorithm "Steady state via preconditioned GMRES": the deflated system L~_eta rho = eta I
// (eq. steady_state_linear_problem), written as -(L~_eta) rho = -eta I and right-preconditioned by
// P_0 = Precond(., 0, eta) (Algorithm "Precond", eq. ShermanMorr), solved by the recycled flexible
// GMRES(m) one cycle at a time from the warm start |0><0| (or rho0).  After every cycle the iterate is
// hermitised and trace-normalised and its FP64 residual bound tested against tol; the best
// iterate is returned.
// ---------------------------------------------------------------------------------------------
__global__ void k_ket0bra0(zd* X, int n) {
  const long long tot = (long long)n * n;
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < tot; t += stride)
    X[t] = zmk(t == 0 ? 1.0 : 0.0, 0.0);
}

int lindx::steady_state_gmres(lind_ctx* X, double tol, const zd* rho0, zd* rho_out, lind_info* info) {
  Ctx& c = X->c;
  const int n = c.n;
  const long long n2 = c.n2;
  const double t0 = now_s();
  const double deadline = c.opts.time_limit_s > 0 ? t0 + c.opts.time_limit_s : 0.0;
  const double eta = c.opts.eta;
  TRY(ensure_solver_bufs(X));
  lind_info inf;
  std::memset(&inf, 0, sizeof(inf));
  inf.kappa_U = c.kappa;
  inf.t_factor_s = c.t_factor;
  inf.route_used = c.route;
  Precond P;
  TRY(make_precond(X, P, cplx(0, 0), eta, false));
  std::function<int(const zd*, zd*)> Aop = [&](const zd* in, zd* out) -> int {
    return apply_shifted_deflated(c, in, out, cplx(0, 0), eta, false);
  };
  std::function<int(const zd*, zd*)> Pop = [&](const zd* in, zd* out) -> int {
    ++inf.n_phi;
    return apply_precond(c, P, in, out, c.prec);
  };
  // right-hand side -eta I (zetaB) and the iterate (rhoB)
  TRY(fill_zero(X->zetaB, n2 * (long long)sizeof(zd), c.st));
  TRY(add_identity(X->zetaB, n, zmk(-eta, 0), c.st));
  if (rho0) TRY(copy(rho0, X->rhoB, n2, c.st));
  else hipLaunchKernelGGL(k_ket0bra0, dim3(1024), dim3(256), 0, c.st, X->rhoB, n);
  const int m = c.opts.m;
  const int k = std::max(0, std::min(m / 2, m - 2));
  c.rec.reset();
  double best = 1e300, best_max = 0;
  bool converged = false;
  for (int cyc = 0; cyc < c.opts.max_restarts; ++cyc) {
    GmresResult gr;
    TRY(gmres_rec(X, Aop, &Pop, X->zetaB, X->rhoB, false, m, k, 1, 1e-15, 0.0, c.rec, gr, deadline));
    inf.n_inner += gr.iters;
    ++inf.n_restarts;
    // rho^ = herm(rho)/Tr rho, FP64 residual
    TRY(copy(X->rhoB, X->delB, n2, c.st));
    double colsum = 0, mx = 0, fro = 0;
    TRY(finish_state(X, X->delB, &colsum, &mx, &fro, nullptr));
    if (colsum < best) {
      best = colsum;
      best_max = mx;
      TRY(copy(X->delB, rho_out, n2, c.st));
    }
    if (colsum <= tol) { converged = true; break; }
    if (gr.stagnated && gr.cycles == 0) break;
    if (deadline > 0 && now_s() > deadline) break;
  }
  c.rec.reset();
  TRY(c.sync());
  inf.resid_trace = best;
  inf.resid_max = best_max;
  inf.err_est = best;
  inf.t_solve_s = now_s() - t0;
  if (info) *info = inf;
  if (!converged) return c.fail(LIND_ENOCONV, "steady state (GMRES): tolerance not reached (best iterate returned)");
  return LIND_OK;
}
