// Right-preconditioned GMRES with Krylov subspace recycling (GCRO-DR: Parks, de Sturler, Mackey,
// Johnson and Maiti, SIAM J. Sci. Comput. 2006), the inner solver of the linear-solver section:
// after every cycle a harmonic-Ritz subspace (U, C) with A U = C, C orthonormal, is kept and
// carried into the next cycle and into later solves with the same operator.
// The preconditioned directions z_j = P(v_j) are stored (flexible form): the solution is updated
// from them directly, so a preconditioner applied in reduced precision (an operator that is
// linear only up to its rounding) limits neither the residual recurrence nor the final accuracy,
// and U lives in the solution space, tied to A alone.
//
// Notation for one cycle with k recycled vectors and j Arnoldi steps (s = k + j):
//   V^ = [C, v_0 .. v_j]        (s + 1 orthonormal vectors, stored contiguously in the K2 basis)
//   W^ = [U D, z_0 .. z_{j-1}]  (D = diag(1 / ||u_i||), z_i = P(v_i), or v_i without P)
//   A W^ = V^ Gbar,  Gbar = [[D, B], [0, Hbar]]  ((s + 1) x s)
// The least-squares problem min || beta e_{k+1} - Gbar z || decouples: the U block of z zeroes the
// first k rows, so the residual estimate is the one of plain GMRES on Hbar.  The new recycle space
// is spanned by the harmonic Ritz vectors for the smallest harmonic Ritz values:
//   Gbar^H Gbar p = theta Gbar^H V^^H W^ p,
// rewritten with Gbar = Qg Rg as the standard problem Rg^{-1} Qg^H (V^^H W^) p = (1/theta) p.
// All vector work (Gram-Schmidt, the tall-skinny products of the update) runs on the device in
// FP64; the (s + 1) x s problems are solved on the host.
//
// Cycles longer than 64 steps (m up to kMaxLong) keep no recycle space: they are plain restarted
// GMRES with a long basis, for operators whose preconditioned form is strongly non-normal (a chain
// of Fock levels needs about as many Krylov steps as it has levels, and restarts lose them).  The
// basis then lives in HBM (m + 3 vectors of n*n complex128).
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <numeric>
#include "ctx.hpp"

namespace lindx {

#define TRY(x)                                           \
  do {                                                   \
    int rc__ = (x);                                      \
    if (rc__) return rc__ < 0 ? rc__ : LIND_EDEVICE;     \
  } while (0)

namespace {

// thin Householder QR of the r x cc row-major matrix A (r >= cc): A = Q R, Q r x cc, R cc x cc
void house_qr(const std::vector<cplx>& A, int r, int cc, std::vector<cplx>& Q, std::vector<cplx>& R) {
  std::vector<cplx> W(A);
  std::vector<std::vector<cplx>> vs(cc);
  for (int j = 0; j < cc; ++j) {
    double nx = 0;
    for (int i = j; i < r; ++i) nx += std::norm(W[(size_t)i * cc + j]);
    nx = std::sqrt(nx);
    std::vector<cplx> v(r - j, 0.0);
    if (nx > 0) {
      const cplx x0 = W[(size_t)j * cc + j];
      const cplx ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cplx(1, 0);
      for (int i = j; i < r; ++i) v[i - j] = W[(size_t)i * cc + j];
      v[0] += ph * nx;  // v = x - alpha e_1 with alpha = -ph ||x||
      double vn = 0;
      for (auto& z : v) vn += std::norm(z);
      vn = std::sqrt(vn);
      for (auto& z : v) z /= vn;
      for (int l = j; l < cc; ++l) {
        cplx s = 0;
        for (int i = j; i < r; ++i) s += std::conj(v[i - j]) * W[(size_t)i * cc + l];
        for (int i = j; i < r; ++i) W[(size_t)i * cc + l] -= 2.0 * v[i - j] * s;
      }
    }
    vs[j] = std::move(v);
  }
  R.assign((size_t)cc * cc, 0.0);
  for (int i = 0; i < cc; ++i)
    for (int l = i; l < cc; ++l) R[(size_t)i * cc + l] = W[(size_t)i * cc + l];
  Q.assign((size_t)r * cc, 0.0);
  for (int i = 0; i < cc; ++i) Q[(size_t)i * cc + i] = 1.0;
  for (int j = cc - 1; j >= 0; --j) {
    const auto& v = vs[j];
    for (int l = 0; l < cc; ++l) {
      cplx s = 0;
      for (int i = j; i < r; ++i) s += std::conj(v[i - j]) * Q[(size_t)i * cc + l];
      for (int i = j; i < r; ++i) Q[(size_t)i * cc + l] -= 2.0 * v[i - j] * s;
    }
  }
}

// h[j] = <V_j, w> for j < k, in chunks of 64 basis vectors
int mdot(Ctx& c, const zd* V, int k, const zd* w, zd* h) {
  for (int c0 = 0; c0 < k; c0 += 64)
    TRY(multi_dot(V + (long long)c0 * c.n2, c.n2, std::min(64, k - c0), w, c.n2, h + c0, (zd*)c.dscr, c.st));
  return 0;
}
// w = [accumulate ? w : 0] + coeff * sum_j h[j] V_j, in chunks of 128 basis vectors
int maxpy(Ctx& c, const zd* V, int k, const zd* h, zd* w, int accumulate, double coeff) {
  for (int c0 = 0; c0 < k; c0 += 128)
    TRY(multi_axpy(V + (long long)c0 * c.n2, c.n2, std::min(128, k - c0), h + c0, w, c.n2,
                   (c0 > 0) ? 1 : accumulate, coeff, c.st));
  return 0;
}

int upload(Ctx& c, const std::vector<cplx>& v, zd* dst) {
  const size_t cnt = v.size();
  if (cnt > (size_t)kHostScalars) return LIND_EINVAL;
  for (size_t i = 0; i < cnt; ++i) c.hsc[i] = zmk(v[i].real(), v[i].imag());
  if (hipMemcpyAsync(dst, c.hsc, sizeof(zd) * cnt, hipMemcpyHostToDevice, c.st) != hipSuccess) return LIND_EDEVICE;
  return c.sync();  // the pinned staging buffer is reused right after
}

// Cout (M x len, rows ld len) = Acoef (M x K, row-major, device) * Vrows (K x len, rows ld len)
int rows_combine(Ctx& c, int M, int K, const zd* Acoef, const zd* Vrows, zd* Cout, long long len, int beta) {
  GemmDesc g;
  g.M = M; g.N = (int)len; g.K = K;
  g.A = Acoef; g.lda = K; g.opA = OP_N;
  g.B = Vrows; g.ldb = len; g.opB = OP_N;
  g.C = Cout; g.ldc = len;
  g.beta = beta;
  return gemm(PREC_F64, g, c.st) ? LIND_EDEVICE : 0;
}

}  // namespace

int long_cycle_len(Ctx& c, int want, bool flexible) {
  size_t fr = 0, tot = 0;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess) fr = 0;
  const double vec = 16.0 * (double)c.n2;
  // at most half of the free HBM and 32 GiB for the basis (and the preconditioned directions)
  const double budget = std::min(0.5 * (double)fr + (double)c.K2cap * vec, 32.0 * (1ull << 30));
  const int fit = ((int)std::max(0.0, budget / vec) - 3) / (flexible ? 2 : 1);
  return std::max(3, std::min({want, kMaxLong, fit}));
}

void release_long_basis(Ctx& c) {
  if (c.K2 && c.K2cap > 67) {
    c.release(c.K2);
    c.K2 = nullptr;
    c.K2cap = 0;
  }
}

int Recycle::ensure(Ctx& c, int kcap) {
  if (cap >= kcap && n2 == c.n2) return 0;
  for (zd** p : {&U, &Un, &C}) {
    if (*p) c.release(*p);
    *p = nullptr;
  }
  k = 0;
  cap = 0;
  n2 = c.n2;
  TRY(c.alloc(&U, (size_t)kcap * c.n2));
  TRY(c.alloc(&Un, (size_t)kcap * c.n2));
  TRY(c.alloc(&C, (size_t)kcap * c.n2));
  cap = kcap;
  return 0;
}

// T (M x N, row-major on device) = Urows (M x len) * Vrows^H (len x N): T[a][b] = sum_t U_a[t] conj(V_b[t]).
// The length-len reduction is split into nb batches reduced by the split-K GEMM, plus a remainder.
int Recycle::cross(Ctx& c, const zd* Urows, int M, const zd* Vrows, int N, zd* T) {
  const long long len = c.n2;
  long long nb = 1;
  while (nb < 1024 && len / (nb * 2) >= 64) nb *= 2;
  const long long kb = len / nb, rem = len - nb * kb;
  const long long need = gemm_ws_bytes(PREC_F64, M, N, (int)nb);
  if (need > ws_bytes) {
    if (ws) c.release(ws);
    ws = nullptr;
    ws_bytes = 0;
    zd* p = nullptr;
    TRY(c.alloc(&p, (size_t)(need + 15) / 16));
    ws = p;
    ws_bytes = need;
  }
  GemmDesc g;
  g.M = M; g.N = N; g.K = (int)kb; g.nbatch = (int)nb;
  g.A = Urows; g.lda = len; g.sA = kb; g.opA = OP_N;
  g.B = Vrows; g.ldb = len; g.sB = kb; g.opB = OP_C;
  g.C = T; g.ldc = N;
  g.ws = need > 0 ? ws : nullptr;
  if (gemm(PREC_F64, g, c.st)) return LIND_EDEVICE;
  if (rem > 0) {
    GemmDesc h;
    h.M = M; h.N = N; h.K = (int)rem;
    h.A = Urows + nb * kb; h.lda = len; h.opA = OP_N;
    h.B = Vrows + nb * kb; h.ldb = len; h.opB = OP_C;
    h.C = T; h.ldc = N;
    h.beta = 1;
    if (gemm(PREC_F64, h, c.st)) return LIND_EDEVICE;
  }
  return 0;
}

int gmres_rec(lind_ctx* X, const std::function<int(const zd*, zd*)>& A, const std::function<int(const zd*, zd*)>* P,
              const zd* b, zd* x, bool x_zero, int m, int kdef, int max_cycles, double rtol, double atol,
              Recycle& rec, GmresResult& res, double t_deadline) {
  Ctx& c = X->c;
  const long long n2 = c.n2;
  m = std::max(3, std::min(m, kMaxLong));
  kdef = (m > 64) ? 0 : std::max(0, std::min(kdef, m - 2));
  const bool flex = P != nullptr;
  TRY(c.ensure_krylov(2, flex ? 2 * m + 3 : m + 3));
  if (kdef > 0) TRY(rec.ensure(c, kdef));
  if (rec.k > kdef) rec.k = 0;  // a space from a larger setting is dropped, not truncated
  if (!rec.coef) TRY(c.alloc(&rec.coef, 3 * 64 * 72));
  if (!rec.hb) TRY(c.alloc(&rec.hb, 2 * (kMaxLong + 1) + 8));
  zd* Vh = c.K2;                          // slots 0 .. m: [C, v_0 .. v_j]
  zd* tmp = Vh + (long long)(m + 1) * n2;  // scratch slot
  zd* dy = Vh + (long long)(m + 2) * n2;   // correction of x accumulated over the cycle
  zd* Zb = flex ? Vh + (long long)(m + 3) * n2 : nullptr;  // z_j = P(v_j), slots m + 3 ..

  // device scalars of a step with nb basis vectors: [norm | h (first pass, nb) | h (second pass, nb)]
  zd* nrmdev = rec.hb;
  zd* hdev = rec.hb + 1;
  zd* crdev = c.dsc + 160;

  double bnorm = 0;
  TRY(op_nrm(c, b, &bnorm));
  if (x_zero) TRY(fill_zero(x, n2 * (long long)sizeof(zd), c.st));
  res = GmresResult();
  const double target = std::max(rtol * bnorm, atol);
  double prev_beta = 0.0;
  int slow = 0, floor_hits = 0;
  bool prev_est_hit = false;
  for (int cyc = 0; cyc < max_cycles; ++cyc) {
    const int kc = rec.k;
    zd* r = Vh + (long long)kc * n2;
    if (cyc == 0 && x_zero) {
      TRY(copy(b, r, n2, c.st));
    } else {
      TRY(A(x, tmp));
      TRY(copy(b, r, n2, c.st));
      TRY(axpby(zmk(-1, 0), tmp, zmk(1, 0), r, n2, c.st));
    }
    double beta = 0;
    TRY(op_nrm(c, r, &beta));
    if (cyc == 0) res.resid0 = beta;
    res.resid = beta;
    if (beta <= target || beta == 0.0) { res.converged = true; break; }
    if (cyc > 0) {
      // rounding floor: the previous cycle's recurrence reached the target but the true residual
      // did not (twice), or restarts no longer reduce the true residual at all (three times)
      if (prev_est_hit && beta > 0.5 * prev_beta) ++floor_hits;
      if (beta > 0.999 * prev_beta) ++slow;
      else slow = 0;
      if (floor_hits >= 2 || slow >= 3) { res.stagnated = true; break; }
    }
    prev_beta = beta;
    prev_est_hit = false;
    if (t_deadline > 0 && now_s() > t_deadline) break;
    // project the residual off range(C); the U part of the correction is U C^H r
    std::vector<cplx> cr(kc);
    if (kc > 0) {
      TRY(copy(rec.C, Vh, (long long)kc * n2, c.st));
      TRY(multi_dot(Vh, n2, kc, r, n2, crdev, (zd*)c.dscr, c.st));
      TRY(multi_axpy(Vh, n2, kc, crdev, r, n2, 1, -1.0, c.st));
      TRY(multi_axpy(rec.U, n2, kc, crdev, dy, n2, 0, 1.0, c.st));
      TRY(c.fetch(crdev, sizeof(zd) * kc));
      for (int i = 0; i < kc; ++i) cr[i] = cplx(c.hsc[i].x, c.hsc[i].y);
      TRY(op_nrm(c, r, &beta));
      if (!(beta > 0)) {
        TRY(axpby(zmk(1, 0), dy, zmk(1, 0), x, n2, c.st));
        res.cycles = cyc + 1;
        continue;
      }
    }
    TRY(scale_by_inv(r, n2, (const double*)c.dsc, c.st));  // dsc[0] holds beta
    const int mm = m - kc;
    // Hraw (the unrotated Hessenberg) is kept only for the recycle update; without recycling (the
    // long cycles, up to kMaxLong steps) the columns go straight into Hg
    std::vector<cplx> Hg((size_t)(mm + 1) * mm, 0.0);
    std::vector<cplx> Hraw(kdef > 0 ? (size_t)(mm + 1) * mm : 0, 0.0);
    std::vector<cplx>& HR = kdef > 0 ? Hraw : Hg;
    std::vector<cplx> Bh((size_t)std::max(kc, 1) * mm, 0.0);
    std::vector<cplx> cs(mm), sn(mm), g(mm + 1, 0.0);
    g[0] = beta;
    int jd = 0;
    double est = beta;
    bool breakdown = false;
    for (int j = 0; j < mm; ++j) {
      zd* vj = Vh + (long long)(kc + j) * n2;
      zd* w = Vh + (long long)(kc + j + 1) * n2;
      if (flex) {
        zd* zj = Zb + (long long)j * n2;
        TRY((*P)(vj, zj));
        TRY(A(zj, w));
      } else {
        TRY(A(vj, w));
      }
      const int nb = kc + j + 1;
      zd* h2dev = hdev + nb;
      TRY(mdot(c, Vh, nb, w, hdev));
      TRY(maxpy(c, Vh, nb, hdev, w, 1, -1.0));
      TRY(mdot(c, Vh, nb, w, h2dev));
      TRY(maxpy(c, Vh, nb, h2dev, w, 1, -1.0));
      TRY(nrm2(w, n2, (double*)nrmdev, c.dscr, c.st));
      TRY(c.fetch(rec.hb, sizeof(zd) * (1 + 2 * nb)));
      const double hn = ((const double*)c.hsc)[0];
      for (int i = 0; i < nb; ++i) {
        const cplx h = cplx(c.hsc[1 + i].x, c.hsc[1 + i].y) + cplx(c.hsc[1 + nb + i].x, c.hsc[1 + nb + i].y);
        if (i < kc) Bh[(size_t)i * mm + j] = h;
        else HR[(size_t)(i - kc) * mm + j] = h;
      }
      HR[(size_t)(j + 1) * mm + j] = hn;
      if (hn > 0) TRY(scale_by_inv(w, n2, (const double*)nrmdev, c.st));
      if (kdef > 0)
        for (int i = 0; i <= j + 1; ++i) Hg[(size_t)i * mm + j] = Hraw[(size_t)i * mm + j];
      for (int i = 0; i < j; ++i) {
        const cplx a = Hg[(size_t)i * mm + j], bb = Hg[(size_t)(i + 1) * mm + j];
        Hg[(size_t)i * mm + j] = cs[i] * a + sn[i] * bb;
        Hg[(size_t)(i + 1) * mm + j] = -std::conj(sn[i]) * a + cs[i] * bb;
      }
      const cplx f = Hg[(size_t)j * mm + j], gg = Hg[(size_t)(j + 1) * mm + j];
      const double af = std::abs(f), ag = std::abs(gg);
      if (ag == 0) { cs[j] = 1; sn[j] = 0; }
      else if (af == 0) { cs[j] = 0; sn[j] = std::conj(gg) / ag; }
      else {
        const double nr = std::hypot(af, ag);
        const cplx ph = f / af;
        cs[j] = af / nr;
        sn[j] = ph * std::conj(gg) / nr;
      }
      Hg[(size_t)j * mm + j] = cs[j] * f + sn[j] * gg;
      Hg[(size_t)(j + 1) * mm + j] = 0;
      const cplx gj = g[j];
      g[j] = cs[j] * gj;
      g[j + 1] = -std::conj(sn[j]) * gj;
      jd = j + 1;
      est = std::abs(g[j + 1]);
      ++res.iters;
      if (hn == 0.0) { breakdown = true; break; }
      if (est <= target) break;
      if (t_deadline > 0 && now_s() > t_deadline) break;
    }
    // z_V from the triangular system; the U block of z is -D^{-1} B z_V, so that
    // dy += Z z_V - U (B z_V)   (Z = V without a preconditioner)
    std::vector<cplx> z(jd);
    for (int i = jd - 1; i >= 0; --i) {
      cplx acc = g[i];
      for (int l = i + 1; l < jd; ++l) acc -= Hg[(size_t)i * mm + l] * z[l];
      z[i] = acc / Hg[(size_t)i * mm + i];
    }
    if (kc > 0) {
      std::vector<cplx> bu(kc, 0.0);
      for (int i = 0; i < kc; ++i)
        for (int l = 0; l < jd; ++l) bu[i] -= Bh[(size_t)i * mm + l] * z[l];
      TRY(upload(c, bu, crdev));
      TRY(multi_axpy(rec.U, n2, kc, crdev, dy, n2, 1, 1.0, c.st));
    }
    TRY(upload(c, z, hdev));
    zd* Zpart = flex ? Zb : Vh + (long long)kc * n2;
    TRY(maxpy(c, Zpart, jd, hdev, dy, kc > 0 ? 1 : 0, 1.0));
    TRY(axpby(zmk(1, 0), dy, zmk(1, 0), x, n2, c.st));
    res.cycles = cyc + 1;
    res.resid = est;
    prev_est_hit = est <= target;
    res.est_hit = prev_est_hit;
    if (log_on() && m > 64)
      std::fprintf(stderr, "[lindx] long GMRES cycle %d: %d steps, residual estimate %.2e of %.2e\n", cyc, jd, est,
                   bnorm);

    // ---- recycle update: harmonic Ritz vectors over span(W^) ----
    // Without a preconditioner W^ and V^ live in one space and F = V^^H W^ is formed exactly.  In
    // the flexible form the harmonic Ritz problem is posed on the orthonormal [C, v_0 ..], i.e.
    // F = [I; 0] (as in flexible GMRES with deflated restarting); any selection keeps A U = C exact.
    const int s = kc + jd;
    int knew = std::min(kdef, s - 1);
    if (kdef == 0 || breakdown || knew < 1) continue;
    std::vector<double> dn(kc, 1.0);
    std::vector<cplx> VU;  // (s + 1) x kc: V^^H U (exact form only)
    if (kc > 0) {
      for (int i = 0; i < kc; ++i) TRY(nrm2(rec.U + (long long)i * n2, n2, (double*)(c.dsc + 200 + i), c.dscr, c.st));
      if (!flex) TRY(rec.cross(c, rec.U, kc, Vh, s + 1, rec.coef));  // T[a][b] = <V^_b, u_a>
      TRY(c.fetch(c.dsc + 200, sizeof(zd) * kc));
      for (int i = 0; i < kc; ++i) dn[i] = ((const double*)(c.hsc + i))[0];
      VU.assign((size_t)(s + 1) * kc, 0.0);
      if (flex) {
        for (int a = 0; a < kc; ++a) VU[(size_t)a * kc + a] = dn[a];  // F's U block becomes I
      } else {
        TRY(c.fetch(rec.coef, sizeof(zd) * kc * (s + 1)));
        for (int a = 0; a < kc; ++a)
          for (int bq = 0; bq <= s; ++bq)
            VU[(size_t)bq * kc + a] = std::conj(cplx(c.hsc[(size_t)a * (s + 1) + bq].x, c.hsc[(size_t)a * (s + 1) + bq].y));
      }
    }
    for (int i = 0; i < kc; ++i)
      if (!(dn[i] > 0) || !std::isfinite(dn[i])) { rec.k = 0; knew = 0; }
    if (knew < 1) continue;
    // Gbar and F = V^^H W^ ((s + 1) x s, row-major)
    std::vector<cplx> Gb((size_t)(s + 1) * s, 0.0), F((size_t)(s + 1) * s, 0.0);
    for (int i = 0; i < kc; ++i) {
      Gb[(size_t)i * s + i] = 1.0 / dn[i];
      for (int l = 0; l < jd; ++l) Gb[(size_t)i * s + kc + l] = Bh[(size_t)i * mm + l];
    }
    for (int i = 0; i <= jd; ++i)
      for (int l = 0; l < jd; ++l) Gb[(size_t)(kc + i) * s + kc + l] = Hraw[(size_t)i * mm + l];
    for (int bq = 0; bq <= s; ++bq)
      for (int a = 0; a < kc; ++a) F[(size_t)bq * s + a] = VU[(size_t)bq * kc + a] / dn[a];
    for (int l = 0; l < jd; ++l) F[(size_t)(kc + l) * s + kc + l] = 1.0;
    std::vector<cplx> Qg, Rg;
    house_qr(Gb, s + 1, s, Qg, Rg);
    // Mh = Rg^{-1} (Qg^H F)
    std::vector<cplx> Mh((size_t)s * s, 0.0);
    for (int i = 0; i < s; ++i)
      for (int l = 0; l < s; ++l) {
        cplx acc = 0;
        for (int q = 0; q <= s; ++q) acc += std::conj(Qg[(size_t)q * s + i]) * F[(size_t)q * s + l];
        Mh[(size_t)i * s + l] = acc;
      }
    bool singular = false;
    for (int i = 0; i < s; ++i) singular |= !(std::abs(Rg[(size_t)i * s + i]) > 0);
    if (singular) { rec.k = 0; continue; }
    for (int l = 0; l < s; ++l)
      for (int i = s - 1; i >= 0; --i) {
        cplx acc = Mh[(size_t)i * s + l];
        for (int q = i + 1; q < s; ++q) acc -= Rg[(size_t)i * s + q] * Mh[(size_t)q * s + l];
        Mh[(size_t)i * s + l] = acc / Rg[(size_t)i * s + i];
      }
    std::vector<cplx> wv, Yv;
    int erc = small_eig_host(X, Mh, s, s, wv, Yv);
    if (erc && erc != LIND_ENOCONV) return erc;
    if (erc) { rec.k = 0; continue; }
    std::vector<int> ord(s);
    std::iota(ord.begin(), ord.end(), 0);
    std::sort(ord.begin(), ord.end(), [&](int a, int bq) { return std::abs(wv[a]) > std::abs(wv[bq]); });
    // Pk (s x knew), then Gbar Pk = Qy Ry
    std::vector<cplx> Pk((size_t)s * knew), GP((size_t)(s + 1) * knew, 0.0);
    for (int i = 0; i < s; ++i)
      for (int t = 0; t < knew; ++t) Pk[(size_t)i * knew + t] = Yv[(size_t)i * s + ord[t]];
    for (int i = 0; i <= s; ++i)
      for (int t = 0; t < knew; ++t) {
        cplx acc = 0;
        for (int q = 0; q < s; ++q) acc += Gb[(size_t)i * s + q] * Pk[(size_t)q * knew + t];
        GP[(size_t)i * knew + t] = acc;
      }
    std::vector<cplx> Qy, Ry;
    house_qr(GP, s + 1, knew, Qy, Ry);
    double rmax = 0;
    for (int t = 0; t < knew; ++t) rmax = std::max(rmax, std::abs(Ry[(size_t)t * knew + t]));
    int keep = 0;
    while (keep < knew && std::abs(Ry[(size_t)keep * knew + keep]) > 1e-10 * rmax) ++keep;
    if (keep < 1) { rec.k = 0; continue; }
    // Pk Ry^{-1} restricted to the first `keep` columns (Ry upper triangular)
    std::vector<cplx> PR((size_t)s * keep, 0.0);
    for (int i = 0; i < s; ++i)
      for (int t = 0; t < keep; ++t) {
        cplx acc = Pk[(size_t)i * knew + t];
        for (int q = 0; q < t; ++q) acc -= PR[(size_t)i * keep + q] * Ry[(size_t)q * knew + t];
        PR[(size_t)i * keep + t] = acc / Ry[(size_t)t * knew + t];
      }
    // C_new = V^ Qy (keep rows), U_new = U D PR[0:kc] + V PR[kc:s]
    std::vector<cplx> Ac((size_t)keep * (s + 1)), Au((size_t)keep * std::max(kc, 1)), Av((size_t)keep * jd);
    for (int t = 0; t < keep; ++t) {
      for (int q = 0; q <= s; ++q) Ac[(size_t)t * (s + 1) + q] = Qy[(size_t)q * knew + t];
      for (int a = 0; a < kc; ++a) Au[(size_t)t * kc + a] = PR[(size_t)a * keep + t] / dn[a];
      for (int l = 0; l < jd; ++l) Av[(size_t)t * jd + l] = PR[(size_t)(kc + l) * keep + t];
    }
    zd* dAc = rec.coef;
    zd* dAu = rec.coef + 64 * 72;
    zd* dAv = rec.coef + 2 * 64 * 72;
    TRY(upload(c, Ac, dAc));
    TRY(rows_combine(c, keep, s + 1, dAc, Vh, rec.C, n2, 0));
    if (kc > 0) {
      Au.resize((size_t)keep * kc);
      TRY(upload(c, Au, dAu));
      TRY(rows_combine(c, keep, kc, dAu, rec.U, rec.Un, n2, 0));
    }
    TRY(upload(c, Av, dAv));
    TRY(rows_combine(c, keep, jd, dAv, Zpart, rec.Un, n2, kc > 0 ? 1 : 0));
    std::swap(rec.U, rec.Un);
    rec.k = keep;
  }
  return 0;
}

}  // namespace lindx
