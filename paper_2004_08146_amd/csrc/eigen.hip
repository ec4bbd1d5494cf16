// GD-lambdaAMG (Alg. GD-lambdaAMG, Sec. 3.3): generalized Davidson for the
// eigenpairs of Q = Gamma5 D of smallest modulus.
//
// Search space V (orthonormal, FP64 fields) and W = Q V; harmonic Ritz pairs
// (Theorem on harmonic Ritz values, Sec. 3.2) from the small generalized
// problem W^H W s = theta W^H V s, solved on the host through a Cholesky
// factor of W^H W and a cyclic Jacobi eigensolver.  The correction equation
// (Q - theta) t = r is solved approximately by the multigrid-preconditioned
// FGMRES of the shifted-solve path (in its Gamma5 form (D - theta Gamma5) t =
// Gamma5 r, eq. (3.7)); converged pairs are locked (the expansion vector is
// kept orthogonal to them), the space is thick-restarted from m_max to m_min
// harmonic Ritz vectors, and the interpolation is rebuilt from the converged
// eigenvectors closest to the current target (Sec. 3.3, interpolation
// updates).  All field arithmetic runs in the library's kernels; the host
// holds only m x m matrices.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <numeric>
#include <vector>

#include "qmg_ctx.h"

using cd = std::complex<double>;

// ---- dense Hermitian eigenproblem (host): cyclic Jacobi with complex
// rotations.  a: m x m Hermitian, column-major; on return w holds the
// eigenvalues in ascending order and z the eigenvectors as columns.
void herm_eig(int m, std::vector<cd> a, std::vector<double>& w, std::vector<cd>& z) {
  auto A = [&](int i, int j) -> cd& { return a[(size_t)j * m + i]; };
  z.assign((size_t)m * m, cd(0));
  for (int i = 0; i < m; ++i) z[(size_t)i * m + i] = 1.0;
  for (int i = 0; i < m; ++i) A(i, i) = cd(A(i, i).real(), 0.0);
  double fro = 0;
  for (const cd& v : a) fro += std::norm(v);
  fro = std::sqrt(fro);
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0;
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i)
        if (i != j) off += std::norm(A(i, j));
    if (std::sqrt(off) <= 1e-15 * fro || fro == 0.0) break;
    for (int p = 0; p < m - 1; ++p)
      for (int q = p + 1; q < m; ++q) {
        const cd apq = A(p, q);
        const double g = std::abs(apq);
        if (g <= 1e-300) continue;
        // D^H A D with D = diag(.., 1 at p, e^{-i phi} at q, ..) makes the pair
        // real; the real rotation R = [[c, s], [-s, c]] then zeroes it
        const cd e = apq / g;  // e^{i phi}
        const double app = A(p, p).real(), aqq = A(q, q).real();
        const double tau = (aqq - app) / (2.0 * g);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        const cd em = std::conj(e);
        // columns: [A_p, A_q] <- [A_p, A_q] G, G = D R = [[c, s], [-s em, c em]]
        for (int i = 0; i < m; ++i) {
          const cd xp = A(i, p), xq = A(i, q);
          A(i, p) = c * xp - s * em * xq;
          A(i, q) = s * xp + c * em * xq;
        }
        // rows: [A_p.; A_q.] <- G^H [A_p.; A_q.]
        for (int j = 0; j < m; ++j) {
          const cd xp = A(p, j), xq = A(q, j);
          A(p, j) = c * xp - s * e * xq;
          A(q, j) = s * xp + c * e * xq;
        }
        A(p, q) = 0.0;
        A(q, p) = 0.0;
        A(p, p) = cd(A(p, p).real(), 0.0);
        A(q, q) = cd(A(q, q).real(), 0.0);
        for (int i = 0; i < m; ++i) {
          cd& zp = z[(size_t)p * m + i];
          cd& zq = z[(size_t)q * m + i];
          const cd xp = zp, xq = zq;
          zp = c * xp - s * em * xq;
          zq = s * xp + c * em * xq;
        }
      }
  }
  std::vector<int> idx(m);
  std::iota(idx.begin(), idx.end(), 0);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return A(x, x).real() < A(y, y).real(); });
  std::vector<cd> zs((size_t)m * m);
  w.resize(m);
  for (int k = 0; k < m; ++k) {
    w[k] = A(idx[k], idx[k]).real();
    for (int i = 0; i < m; ++i) zs[(size_t)k * m + i] = z[(size_t)idx[k] * m + i];
  }
  z.swap(zs);
}

namespace {

// Harmonic Ritz pairs of the pencil G s = theta M s (G = W^H W Hermitian
// positive definite, M = W^H V Hermitian), column-major m x m.  With
// G = L L^H: L^{-1} M L^{-H} y = mu y, s = L^{-H} y, theta = 1 / mu.
// Returns the pairs sorted by |theta| (pairs with mu = 0 are dropped).
bool harmonic_ritz(int m, const std::vector<cd>& G, const std::vector<cd>& M, std::vector<double>& theta,
                   std::vector<std::vector<cd>>& S) {
  std::vector<cd> L((size_t)m * m, cd(0));
  auto Lr = [&](int i, int j) -> cd& { return L[(size_t)j * m + i]; };
  for (int j = 0; j < m; ++j) {
    double d = G[(size_t)j * m + j].real();
    for (int k = 0; k < j; ++k) d -= std::norm(Lr(j, k));
    if (!(d > 0) || !std::isfinite(d)) return false;
    Lr(j, j) = std::sqrt(d);
    for (int i = j + 1; i < m; ++i) {
      cd v = G[(size_t)j * m + i];
      for (int k = 0; k < j; ++k) v -= Lr(i, k) * std::conj(Lr(j, k));
      Lr(i, j) = v / Lr(j, j);
    }
  }
  // B = L^{-1} M (forward substitution column by column), C = L^{-1} B^H ^H
  std::vector<cd> B((size_t)m * m);
  for (int col = 0; col < m; ++col)
    for (int i = 0; i < m; ++i) {
      cd v = 0.5 * (M[(size_t)col * m + i] + std::conj(M[(size_t)i * m + col]));
      for (int k = 0; k < i; ++k) v -= Lr(i, k) * B[(size_t)col * m + k];
      B[(size_t)col * m + i] = v / Lr(i, i);
    }
  // C = B L^{-H}: C^H = L^{-1} B^H; solve per column of B^H
  std::vector<cd> C((size_t)m * m);
  for (int row = 0; row < m; ++row) {
    std::vector<cd> x(m);
    for (int i = 0; i < m; ++i) {
      cd v = std::conj(B[(size_t)i * m + row]);
      for (int k = 0; k < i; ++k) v -= Lr(i, k) * x[k];
      x[i] = v / Lr(i, i);
    }
    for (int i = 0; i < m; ++i) C[(size_t)i * m + row] = std::conj(x[i]);
  }
  std::vector<double> mu;
  std::vector<cd> Y;
  herm_eig(m, C, mu, Y);
  std::vector<int> idx;
  for (int k = 0; k < m; ++k)
    if (std::abs(mu[k]) > 1e-300) idx.push_back(k);
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return std::abs(mu[x]) > std::abs(mu[y]); });
  theta.clear();
  S.clear();
  for (int k : idx) {
    std::vector<cd> s(m);
    for (int i = m - 1; i >= 0; --i) {  // L^H s = y
      cd v = Y[(size_t)k * m + i];
      for (int l = i + 1; l < m; ++l) v -= std::conj(Lr(l, i)) * s[l];
      s[i] = v / std::conj(Lr(i, i));
    }
    double nrm = 0;
    for (const cd& v : s) nrm += std::norm(v);
    nrm = std::sqrt(nrm);
    for (cd& v : s) v /= nrm;
    theta.push_back(1.0 / mu[k]);
    S.push_back(s);
  }
  return true;
}

// Rayleigh-Ritz pairs of Q on the orthonormal search space: V^H Q V = M^H (M = W^H V,
// Hermitian in exact arithmetic), taken symmetrised; sorted by |theta|.
void rayleigh_ritz(int m, const std::vector<cd>& M, std::vector<double>& theta, std::vector<std::vector<cd>>& S) {
  std::vector<cd> H((size_t)m * m);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) H[(size_t)j * m + i] = 0.5 * (std::conj(M[(size_t)i * m + j]) + M[(size_t)j * m + i]);
  std::vector<double> w;
  std::vector<cd> Y;
  herm_eig(m, H, w, Y);
  std::vector<int> idx(m);
  for (int k = 0; k < m; ++k) idx[k] = k;
  std::sort(idx.begin(), idx.end(), [&](int x, int y) { return std::abs(w[x]) < std::abs(w[y]); });
  theta.clear();
  S.clear();
  for (int k : idx) {
    theta.push_back(w[k]);
    S.emplace_back(Y.begin() + (size_t)k * m, Y.begin() + (size_t)(k + 1) * m);
  }
}

}  // namespace

qmg_status solver_eigensolve(qmg_ctx* c, int nev, double* lambda, void* X, const void* V0, int n0, const void* t0,
                             const qmg_eig_params* prm, qmg_eig_stats* stats, hipStream_t s) {
  auto tstart = std::chrono::steady_clock::now();
  const int64_t n = (int64_t)field_elems(c);
  const size_t fb = (size_t)n * 16;
  const int mmax = prm->m_max, mmin = prm->m_min, nblk = prm->block;
  const int ntgt = prm->both_signs ? 2 * nblk : nblk;  // correction equations per outer step
  auto fld = [&](void* base, int j) { return (void*)((char*)base + (size_t)j * fb); };
  void* V = ws_get(c, "eg_V", fb * (mmax + 1));
  void* W = ws_get(c, "eg_W", fb * (mmax + 1));
  void* T = ws_get(c, "eg_T", fb * (mmax + 1));
  // per target of a block step: correction t, Ritz vector u, Q u, residual r
  void* Tc = ws_get(c, "eg_t", fb * ntgt);
  void* U = ws_get(c, "eg_u", fb * ntgt);
  void* QU = ws_get(c, "eg_Qu", fb * ntgt);
  void* R = ws_get(c, "eg_r", fb * ntgt);
  const int nmax = std::max(std::max(mmax, nev), c->ntv) + 2;
  double* d_dots = (double*)ws_get(c, "eg_dots", sizeof(double) * 4 * nmax);
  double* d_part = (double*)ws_get(c, "eg_part", sizeof(double) * multidot_partial_doubles(n, nmax, 2));
  double* d_coef = (double*)ws_get(c, "eg_coef", sizeof(double) * 2 * nmax);
  if (!V || !W || !T || !Tc || !U || !QU || !R || !d_dots || !d_part || !d_coef)
    return set_err(c, QMG_E_NOMEM, "out of device memory (eigensolver)");
  std::vector<double> hbuf(4 * nmax);
  const double zero_tau = 0.0;

  // ---- field helpers (one field, FP64)
  auto dots = [&](const void* Vb, int J, const void* w, std::vector<cd>& out) -> qmg_status {
    out.assign(J, cd(0));
    if (J == 0) return QMG_OK;
    hipError_t e = launch_multidot(QMG_F64, d_dots, Vb, n, J, w, n, n, 1, d_part, s, 0);
    if (e == hipSuccess) e = hipMemcpyAsync(hbuf.data(), d_dots, sizeof(double) * 2 * J, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "eigensolver dots");
    for (int j = 0; j < J; ++j) out[j] = cd(hbuf[2 * j], hbuf[2 * j + 1]);
    return QMG_OK;
  };
  auto axpy = [&](void* w, const void* Vb, int J, const std::vector<cd>& coef) -> qmg_status {
    if (J == 0) return QMG_OK;
    for (int j = 0; j < J; ++j) { hbuf[2 * j] = coef[j].real(); hbuf[2 * j + 1] = coef[j].imag(); }
    hipError_t e = hipMemcpyAsync(d_coef, hbuf.data(), sizeof(double) * 2 * J, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_multiaxpy(QMG_F64, w, Vb, n, J, d_coef, n, n, 1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // hbuf is reused by the next call
    return e == hipSuccess ? QMG_OK : hip_err(c, e, "eigensolver axpy");
  };
  auto scale = [&](void* y, const void* x, cd a) -> qmg_status {
    hbuf[0] = a.real();
    hbuf[1] = a.imag();
    hipError_t e = hipMemcpyAsync(d_coef, hbuf.data(), sizeof(double) * 2, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_scale(QMG_F64, y, x, d_coef, n, n, 1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? QMG_OK : hip_err(c, e, "eigensolver scale");
  };
  auto norm = [&](const void* x, double& out) -> qmg_status {
    std::vector<cd> d;
    qmg_status st = dots(x, 1, x, d);
    out = std::sqrt(std::max(0.0, d[0].real()));
    if (st == QMG_OK && !std::isfinite(d[0].real())) return set_err(c, QMG_E_NUMERIC, "non-finite norm (eigensolver)");
    return st;
  };
  auto applyQ = [&](void* out, const void* in) -> qmg_status {
    hipError_t e = launch_dslash(c, QMG_F64, out, in, &zero_tau, 1, 1, s);
    return e == hipSuccess ? QMG_OK : hip_err(c, e, "eigensolver apply");
  };
  auto copy = [&](void* dst, const void* src) -> qmg_status {
    hipError_t e = hipMemcpyAsync(dst, src, fb, hipMemcpyDeviceToDevice, s);
    return e == hipSuccess ? QMG_OK : hip_err(c, e, "eigensolver copy");
  };
  // x <- x - X X^H x - B B^H x by classical Gram-Schmidt; a second pass only
  // when the first removed more than half of ||x||^2 (DGKS test, the norm
  // before the pass following from the projections); returns ||x||
  int nconv = 0, m = 0;
  auto orth = [&](void* x, const void* B, int nb, double& nrm) -> qmg_status {
    std::vector<cd> d;
    for (int pass = 0; pass < 2; ++pass) {
      double removed = 0;
      if (nconv > 0) {
        qmg_status st = dots(X, nconv, x, d);
        if (st != QMG_OK) return st;
        for (cd& v : d) { removed += std::norm(v); v = -v; }
        st = axpy(x, X, nconv, d);
        if (st != QMG_OK) return st;
      }
      if (nb > 0) {
        qmg_status st = dots(B, nb, x, d);
        if (st != QMG_OK) return st;
        for (cd& v : d) { removed += std::norm(v); v = -v; }
        st = axpy(x, B, nb, d);
        if (st != QMG_OK) return st;
      }
      qmg_status st = norm(x, nrm);
      if (st != QMG_OK) return st;
      if (nrm * nrm >= 0.5 * (nrm * nrm + removed)) break;
    }
    return QMG_OK;
  };
  // small matrices (column-major, leading dimension mmax + 1)
  const int ld = mmax + 1;
  std::vector<cd> G((size_t)ld * ld), M((size_t)ld * ld);
  // XV = X^H V for eigenvectors locked since the last restart (others: 0)
  std::vector<std::vector<cd>> XV;
  // append src / nrm as v_m; W_m = Q v_m; new columns of G, M
  auto append = [&](const void* src, double nrm) -> qmg_status {
    qmg_status st = scale(fld(V, m), src, cd(1.0 / nrm));
    if (st == QMG_OK) st = applyQ(fld(W, m), fld(V, m));
    if (st != QMG_OK) return st;
    // the new columns W^H w_m and W^H v_m in one pass over W
    const int64_t wstride = ((char*)fld(V, m) - (char*)fld(W, m)) / 16;
    hipError_t e = launch_multidot_shared(QMG_F64, d_dots, W, n, m + 1, fld(W, m), wstride, 2, n, d_part, s);
    if (e == hipSuccess) e = hipMemcpyAsync(hbuf.data(), d_dots, sizeof(double) * 4 * (m + 1), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "eigensolver dots");
    std::vector<cd> gw(m + 1), mv(m + 1);
    for (int i = 0; i <= m; ++i) {
      gw[i] = cd(hbuf[2 * i], hbuf[2 * i + 1]);
      mv[i] = cd(hbuf[2 * (m + 1 + i)], hbuf[2 * (m + 1 + i) + 1]);
    }
    for (int i = 0; i <= m; ++i) {
      G[(size_t)m * ld + i] = gw[i];
      G[(size_t)i * ld + m] = std::conj(gw[i]);
      M[(size_t)m * ld + i] = mv[i];
      M[(size_t)i * ld + m] = std::conj(mv[i]);
    }
    for (auto& row : XV) row.push_back(cd(0));
    ++m;
    return QMG_OK;
  };
  auto pencil = [&](std::vector<double>& th, std::vector<std::vector<cd>>& S) -> qmg_status {
    std::vector<cd> g((size_t)m * m), mm((size_t)m * m);
    for (int j = 0; j < m; ++j)
      for (int i = 0; i < m; ++i) {
        g[(size_t)j * m + i] = G[(size_t)j * ld + i];
        mm[(size_t)j * m + i] = M[(size_t)j * ld + i];
      }
    if (prm->extraction == 1) {
      rayleigh_ritz(m, mm, th, S);
      return QMG_OK;
    }
    if (!harmonic_ritz(m, g, mm, th, S)) return set_err(c, QMG_E_NUMERIC, "W^H W is not positive definite");
    return QMG_OK;
  };
  // a harmonic Ritz vector that lies mostly in the span of locked vectors is
  // that locked eigenpair again
  auto is_locked = [&](const std::vector<cd>& sv) {
    double ov = 0;
    for (const auto& row : XV) {
      cd a = 0;  // x^H (V s) = s_x^H s, V orthonormal
      for (int i = 0; i < m; ++i) a += std::conj(row[i]) * sv[i];
      ov += std::norm(a);
    }
    return ov > 0.5;
  };
  // u = V s, Qu = W s, r = Qu - theta u (u normalised); returns ||r||
  auto ritz = [&](const std::vector<cd>& sv, double th, void* u, void* Qu, void* r, double& rn) -> qmg_status {
    hipError_t e = launch_fill_zero(u, fb, s);
    if (e == hipSuccess) e = launch_fill_zero(Qu, fb, s);
    if (e != hipSuccess) return hip_err(c, e, "eigensolver zero");
    qmg_status st = axpy(u, V, m, sv);
    if (st == QMG_OK) st = axpy(Qu, W, m, sv);
    double un = 0;
    if (st == QMG_OK) st = norm(u, un);
    if (st != QMG_OK) return st;
    if (!(un > 0)) return set_err(c, QMG_E_NUMERIC, "vanishing Ritz vector");
    if (st == QMG_OK) st = scale(u, u, cd(1.0 / un));
    if (st == QMG_OK) st = scale(Qu, Qu, cd(1.0 / un));
    if (st == QMG_OK) st = copy(r, Qu);
    if (st == QMG_OK) st = axpy(r, u, 1, std::vector<cd>{cd(-th)});
    if (st == QMG_OK) st = norm(r, rn);
    return st;
  };

  std::vector<double> lam;
  // largest |lambda| among the locked pairs (the one a smaller pair replaces)
  auto worst = [&]() {
    int w = 0;
    for (int k = 1; k < nconv; ++k)
      if (std::abs(lam[k]) > std::abs(lam[w])) w = k;
    return w;
  };
  // lock the Ritz pair (u, Qu) of coefficient vector sv: u is first made
  // orthogonal to the locked vectors (a Ritz vector formed before the last
  // lock overlaps it by about residual / gap); lambda = u^H Q u
  auto lock = [&](void* u, void* Qu, const std::vector<cd>& sv) -> qmg_status {
    double un = 0;
    qmg_status st = orth(u, nullptr, 0, un);
    if (st != QMG_OK) return st;
    if (!(un > 0)) return set_err(c, QMG_E_NUMERIC, "converged vector lies in the locked space");
    st = scale(u, u, cd(1.0 / un));
    if (st == QMG_OK) st = applyQ(Qu, u);
    std::vector<cd> rq;
    if (st == QMG_OK) st = dots(u, 1, Qu, rq);
    const int slot = nconv < nev ? nconv : worst();
    if (st == QMG_OK) st = copy(fld(X, slot), u);
    if (st != QMG_OK) return st;
    if (nconv < nev) {
      lam.push_back(rq[0].real());
      ++nconv;
    } else {
      lam[slot] = rq[0].real();
    }
    XV.push_back(sv);
    return QMG_OK;
  };

  // ---- initial space: V0 orthonormalised; the first expansion vector is t0
  for (int j = 0; j < n0 && m < mmax; ++j) {
    qmg_status st = copy(fld(Tc, 0), (const char*)V0 + (size_t)j * fb);
    double nrm = 0;
    if (st == QMG_OK) st = orth(fld(Tc, 0), V, m, nrm);
    if (st != QMG_OK) return st;
    if (nrm > 1e-10) {
      st = append(fld(Tc, 0), nrm);
      if (st != QMG_OK) return st;
    }
  }
  qmg_status st = copy(fld(Tc, 0), t0);
  if (st != QMG_OK) return st;
  int nt = 1;
  qmg_params ip = prm->solve;
  ip.tol = prm->inner_tol;
  ip.maxiter = prm->inner_maxiter;
  ip.use_graph = 0;  // every correction equation has its own shift
  ip.x0 = 0;         // correction equations start from t = 0
  int iters = 0, inner = 0, updates = 0;
  bool done = false;
  std::vector<qmg_stats> ist(ntgt);
  // QMG_PROGRESS=1: one line on stderr every 25 outer iterations (long runs)
  const char* pe = std::getenv("QMG_PROGRESS");
  const bool progress = pe && pe[0] == '1';
  while (!done && iters < prm->maxiter) {
    if (progress && iters % 25 == 0)
      std::fprintf(stderr, "[eigensolve] outer %d locked %d inner %d updates %d\n", iters, nconv, inner, updates);
    // expand with the corrections: t <- (I - V V^H)(I - X X^H) t, v_m = t / ||t||
    const int m_before = m;
    for (int j = 0; j < nt && m < mmax; ++j) {
      double nrm = 0;
      st = orth(fld(Tc, j), V, m, nrm);
      if (st != QMG_OK) return st;
      if (nrm > 1e-12) {
        st = append(fld(Tc, j), nrm);
        if (st != QMG_OK) return st;
      }
    }
    if (m == m_before) return set_err(c, QMG_E_NUMERIC, "eigensolver expansion vectors vanished");
    ++iters;
    // targets: the (up to) nblk unlocked harmonic Ritz pairs of smallest |theta|
    std::vector<double> th;
    std::vector<std::vector<cd>> S;
    std::vector<int> cand;
    std::vector<double> rns;
    bool newly_locked = false;
    while (true) {
      st = pencil(th, S);
      if (st != QMG_OK) return st;
      cand.clear();
      if (prm->both_signs) {
        // the `block` unlocked pairs of smallest |theta| of each sign, interleaved
        std::vector<int> pos, neg;
        for (size_t k = 0; k < th.size(); ++k) {
          if (is_locked(S[k])) continue;
          std::vector<int>& side = th[k] >= 0 ? pos : neg;
          if ((int)side.size() < nblk) side.push_back((int)k);
        }
        for (int q = 0; q < nblk; ++q) {
          if (q < (int)pos.size()) cand.push_back(pos[q]);
          if (q < (int)neg.size()) cand.push_back(neg[q]);
        }
        // smallest |theta| first (the verification test below looks at the first target)
        std::stable_sort(cand.begin(), cand.end(), [&](int a, int b) { return std::abs(th[a]) < std::abs(th[b]); });
      } else {
        for (size_t k = 0; k < th.size() && (int)cand.size() < nblk; ++k)
          if (!is_locked(S[k])) cand.push_back((int)k);
      }
      if (cand.empty()) return set_err(c, QMG_E_NUMERIC, "no unlocked harmonic Ritz pair");
      rns.assign(cand.size(), 0.0);
      bool relock = false;
      for (size_t i = 0; i < cand.size(); ++i) {
        // ||r||^2 = s^H G s - 2 theta Re(s^H M s) + theta^2 (V orthonormal, ||s|| = 1);
        // far from convergence only r = (W - theta V) s is formed
        const std::vector<cd>& sv = S[cand[i]];
        const double thi = th[cand[i]];
        cd sgs = 0, sms = 0;
        for (int b = 0; b < m; ++b)
          for (int a = 0; a < m; ++a) {
            sgs += std::conj(sv[a]) * G[(size_t)b * ld + a] * sv[b];
            sms += std::conj(sv[a]) * M[(size_t)b * ld + a] * sv[b];
          }
        const double est = std::sqrt(std::max(0.0, sgs.real() - 2.0 * thi * sms.real() + thi * thi));
        if (est > 100.0 * prm->tol) {
          void* ri = fld(R, (int)i);
          hipError_t e = launch_fill_zero(ri, fb, s);
          if (e != hipSuccess) return hip_err(c, e, "eigensolver zero");
          std::vector<cd> ms(m);
          for (int a = 0; a < m; ++a) ms[a] = -thi * sv[a];
          st = axpy(ri, W, m, sv);
          if (st == QMG_OK) st = axpy(ri, V, m, ms);
          if (st != QMG_OK) return st;
          rns[i] = est;
        } else {
          st = ritz(sv, thi, fld(U, (int)i), fld(QU, (int)i), fld(R, (int)i), rns[i]);
          if (st != QMG_OK) return st;
        }
        // with nev pairs locked, go on only while the first target lies below
        // the largest locked |lambda| by more than its residual (greedy
        // locking can take a slightly larger pair first); a pair that then
        // converges replaces that largest one
        if (i == 0 && nconv >= nev && std::abs(th[cand[0]]) - rns[0] >= std::abs(lam[worst()])) {
          done = true;
          break;
        }
        if (rns[i] <= prm->tol) {
          st = lock(fld(U, (int)i), fld(QU, (int)i), S[cand[i]]);
          if (st != QMG_OK) return st;
          relock = newly_locked = true;
          break;  // the candidate list changes: form it again
        }
      }
      if (done || !relock) break;
    }
    if (done) break;
    const double theta = th[cand[0]];
    // after a lock: rebuild the interpolation from the ntv converged
    // eigenvectors closest to the new target theta
    if (newly_locked && prm->update_interp && c->ntv > 0 && nconv >= c->ntv) {
      std::vector<int> idx(nconv);
      std::iota(idx.begin(), idx.end(), 0);
      std::sort(idx.begin(), idx.end(),
                [&](int a, int b) { return std::abs(lam[a] - theta) < std::abs(lam[b] - theta); });
      void* Wint = ws_get(c, "eg_int", fb * c->ntv);
      if (!Wint) return set_err(c, QMG_E_NOMEM, "out of device memory (interpolation update)");
      for (int k = 0; k < c->ntv; ++k) {
        st = copy(fld(Wint, k), fld(X, idx[k]));
        if (st != QMG_OK) return st;
      }
      st = build_mg(c, Wint, c->ntv, s);
      if (st != QMG_OK) return st;
      if (ip.use_coarse && ip.levels == 3) {
        // the third level follows the new P: its level-2 test vectors are
        // P^H w_j of the first ntv2 new test vectors (same aggregates)
        const int ntv2 = c->l3.ntv2;
        const int b2[4] = {c->l3.block2[0], c->l3.block2[1], c->l3.block2[2], c->l3.block2[3]};
        const size_t cb = coarse_elems(c) * 16;
        void* W2 = ws_get(c, "eg_w2", cb * ntv2);
        if (!W2) return set_err(c, QMG_E_NOMEM, "out of device memory (level-3 update)");
        for (int k = 0; k < ntv2; ++k) {
          hipError_t e = launch_restrict(c, QMG_F64, (char*)W2 + k * cb, fld(Wint, k), 1, s);
          if (e != hipSuccess) return hip_err(c, e, "level-3 update");
        }
        st = build_l3(c, W2, ntv2, b2, s);
        if (st != QMG_OK) return st;
      }
      ++updates;
    }
    // correction equations (Q - theta_i) t_i = r_i for all targets, as one
    // batched multi-shift solve
    nt = (int)cand.size();
    std::vector<double> taus(nt);
    for (int i = 0; i < nt; ++i) taus[i] = th[cand[i]];
    st = solver_fgmres(c, Tc, R, taus.data(), nt, &ip, ist.data(), s);
    if (st < 0) return st;
    for (int i = 0; i < nt; ++i) inner += ist[i].iters;
    // thick restart: keep the m_min unlocked harmonic Ritz vectors of smallest
    // |theta| when the next expansion would not fit
    if (m + nt > mmax) {
      st = pencil(th, S);
      if (st != QMG_OK) return st;
      // the m_min unlocked pairs of smallest |theta| (with both_signs: alternately
      // the smallest of each sign, so neither side's approximations are dropped)
      std::vector<int> keep;
      if (prm->both_signs) {
        std::vector<int> pos, neg;
        for (size_t k = 0; k < th.size(); ++k)
          if (!is_locked(S[k])) (th[k] >= 0 ? pos : neg).push_back((int)k);
        for (size_t q = 0; (int)keep.size() < mmin && (q < pos.size() || q < neg.size()); ++q) {
          if (q < pos.size() && (int)keep.size() < mmin) keep.push_back(pos[q]);
          if (q < neg.size() && (int)keep.size() < mmin) keep.push_back(neg[q]);
        }
      } else {
        for (size_t k = 0; k < th.size() && (int)keep.size() < mmin; ++k)
          if (!is_locked(S[k])) keep.push_back((int)k);
      }
      int kept = 0;
      for (int k : keep) {
        hipError_t e = launch_fill_zero(fld(T, kept), fb, s);
        if (e != hipSuccess) return hip_err(c, e, "zero");
        st = axpy(fld(T, kept), V, m, S[k]);
        if (st != QMG_OK) return st;
        ++kept;
      }
      m = 0;
      XV.clear();
      for (int k = 0; k < kept; ++k) {
        double nk = 0;
        st = orth(fld(T, k), V, m, nk);
        if (st != QMG_OK) return st;
        if (nk > 1e-10) {
          st = append(fld(T, k), nk);
          if (st != QMG_OK) return st;
        }
      }
    }
  }
  for (int k = 0; k < nconv; ++k) lambda[k] = lam[k];
  if (stats) {
    stats->iters = iters;
    stats->converged = nconv;
    stats->inner_iters = inner;
    stats->interp_updates = updates;
    stats->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - tstart).count();
  }
  return done ? QMG_OK : QMG_NOT_CONVERGED;
}
