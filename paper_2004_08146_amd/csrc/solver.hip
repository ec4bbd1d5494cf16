// Krylov drivers: FGMRES (outer, FP64) preconditioned by the two-level
// V-cycle (SAP smoother, aggregation coarse grid solved by GMRES), the
// multigrid setup, and the assembly of P and D_c.
//
// Outer method: right-preconditioned flexible GMRES (Sec. 2 names FGMRES with
// a multigrid preconditioner) on the Gamma5-preconditioned system
// (D - tau Gamma5) x = Gamma5 b (eq. (3.6) <=> eq. (3.7)).  Arnoldi uses
// batched classical Gram-Schmidt with a second pass when the projection
// cancels most of the vector (DGKS test); the small least-squares problems are
// solved on the host with complex Givens rotations.  Each right-hand side runs
// its own Krylov space; the batch advances in lock step within a restart
// cycle (a column that converges inside a cycle keeps being orthogonalised,
// its coefficients unused), and columns that have converged when a cycle ends
// leave the batch.
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <limits>
#include <vector>

#include "qmg_ctx.h"

using cd = std::complex<double>;

namespace {

struct Lsq {
  int m = 0;
  std::vector<cd> H, g, sn;
  std::vector<double> cs;
  void init(int m_, double beta) {
    m = m_;
    H.assign((size_t)(m + 1) * m, cd(0));
    g.assign(m + 1, cd(0));
    g[0] = beta;
    cs.assign(m, 0.0);
    sn.assign(m, cd(0));
  }
  // add Hessenberg column j (h has j+2 entries); returns |g[j+1]|
  double update(int j, std::vector<cd> h) {
    for (int i = 0; i < j; ++i) {
      cd t = cs[i] * h[i] + sn[i] * h[i + 1];
      h[i + 1] = -std::conj(sn[i]) * h[i] + cs[i] * h[i + 1];
      h[i] = t;
    }
    double c;
    cd s;
    const cd a = h[j], b = h[j + 1];
    if (b == cd(0)) { c = 1.0; s = 0.0; }
    else if (a == cd(0)) { c = 0.0; s = 1.0; }
    else {
      const double rho = std::sqrt(std::norm(a) + std::norm(b));
      c = std::abs(a) / rho;
      s = (a / std::abs(a)) * std::conj(b) / rho;
    }
    cs[j] = c;
    sn[j] = s;
    h[j] = c * h[j] + s * h[j + 1];
    h[j + 1] = 0.0;
    g[j + 1] = -std::conj(s) * g[j];
    g[j] = c * g[j];
    for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = h[i];
    return std::abs(g[j + 1]);
  }
  std::vector<cd> solve(int k) const {
    std::vector<cd> y(k);
    for (int i = k - 1; i >= 0; --i) {
      cd t = g[i];
      for (int l = i + 1; l < k; ++l) t -= H[(size_t)i * m + l] * y[l];
      y[i] = t / H[(size_t)i * m + i];
    }
    return y;
  }
};

// squared norm ratio below which a second Gram-Schmidt pass is made
constexpr double kReorthRatio2 = 0.05 * 0.05;

double* host_buf(qmg_ctx* c, const std::string& name, size_t ndouble) {
  auto& v = c->hbuf[name];
  if (v.size() < ndouble) v.resize(ndouble);
  return v.data();
}

// batched vector space helper (n complex per vector, nrhs vectors per batch)
struct Space {
  qmg_ctx* c;
  int p;
  int64_t n;
  int nrhs;
  hipStream_t s;
  size_t vbytes() const { return (size_t)n * cbytes(p); }
  size_t bbytes() const { return vbytes() * nrhs; }
  char* at(void* base, int j) const { return (char*)base + (size_t)j * bbytes(); }
  int64_t vstride() const { return n * nrhs; }

  // out[k*J + j] = <V_j,k, w_k>
  qmg_status dots(std::vector<cd>& out, const void* V, int J, int64_t vstr, const void* w) {
    double* d = (double*)ws_get(c, "sp_dots", sizeof(double) * 2 * J * nrhs);
    double* part = (double*)ws_get(c, "sp_part", sizeof(double) * multidot_partial_doubles(n, J, nrhs));
    if (!d || !part) return set_err(c, QMG_E_NOMEM, "out of device memory (dots)");
    hipError_t e = launch_multidot(p, d, V, vstr, J, w, n, n, nrhs, part, s);
    if (e != hipSuccess) return hip_err(c, e, "multidot");
    double* h = host_buf(c, "dots", 2 * J * nrhs);
    e = hipMemcpyAsync(h, d, sizeof(double) * 2 * J * nrhs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "dots D2H");
    out.resize((size_t)J * nrhs);
    for (int i = 0; i < J * nrhs; ++i) out[i] = cd(h[2 * i], h[2 * i + 1]);
    return QMG_OK;
  }
  qmg_status norms(std::vector<double>& out, const void* w) {
    std::vector<cd> d;
    qmg_status st = dots(d, w, 1, 0, w);
    if (st != QMG_OK) return st;
    out.resize(nrhs);
    for (int k = 0; k < nrhs; ++k) {
      const double v = d[k].real();  // NaN/Inf must survive to the callers' checks
      out[k] = std::isfinite(v) ? std::sqrt(std::max(0.0, v)) : std::numeric_limits<double>::quiet_NaN();
    }
    return QMG_OK;
  }
  // w_k += sum_j coef[k*J + j] V_j,k
  qmg_status axpy(void* w, const void* V, int J, int64_t vstr, const std::vector<cd>& coef, int vprec = -1) {
    double* d = (double*)ws_get(c, "sp_coef", sizeof(double) * 2 * J * nrhs);
    if (!d) return set_err(c, QMG_E_NOMEM, "out of device memory (coef)");
    double* h = host_buf(c, "coef", 2 * J * nrhs);
    for (int i = 0; i < J * nrhs; ++i) { h[2 * i] = coef[i].real(); h[2 * i + 1] = coef[i].imag(); }
    hipError_t e = hipMemcpyAsync(d, h, sizeof(double) * 2 * J * nrhs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = (vprec < 0 || vprec == p) ? launch_multiaxpy(p, w, V, vstr, J, d, n, n, nrhs, s)
                                    : launch_multiaxpy_d(w, V, vprec, vstr, J, d, n, n, nrhs, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);  // host coef buffer is reused next call
    if (e != hipSuccess) return hip_err(c, e, "axpy");
    return QMG_OK;
  }
  qmg_status scale(void* y, const void* x, const std::vector<cd>& a, void* copy = nullptr, int copy_prec = QMG_F64) {
    double* d = (double*)ws_get(c, "sp_scale", sizeof(double) * 2 * nrhs);
    if (!d) return set_err(c, QMG_E_NOMEM, "out of device memory (scale)");
    double* h = host_buf(c, "scale", 2 * nrhs);
    for (int k = 0; k < nrhs; ++k) { h[2 * k] = a[k].real(); h[2 * k + 1] = a[k].imag(); }
    hipError_t e = hipMemcpyAsync(d, h, sizeof(double) * 2 * nrhs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_scale(p, y, x, d, n, n, nrhs, s, copy, copy_prec);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "scale");
    return QMG_OK;
  }
  // One Arnoldi step on basis V_0..V_j with new vector w; h[k] gets j+2 entries.
  // Classical Gram-Schmidt with a DGKS-type test: a second pass is made when the
  // projection cancelled so much of some column that ||w_new|| < 0.05 ||w||.
  // One pass leaves an orthogonality error of about eps ||w|| / ||w_new||
  // (<= 20 eps here); the true residual is recomputed after every restart
  // cycle anyway.  The new norm comes out of the update pass.
  // sig (optional, [nrhs][j + 1]): the basis is stored unnormalised, v_i = sig_i W_i,
  // so the projections use sig_i (W_i^H w) and the update subtracts sig_i^2 (W_i^H w) W_i.
  // copy (optional): the update pass also writes the new w there in copy_prec.
  qmg_status arnoldi(std::vector<std::vector<cd>>& h, void* V, int j, void* w,
                     const std::vector<std::vector<double>>* sig = nullptr, void* copy = nullptr,
                     int copy_prec = QMG_F64) {
    const int J = j + 1;
    h.assign(nrhs, std::vector<cd>(j + 2, cd(0)));
    double* d = (double*)ws_get(c, "sp_dots", sizeof(double) * 2 * (J + 1) * nrhs);
    double* part = (double*)ws_get(c, "sp_part", sizeof(double) * multidot_partial_doubles(n, J + 1, nrhs));
    double* dc = (double*)ws_get(c, "sp_coef", sizeof(double) * 2 * J * nrhs);
    if (!d || !part || !dc) return set_err(c, QMG_E_NOMEM, "out of device memory (Arnoldi)");
    double* hd = host_buf(c, "dots", 2 * (J + 1) * nrhs);
    double* hc = host_buf(c, "coef", 2 * J * nrhs);
    std::vector<double> before(nrhs), after(nrhs);
    for (int pass = 0; pass < 2; ++pass) {
      const int self = pass == 0 ? 1 : 0;
      hipError_t e = launch_multidot(p, d, V, vstride(), J, w, n, n, nrhs, part, s, self);
      if (e == hipSuccess) e = hipMemcpyAsync(hd, d, sizeof(double) * 2 * (J + self) * nrhs, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_err(c, e, "Arnoldi dots");
      for (int k = 0; k < nrhs; ++k) {
        for (int i = 0; i < J; ++i) {
          const double* q = hd + 2 * ((size_t)k * (J + self) + i);
          const double si = sig ? (*sig)[k][i] : 1.0;
          h[k][i] += si * cd(q[0], q[1]);
          hc[2 * ((size_t)k * J + i)] = -si * si * q[0];
          hc[2 * ((size_t)k * J + i) + 1] = -si * si * q[1];
        }
        if (self) before[k] = hd[2 * ((size_t)k * (J + 1) + J)];
      }
      e = hipMemcpyAsync(dc, hc, sizeof(double) * 2 * J * nrhs, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = launch_axpy_norm(p, w, V, vstride(), J, dc, n, n, nrhs, d, part, s, copy, copy_prec);
      if (e == hipSuccess) e = hipMemcpyAsync(hd, d, sizeof(double) * 2 * nrhs, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return hip_err(c, e, "Arnoldi update");
      bool again = false;
      for (int k = 0; k < nrhs; ++k) {
        after[k] = hd[2 * k];
        if (!std::isfinite(after[k]) || !std::isfinite(before[k]))
          return set_err(c, QMG_E_NUMERIC, "non-finite norm in Arnoldi step");
        if (after[k] < kReorthRatio2 * before[k]) again = true;
        before[k] = after[k];
      }
      if (!again) break;
    }
    for (int k = 0; k < nrhs; ++k) h[k][j + 1] = std::sqrt(std::max(0.0, after[k]));
    return QMG_OK;
  }
  // The last Arnoldi step of a restart cycle. Its new vector is never used (the
  // next cycle starts from the true residual), so only the projections h and
  // the norm of the projected part are formed: one pass gives W_i^H w and
  // ||w||^2, and ||w - sum_i h_i v_i||^2 = ||w||^2 - sum_i |h_i|^2 with the v_i
  // orthonormal. The subtraction loses about eps ||w||^2 / ||w_new||^2 in
  // relative accuracy, which only perturbs this cycle's last rotation.
  qmg_status arnoldi_last(std::vector<std::vector<cd>>& h, void* V, int j, void* w,
                          const std::vector<std::vector<double>>* sig = nullptr) {
    const int J = j + 1;
    h.assign(nrhs, std::vector<cd>(j + 2, cd(0)));
    double* d = (double*)ws_get(c, "sp_dots", sizeof(double) * 2 * (J + 1) * nrhs);
    double* part = (double*)ws_get(c, "sp_part", sizeof(double) * multidot_partial_doubles(n, J + 1, nrhs));
    if (!d || !part) return set_err(c, QMG_E_NOMEM, "out of device memory (Arnoldi)");
    double* hd = host_buf(c, "dots", 2 * (J + 1) * nrhs);
    hipError_t e = launch_multidot(p, d, V, vstride(), J, w, n, n, nrhs, part, s, 1);
    if (e == hipSuccess) e = hipMemcpyAsync(hd, d, sizeof(double) * 2 * (J + 1) * nrhs, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "Arnoldi dots");
    for (int k = 0; k < nrhs; ++k) {
      double proj = 0.0;
      for (int i = 0; i < J; ++i) {
        const double* q = hd + 2 * ((size_t)k * (J + 1) + i);
        const double si = sig ? (*sig)[k][i] : 1.0;
        h[k][i] = si * cd(q[0], q[1]);
        proj += std::norm(h[k][i]);
      }
      const double ww = hd[2 * ((size_t)k * (J + 1) + J)];
      if (!std::isfinite(ww) || !std::isfinite(proj)) return set_err(c, QMG_E_NUMERIC, "non-finite norm in Arnoldi step");
      h[k][j + 1] = std::sqrt(std::max(0.0, ww - proj));
    }
    return QMG_OK;
  }
};

}  // namespace

// ------------------------------------------------------------ coarse GMRES --
qmg_status solver_coarse_gmres(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int iters,
                               double tol, int* iters_done, hipStream_t s, int qform) {
  const int cp = coarse_prec(p);
  Space sp{c, cp, (int64_t)coarse_elems(c), nrhs, s};
  if (iters < 1) iters = 1;
  void* V = ws_get(c, "cg_V", sp.bbytes() * (iters + 1));
  void* w = ws_get(c, "cg_w", sp.bbytes());
  if (!V || !w) return set_err(c, QMG_E_NOMEM, "out of device memory (coarse GMRES)");
  std::vector<double> beta;
  qmg_status st = sp.norms(beta, r);
  if (st != QMG_OK) return st;
  std::vector<cd> a(nrhs);
  std::vector<Lsq> lsq(nrhs);
  std::vector<char> act(nrhs);
  for (int k = 0; k < nrhs; ++k) {
    if (!std::isfinite(beta[k])) return set_err(c, QMG_E_NUMERIC, "non-finite coarse right-hand side");
    act[k] = beta[k] > 0;
    a[k] = act[k] ? 1.0 / beta[k] : 0.0;
    lsq[k].init(iters, beta[k]);
  }
  st = sp.scale(sp.at(V, 0), r, a);
  if (st != QMG_OK) return st;
  std::vector<int> kk(nrhs, 0);
  int done_it = 0;
  for (int j = 0; j < iters; ++j) {
    hipError_t e = launch_coarse_apply(c, p, w, sp.at(V, j), tau, nrhs, s, qform);
    if (e != hipSuccess) return hip_err(c, e, "coarse apply");
    std::vector<std::vector<cd>> h;
    st = sp.arnoldi(h, V, j, w);
    if (st != QMG_OK) return st;
    bool all = true;
    for (int k = 0; k < nrhs; ++k) {
      if (!act[k]) { a[k] = 0.0; continue; }
      double est = lsq[k].update(j, h[k]);
      kk[k] = j + 1;
      const double hn = h[k][j + 1].real();
      if (hn == 0.0 || (tol > 0 && est <= tol * beta[k])) act[k] = 0;
      a[k] = act[k] ? 1.0 / hn : 0.0;
      all = all && !act[k];
    }
    done_it = j + 1;
    if (all || j + 1 == iters) break;
    st = sp.scale(sp.at(V, j + 1), w, a);
    if (st != QMG_OK) return st;
  }
  int J = 0;
  for (int k = 0; k < nrhs; ++k) J = std::max(J, kk[k]);
  hipError_t e = launch_fill_zero(y, sp.bbytes(), s);
  if (e != hipSuccess) return hip_err(c, e, "zero");
  if (J > 0) {
    std::vector<cd> coef((size_t)J * nrhs, cd(0));
    for (int k = 0; k < nrhs; ++k) {
      if (kk[k] == 0) continue;
      std::vector<cd> yk = lsq[k].solve(kk[k]);
      for (int i = 0; i < kk[k]; ++i) coef[(size_t)k * J + i] = yk[i];
    }
    st = sp.axpy(y, V, J, sp.vstride(), coef);
    if (st != QMG_OK) return st;
  }
  if (iters_done) *iters_done = done_it;
  return QMG_OK;
}

// ----------------------------------------------------------------- V-cycle --
// graph_safe: the coarse GMRES runs a fixed number of steps with its scalars on
// the device, so the whole V-cycle is a pure kernel sequence (no host sync).
static qmg_status vcycle_body(qmg_ctx* c, void* z, const void* r, const double* tau, int nrhs, const qmg_params* prm,
                              int* coarse_iters, hipStream_t s, bool graph_safe, int zprec, int rprec);

qmg_status solver_vcycle(qmg_ctx* c, void* z, const void* r, const double* tau, int nrhs, const qmg_params* prm,
                         int* coarse_iters, hipStream_t s, int zprec, int rprec) {
  if (zprec != QMG_F64 && zprec != prm->mg_prec) return set_err(c, QMG_E_ARG, "V-cycle output precision");
  if (rprec != QMG_F64 && rprec != prm->mg_prec) return set_err(c, QMG_E_ARG, "V-cycle input precision");
  if (!prm->use_graph) return vcycle_body(c, z, r, tau, nrhs, prm, coarse_iters, s, false, zprec, rprec);
  // HIP-graph mode: capture the V-cycle once per (buffers, shifts, parameters) and replay it
  std::string key;
  {
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%p|%p|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|%d|", z, r, nrhs, prm->nu_post,
                  prm->n_mr, prm->coarse_maxiter, (int)prm->mg_prec, prm->use_coarse, zprec, rprec, prm->q_form,
                  prm->smoother, prm->levels, prm->l3_iters, prm->l2_smooth);
    key = buf;
    for (int k = 0; k < nrhs; ++k) {
      std::snprintf(buf, sizeof(buf), "%.17g,", tau[k]);
      key += buf;
    }
  }
  if (coarse_iters && prm->use_coarse && c->have_mg) *coarse_iters += prm->coarse_maxiter;
  auto it = c->graphs.find(key);
  if (it != c->graphs.end()) {
    hipError_t e = hipGraphLaunch(it->second, s);
    return e == hipSuccess ? QMG_OK : hip_err(c, e, "graph launch");
  }
  // first use: run eagerly on the caller's stream (this also sizes every
  // workspace buffer), then record the same sequence on the library's own
  // stream (the caller's stream may be the legacy default stream, which
  // cannot be captured); the recorded graph is later launched on `s`.
  qmg_status st = vcycle_body(c, z, r, tau, nrhs, prm, nullptr, s, true, zprec, rprec);
  if (st != QMG_OK) return st;
  hipError_t e = hipSuccess;
  if (!c->cap_stream) e = hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "capture stream");
  const uint64_t epoch = c->ws_epoch;
  hipGraph_t graph = nullptr;
  e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_err(c, e, "begin capture");
  st = vcycle_body(c, z, r, tau, nrhs, prm, nullptr, c->cap_stream, true, zprec, rprec);
  e = hipStreamEndCapture(c->cap_stream, &graph);
  if (st != QMG_OK) {
    if (graph) hipGraphDestroy(graph);
    return st;
  }
  if (e != hipSuccess) return hip_err(c, e, "end capture");
  if (c->ws_epoch != epoch) {  // a buffer moved while recording: do not keep this graph
    hipGraphDestroy(graph);
    return set_err(c, QMG_E_HIP, "workspace changed during V-cycle capture");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_err(c, e, "graph instantiate");
  c->graphs[key] = exec;
  return QMG_OK;
}

static qmg_status vcycle_body(qmg_ctx* c, void* z, const void* r, const double* tau, int nrhs, const qmg_params* prm,
                              int* coarse_iters, hipStream_t s, bool graph_safe, int zprec, int rprec) {
  const int p = prm->mg_prec;
  const int64_t n = (int64_t)field_elems(c);
  void* rp = (void*)r;
  void* zp = z;
  hipError_t e;
  if (p != QMG_F64) {
    // an input already in the preconditioner's precision is read in place (the
    // V-cycle only reads r)
    if (rprec != p) rp = ws_get(c, "vc_r", (size_t)n * nrhs * cbytes(p));
    // with zprec == p the result is written straight into z
    if (zprec != p) zp = ws_get(c, "vc_z", (size_t)n * nrhs * cbytes(p));
    if (!rp || !zp) return set_err(c, QMG_E_NOMEM, "out of device memory (V-cycle)");
    if (rprec != p) {
      e = launch_convert(rp, p, r, QMG_F64, n * nrhs, s);
      if (e != hipSuccess) return hip_err(c, e, "convert");
    }
  }
  if (prm->use_coarse && c->have_mg) {
    const int cp = coarse_prec(p);
    const size_t cb = coarse_elems(c) * cbytes(cp) * nrhs;
    void* rc = ws_get(c, "vc_rc", cb);
    void* yc = ws_get(c, "vc_yc", cb);
    if (!rc || !yc) return set_err(c, QMG_E_NOMEM, "out of device memory (V-cycle)");
    e = launch_restrict(c, p, rc, rp, nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "restrict");
    int it = 0;
    // a fixed number of coarse steps (graph mode, or coarse_tol <= 0) runs the
    // device-resident GMRES, which never waits for the host; three levels
    // always take coarse_maxiter K-cycle steps on level 2
    const bool three = prm->levels == 3;
    const bool fixed = three || graph_safe || !(prm->coarse_tol > 0);
    qmg_status st =
        three ? level2_kcycle(c, p, yc, rc, tau, nrhs, prm->coarse_maxiter, prm->l3_iters, prm->l2_smooth, s,
                              prm->q_form)
        : fixed ? coarse_gmres_device(c, p, yc, rc, tau, nrhs, prm->coarse_maxiter, s, prm->q_form)
                : solver_coarse_gmres(c, p, yc, rc, tau, nrhs, prm->coarse_maxiter, prm->coarse_tol, &it, s,
                                      prm->q_form);
    if (st != QMG_OK) return st;
    if (fixed) it = prm->coarse_maxiter;
    if (coarse_iters) *coarse_iters += it;
    e = launch_prolong(c, p, zp, yc, nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "prolong");
  } else {
    e = launch_fill_zero(zp, (size_t)n * nrhs * cbytes(p), s);
    if (e != hipSuccess) return hip_err(c, e, "zero");
  }
  if (prm->smoother == 1 && prm->nu_post > 0) {
    // GMRES smoothing (Sec. 2's alternative to SAP): nu_post fixed GMRES steps
    // from zero on A e = r - A z, then z += e (A = D - tau Gamma5, or Q - tau)
    void* az = ws_get(c, "vc_az", (size_t)n * nrhs * cbytes(p));
    void* ez = ws_get(c, "vc_ez", (size_t)n * nrhs * cbytes(p));
    if (!az || !ez) return set_err(c, QMG_E_NOMEM, "out of device memory (GMRES smoother)");
    e = launch_dslash(c, p, az, zp, tau, nrhs, prm->q_form ? 1 : 0, s);
    if (e == hipSuccess) e = launch_xmy(p, az, rp, n, n, nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "smoother residual");
    qmg_status st = fine_gmres_device(c, p, ez, az, tau, nrhs, prm->nu_post, s, prm->q_form);
    if (st != QMG_OK) return st;
    e = launch_add(p, zp, ez, n, n, nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "smoother update");
  } else {
    for (int sw = 0; sw < prm->nu_post; ++sw)
      for (int col = 0; col < 2; ++col) {
        e = launch_sap_colour(c, p, zp, rp, tau, nrhs, col, prm->n_mr, s, prm->q_form);
        if (e != hipSuccess) return hip_err(c, e, "sap");
      }
  }
  if (p != QMG_F64 && zprec != p) {
    e = launch_convert(z, QMG_F64, zp, p, n * nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "convert");
  }
  return QMG_OK;
}

// ------------------------------------------------------------------ FGMRES --
// Columns that have converged when a restart cycle ends are dropped from the
// batch: the next cycles run on the unconverged columns only (gathered to the
// front of library buffers; every column is an independent system, so its
// arithmetic does not depend on which others share the batch), and each
// column's x is written back to the caller's x when it leaves the batch.
qmg_status solver_fgmres(qmg_ctx* c, void* x, const void* b, const double* tau, int nrhs, const qmg_params* prm,
                         qmg_stats* stats, hipStream_t s) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = std::max(1, prm->restart);
  const int64_t n = (int64_t)field_elems(c);
  const size_t fb = (size_t)n * 16;  // one FP64 field
  const size_t bb = fb * nrhs;
  // the preconditioned directions Z are kept in the preconditioner's own
  // precision: the V-cycle output is exact there, so the FP64 products read it
  // unchanged and half (or a quarter) of the bytes
  const int zprec = prm->mg_prec;
  const size_t zb_full = (size_t)n * nrhs * cbytes(zprec);
  void* V = ws_get(c, "fg_V", bb * (m + 1));
  void* Z = ws_get(c, "fg_Z", zb_full * m);
  void* f = ws_get(c, "fg_f", bb);
  void* r = ws_get(c, "fg_r", bb);
  // a reduced-precision V-cycle reads its input in its own precision: the
  // Gram-Schmidt update writes that copy of the next basis vector as it writes
  // the FP64 one, which saves the V-cycle a conversion pass over the FP64 vector
  const bool vin = prm->mg_prec != QMG_F64;
  void* vc_in = vin ? ws_get(c, "fg_vin", zb_full) : nullptr;
  if (!V || !Z || !f || !r || (vin && !vc_in)) return set_err(c, QMG_E_NOMEM, "out of device memory (FGMRES)");
  // Gamma5-preconditioned form: (D - tau Gamma5) x = Gamma5 b; q_form: (Q - tau) x = b itself
  const int mode = prm->q_form ? 1 : 0;
  hipError_t e = prm->q_form ? hipMemcpyAsync(f, b, bb, hipMemcpyDeviceToDevice, s)
                             : launch_gamma5_bs(QMG_F64, f, b, n * nrhs, c->g.bs_log, s);
  if (e == hipSuccess && !prm->x0) e = launch_fill_zero(x, bb, s);
  if (prm->x0) {
    // initial guess from the caller: r = Gamma5 b - A_tau x (or b - (Q - tau) x)
    if (e == hipSuccess) e = launch_dslash(c, QMG_F64, r, x, tau, nrhs, mode, s);
    if (e == hipSuccess) e = launch_xmy(QMG_F64, r, f, n, n, nrhs, s);
  } else if (e == hipSuccess) {
    e = hipMemcpyAsync(r, f, bb, hipMemcpyDeviceToDevice, s);
  }
  if (e != hipSuccess) return hip_err(c, e, "fgmres init");
  std::vector<double> bnorm;
  {
    Space sp0{c, QMG_F64, n, nrhs, s};
    qmg_status st = sp0.norms(bnorm, b);
    if (st != QMG_OK) return st;
  }
  for (int k = 0; k < nrhs; ++k)
    if (!std::isfinite(bnorm[k])) return set_err(c, QMG_E_NUMERIC, "non-finite right-hand side");
  std::vector<int> iters(nrhs, 0), restarts(nrhs, 0), cits(nrhs, 0);
  std::vector<double> relres(nrhs, 0.0), rnorm(nrhs, 0.0);
  std::vector<std::vector<double>> hist(nrhs);
  std::vector<char> done(nrhs, 0);
  // phase timing: four events per Arnoldi step (before the V-cycle, after it,
  // after the product, after the Gram-Schmidt), read once the solve has synchronised
  std::vector<hipEvent_t> evs;
  struct EvPool {
    std::vector<hipEvent_t>& v;
    ~EvPool() { for (hipEvent_t e : v) (void)hipEventDestroy(e); }
  } ev_pool{evs};
  auto mark = [&]() -> hipError_t {
    hipEvent_t ev;
    hipError_t er = hipEventCreate(&ev);
    if (er != hipSuccess) return er;
    evs.push_back(ev);
    return hipEventRecord(ev, s);
  };
  // the working batch: na columns, column i is the caller's column cols[i]
  int na = nrhs;
  std::vector<int> cols(nrhs);
  for (int k = 0; k < nrhs; ++k) cols[k] = k;
  std::vector<double> tw(tau, tau + nrhs);
  void *xw = x, *fw = f, *rw = r;
  auto col = [&](void* base, int i) { return (char*)base + (size_t)i * fb; };
  int total = 0;
  qmg_status st = QMG_OK;
  while (true) {
    Space sp{c, QMG_F64, n, na, s};
    std::vector<double> beta;
    st = sp.norms(beta, rw);
    if (st != QMG_OK) return st;
    std::vector<char> act(na);
    int nact = 0;
    for (int i = 0; i < na; ++i) {
      if (!std::isfinite(beta[i])) return set_err(c, QMG_E_NUMERIC, "non-finite residual");
      const int k = cols[i];
      rnorm[k] = beta[i];
      relres[k] = bnorm[k] > 0 ? beta[i] / bnorm[k] : 0.0;
      act[i] = relres[k] > prm->tol;
      nact += act[i];
      if (!done[k]) hist[k].push_back(relres[k]);
      if (!act[i]) done[k] = 1;
    }
    if (nact == 0 || total >= prm->maxiter) break;
    if (nact <= (3 * na) / 4) {
      // drop the converged columns: their x goes home, the others move to the front
      void* xa = ws_get(c, "fg_xa", bb);
      void* fa = ws_get(c, "fg_fa", bb);
      void* ra = ws_get(c, "fg_ra", bb);
      if (!xa || !fa || !ra) return set_err(c, QMG_E_NOMEM, "out of device memory (FGMRES compaction)");
      int j = 0;
      std::vector<int> ncols;
      std::vector<double> ntw;
      for (int i = 0; i < na && e == hipSuccess; ++i) {
        if (!act[i]) {
          if (xw != x) e = hipMemcpyAsync(col(x, cols[i]), col(xw, i), fb, hipMemcpyDeviceToDevice, s);
          continue;
        }
        // destination index j <= i: moving front to back in order never overwrites a pending column
        if (xw != xa || j != i) {
          e = hipMemcpyAsync(col(xa, j), col(xw, i), fb, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipMemcpyAsync(col(fa, j), col(fw, i), fb, hipMemcpyDeviceToDevice, s);
          if (e == hipSuccess) e = hipMemcpyAsync(col(ra, j), col(rw, i), fb, hipMemcpyDeviceToDevice, s);
        }
        ncols.push_back(cols[i]);
        ntw.push_back(tw[i]);
        ++j;
      }
      if (e != hipSuccess) return hip_err(c, e, "fgmres compaction");
      xw = xa;
      fw = fa;
      rw = ra;
      cols = ncols;
      tw = ntw;
      na = j;
      act.assign(na, 1);
      sp.nrhs = na;
    }
    const size_t zb = (size_t)n * na * cbytes(zprec);
    auto zat = [&](int jj) { return (void*)((char*)Z + (size_t)jj * zb); };
    std::vector<cd> a(na);
    std::vector<Lsq> lsq(na);
    for (int i = 0; i < na; ++i) {
      a[i] = act[i] ? 1.0 / rnorm[cols[i]] : 0.0;
      lsq[i].init(m, rnorm[cols[i]]);
      if (act[i]) restarts[cols[i]] += 1;
    }
    // the first basis vector, and the V-cycle's reduced-precision copy of it
    st = sp.scale(sp.at(V, 0), rw, a, vc_in, zprec);
    if (st != QMG_OK) return st;
    // basis vectors after the first stay unnormalised (v_j = sig_j W_j): the
    // product A z_j is orthogonalised in place in the next basis slot, and the
    // preconditioner takes W_j itself (flexible GMRES allows any z_j)
    std::vector<std::vector<double>> sig(na, std::vector<double>(m + 1, 0.0));
    for (int i = 0; i < na; ++i) sig[i][0] = 1.0;
    std::vector<int> kk(na, 0);
    for (int jj = 0; jj < m; ++jj) {
      int ci = 0;
      void* w = sp.at(V, jj + 1);
      e = mark();
      if (e != hipSuccess) return hip_err(c, e, "event");
      st = vin ? solver_vcycle(c, zat(jj), vc_in, tw.data(), na, prm, &ci, s, zprec, zprec)
               : solver_vcycle(c, zat(jj), sp.at(V, jj), tw.data(), na, prm, &ci, s, zprec);
      if (st != QMG_OK) return st;
      e = mark();
      if (e == hipSuccess) e = launch_dslash_d_in(c, w, zat(jj), zprec, tw.data(), na, s, mode);
      if (e == hipSuccess) e = mark();
      if (e != hipSuccess) return hip_err(c, e, "apply");
      std::vector<std::vector<cd>> h;
      // the last step of a restart cycle that another cycle follows keeps no new
      // basis vector (and has no next V-cycle); a step at which maxiter ends the
      // solve keeps the full update, so short inner solves (the eigensolver's
      // correction equations) are unchanged by this shortcut
      const bool last = jj + 1 == m && total + 1 < prm->maxiter;
      st = last ? sp.arnoldi_last(h, V, jj, w, &sig) : sp.arnoldi(h, V, jj, w, &sig, vin ? vc_in : nullptr, zprec);
      if (st != QMG_OK) return st;
      e = mark();
      if (e != hipSuccess) return hip_err(c, e, "event");
      bool all = true;
      for (int i = 0; i < na; ++i) {
        if (!act[i]) { a[i] = 0.0; continue; }
        double est = lsq[i].update(jj, h[i]);
        kk[i] = jj + 1;
        iters[cols[i]] += 1;
        cits[cols[i]] += ci;
        const double hn = h[i][jj + 1].real();
        if (hn == 0.0 || est <= prm->tol * bnorm[cols[i]]) act[i] = 0;
        all = all && !act[i];
      }
      // converged right-hand sides are orthogonalised like the others, so their
      // vectors stay bounded; their coefficients are no longer used
      for (int i = 0; i < na; ++i) {
        const double hn = h[i][jj + 1].real();
        sig[i][jj + 1] = (hn > 0.0 && std::isfinite(hn)) ? 1.0 / hn : 0.0;
      }
      ++total;
      if (all || jj + 1 == m || total >= prm->maxiter) break;
    }
    int J = 0;
    for (int i = 0; i < na; ++i) J = std::max(J, kk[i]);
    if (J > 0) {
      std::vector<cd> coef((size_t)J * na, cd(0));
      for (int i = 0; i < na; ++i) {
        if (kk[i] == 0) continue;
        std::vector<cd> yk = lsq[i].solve(kk[i]);
        for (int l = 0; l < kk[i]; ++l) {
          if (!std::isfinite(yk[l].real()) || !std::isfinite(yk[l].imag()))
            return set_err(c, QMG_E_NUMERIC, "non-finite least-squares solution");
          coef[(size_t)i * J + l] = yk[l];
        }
      }
      st = sp.axpy(xw, Z, J, sp.vstride(), coef, zprec);
      if (st != QMG_OK) return st;
    }
    // true residual r = Gamma5 b - A_tau x
    e = launch_dslash(c, QMG_F64, rw, xw, tw.data(), na, mode, s);
    if (e == hipSuccess) e = launch_xmy(QMG_F64, rw, fw, n, n, na, s);
    if (e != hipSuccess) return hip_err(c, e, "residual");
  }
  // columns still in a compacted batch go home
  if (xw != x)
    for (int i = 0; i < na && e == hipSuccess; ++i)
      e = hipMemcpyAsync(col(x, cols[i]), col(xw, i), fb, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "sync");
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  double ph[3] = {0.0, 0.0, 0.0};
  for (size_t i = 0; i + 3 < evs.size(); i += 4)
    for (int q = 0; q < 3; ++q) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, evs[i + q], evs[i + q + 1]) == hipSuccess) ph[q] += 1e-3 * ms;
    }
  bool conv = true;
  for (int k = 0; k < nrhs; ++k) {
    conv = conv && relres[k] <= prm->tol;
    if (stats) {
      stats[k].iters = iters[k];
      stats[k].restarts = restarts[k];
      stats[k].coarse_iters = cits[k];
      stats[k].true_relres = relres[k];
      stats[k].seconds = secs;
      stats[k].vcycle_seconds = ph[0];
      stats[k].apply_seconds = ph[1];
      stats[k].orth_seconds = ph[2];
      const int nh = (int)std::min<size_t>(hist[k].size(), QMG_STATS_HIST);
      stats[k].n_hist = nh;
      for (int i = 0; i < QMG_STATS_HIST; ++i) stats[k].relres_hist[i] = i < nh ? hist[k][i] : 0.0;
    }
  }
  return conv ? QMG_OK : QMG_NOT_CONVERGED;
}

// ---------------------------------------------------- P and D_c assembly --
qmg_status build_mg(qmg_ctx* c, const void* W, int ntv, hipStream_t s) {
  const Geom& g = c->g;
  const int nc = 2 * ntv;
  const size_t pel = (size_t)g.nb * 2 * ntv * 6 * ((size_t)1 << g.bs_log);
  const size_t del = (size_t)g.nb * 5 * nc * nc;  // self + 4 forward blocks per coarse site
  c->have_mg = false;
  c->l3.ok = false;  // the third level is built on D_c
  c->ntv = ntv;
  drop_graphs(c);
  for (int p = 0; p < 3; ++p) {
    const std::string ps = std::to_string(p);
    c->P[p] = ws_get(c, "mg_P" + ps, pel * cbytes(p));
    c->Dc[p] = ws_get(c, "mg_Dc" + ps, del * cbytes(p));
    if (!c->P[p] || !c->Dc[p]) return set_err(c, QMG_E_NOMEM, "out of device memory (P, D_c)");
  }
  int* fail = (int*)ws_get(c, "mg_fail", sizeof(int));
  if (!fail) return set_err(c, QMG_E_NOMEM, "out of device memory");
  hipError_t e = hipMemsetAsync(fail, 0, sizeof(int), s);
  if (e == hipSuccess) e = launch_build_P(c, c->P[QMG_F64], W, ntv, fail, s);
  int hfail = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "build P");
  if (hfail) return set_err(c, QMG_E_NUMERIC, "test vectors are locally rank deficient");
  // D_c column by column, kb columns per batch (workspace capped near 8 GiB):
  // one multi-rhs prolongation and one multi-rhs restriction per batch read P
  // once per 16 right-hand sides instead of once per part
  const size_t fb = field_elems(c) * 16, cb = coarse_elems(c) * 16;
  const int K = (int)std::max<size_t>(1, std::min<size_t>((size_t)nc, ((size_t)8 << 30) / (6 * fb)));
  void* ycol = ws_get(c, "mg_ycol", cb * K);
  void* pcol = ws_get(c, "mg_pcol", fb * K);
  void* five = ws_get(c, "mg_five", fb * 5 * K);
  void* part = ws_get(c, "mg_part", cb * 5 * K);
  if (!ycol || !pcol || !five || !part) return set_err(c, QMG_E_NOMEM, "out of device memory (D_c assembly)");
  for (int c0 = 0; c0 < nc; c0 += K) {
    const int kb = std::min(K, nc - c0);
    for (int kk = 0; kk < kb && e == hipSuccess; ++kk) e = launch_unit_coarse((char*)ycol + kk * cb, g.nb, nc, c0 + kk, s);
    if (e == hipSuccess) e = launch_prolong(c, QMG_F64, pcol, ycol, kb, s);
    for (int kk = 0; kk < kb && e == hipSuccess; ++kk)
      e = launch_split_stencil(c, (char*)five + (size_t)kk * 5 * fb, (char*)pcol + (size_t)kk * fb, s);
    if (e == hipSuccess) e = launch_restrict(c, QMG_F64, part, five, 5 * kb, s);
    if (e == hipSuccess) e = launch_scatter_dc(c, c->Dc[QMG_F64], part, c0, kb, s);
    if (e != hipSuccess) return hip_err(c, e, "assemble D_c");
  }
  for (int p = 1; p < 3; ++p) {
    e = launch_convert(c->P[p], p, c->P[QMG_F64], QMG_F64, (int64_t)pel, s);
    if (e == hipSuccess) e = launch_convert(c->Dc[p], p, c->Dc[QMG_F64], QMG_F64, (int64_t)del, s);
    if (e != hipSuccess) return hip_err(c, e, "convert P/D_c");
  }
  e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "sync");
  c->have_mg = true;
  return QMG_OK;
}

// ------------------------------------------------------------------- setup --
// Reading of the paper's setup parameters (test vectors, setup iterations,
// smoothing steps): smooth random W on D w = 0 with SAP, then repeat
// V-cycle inverse iteration (tau = 0), rebuilding P and D_c after each round.
qmg_status solver_setup(qmg_ctx* c, void* W, int ntv, int iters, int smooth, int n_mr, int kc, double ctol,
                        int prec, hipStream_t s) {
  const int64_t n = (int64_t)field_elems(c);
  const size_t fb = (size_t)n * 16;
  Space sp{c, QMG_F64, n, ntv, s};
  std::vector<double> tau0(ntv, 0.0);
  void* zero = ws_get(c, "su_zero", fb * ntv);
  if (!zero) return set_err(c, QMG_E_NOMEM, "out of device memory (setup)");
  hipError_t e = launch_fill_zero(zero, fb * ntv, s);
  if (e != hipSuccess) return hip_err(c, e, "zero");
  for (int sw = 0; sw < smooth; ++sw)
    for (int col = 0; col < 2; ++col) {
      e = launch_sap_colour(c, QMG_F64, W, zero, tau0.data(), ntv, col, n_mr, s);
      if (e != hipSuccess) return hip_err(c, e, "setup sap");
    }
  auto normalise = [&](void* X) -> qmg_status {
    std::vector<double> nn;
    qmg_status st = sp.norms(nn, X);
    if (st != QMG_OK) return st;
    std::vector<cd> a(ntv);
    for (int k = 0; k < ntv; ++k) {
      if (!(nn[k] > 0) || !std::isfinite(nn[k])) return set_err(c, QMG_E_NUMERIC, "setup vector vanished");
      a[k] = 1.0 / nn[k];
    }
    return sp.scale(X, X, a);
  };
  qmg_status st = normalise(W);
  if (st != QMG_OK) return st;
  st = build_mg(c, W, ntv, s);
  if (st != QMG_OK) return st;
  qmg_params prm = qmg_default_params();
  prm.nu_post = smooth;
  prm.n_mr = n_mr;
  prm.coarse_maxiter = kc;
  prm.coarse_tol = ctol;
  prm.mg_prec = (qmg_prec)prec;
  prm.use_coarse = 1;
  void* Wn = ws_get(c, "su_new", fb * ntv);
  if (!Wn) return set_err(c, QMG_E_NOMEM, "out of device memory (setup)");
  for (int it = 1; it < iters; ++it) {
    st = solver_vcycle(c, Wn, W, tau0.data(), ntv, &prm, nullptr, s);
    if (st != QMG_OK) return st;
    st = normalise(Wn);
    if (st != QMG_OK) return st;
    e = hipMemcpyAsync(W, Wn, fb * ntv, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_err(c, e, "copy");
    st = build_mg(c, W, ntv, s);
    if (st != QMG_OK) return st;
  }
  ws_release(c, "su_zero");
  ws_release(c, "su_new");
  ws_release(c, "mg_five");
  ws_release(c, "mg_pcol");
  return QMG_OK;
}
