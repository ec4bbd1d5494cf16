// Device-resident GMRES scalars (Hessenberg column, Givens rotations,
// back-substitution) so a fixed-step coarse GMRES -- and with it the whole
// V-cycle -- runs without host round trips and can be captured in a HIP graph.
// The same driver runs the GMRES smoother on the fine level and, with a third
// level, the level-3 GMRES and the level-2 flexible GMRES (K-cycle).
// Being part of the preconditioner, this coarse GMRES makes a single classical
// Gram-Schmidt pass per step (no data-dependent second pass).  The basis is
// stored unnormalised after its first vector (v_j = sig_j W_j, W_j the stored
// vector): each product is orthogonalised in place in the next basis slot, so
// no scaling pass is needed, and the last step, whose new vector is never used,
// takes ||w_new||^2 = ||w||^2 - sum_i |v_i^H w|^2 from its dot pass instead of
// an update pass.
// One thread per right-hand side; the rotations follow the same convention as
// the host solver: [[c, s], [-conj(s), c]] [a; b] = [r; 0], c real.
#include <functional>
#include <string>

#include "qmg_ctx.h"

namespace {

struct GmState {
  double* H;     // [nrhs][m+1][m] complex (row-major: (i, j) at i*m + j)
  double* g;     // [nrhs][m+1] complex
  double* cs;    // [nrhs][m]
  double* sn;    // [nrhs][m] complex
  double* beta;  // [nrhs]
  double* sig;   // [nrhs][m+1]: v_j = sig_j W_j
  int m;
};

__device__ inline cpx<double> ldz(const double* p, int64_t i) { return {p[2 * i], p[2 * i + 1]}; }
__device__ inline void stz(double* p, int64_t i, cpx<double> v) { p[2 * i] = v.re; p[2 * i + 1] = v.im; }

// beta = ||r||, a = 1/beta (0 if beta == 0), g = (beta, 0, ...), H = 0
__global__ void k_gm_init(GmState st, const double* norms, double* a, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  const double b = sqrt(fmax(norms[2 * k], 0.0));
  st.beta[k] = b;
  a[2 * k] = b > 0 ? 1.0 / b : 0.0;
  a[2 * k + 1] = 0.0;
  const int m = st.m;
  for (int i = 0; i <= m; ++i) stz(st.g, (int64_t)k * (m + 1) + i, cpx<double>{i == 0 ? b : 0.0, 0.0});
  for (int i = 0; i < (m + 1) * m; ++i) stz(st.H, (int64_t)k * (m + 1) * m + i, czero<double>());
  for (int i = 0; i <= m; ++i) st.sig[(int64_t)k * (m + 1) + i] = i == 0 ? 1.0 : 0.0;
}

// one classical Gram-Schmidt pass for w = A W_j, d_i = W_i^H w:
// H[i][j] = sig_i sig_j d_i, coef_i = -sig_i^2 d_i (w -= (v_i^H w) v_i).
// last: dots also holds ||w||^2 (at index J), and norms[2k] gets the squared
// norm of the projected w, ||w||^2 - sum_i sig_i^2 |d_i|^2, in place of the
// update pass
__global__ void k_gm_coef(GmState st, const double* dots, double* coef, int j, int nrhs, int last,
                          double* norms) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  const int J = j + 1, m = st.m, ld = J + (last ? 1 : 0);
  const double* sg = st.sig + (int64_t)k * (m + 1);
  double proj = 0.0;
  for (int i = 0; i < J; ++i) {
    const cpx<double> d = ldz(dots, (int64_t)k * ld + i);
    const int64_t hi = (int64_t)k * (m + 1) * m + (int64_t)i * m + j;
    stz(st.H, hi, ldz(st.H, hi) + (sg[i] * sg[j]) * d);
    stz(coef, (int64_t)k * J + i, -(sg[i] * sg[i]) * d);
    proj += sg[i] * sg[i] * norm2(d);
  }
  if (last) {
    norms[2 * k] = fmax(dots[2 * ((int64_t)k * ld + J)] - proj, 0.0);
    norms[2 * k + 1] = 0.0;
  }
}

// close column j: h_{j+1,j} = sig_j ||w_new|| (w_new = the projected A W_j,
// stored as W_{j+1}, so sig_{j+1} = 1 / ||w_new||), rotate, update g
__global__ void k_gm_col(GmState st, const double* norms, int j, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  const int m = st.m;
  double* H = st.H + (int64_t)k * (m + 1) * m * 2;
  double* g = st.g + (int64_t)k * (m + 1) * 2;
  double* cs = st.cs + (int64_t)k * m;
  double* sn = st.sn + (int64_t)k * m * 2;
  double* sg = st.sig + (int64_t)k * (m + 1);
  const double wn = sqrt(fmax(norms[2 * k], 0.0));
  const double hn = sg[j] * wn;
  sg[j + 1] = wn > 0 ? 1.0 / wn : 0.0;
  cpx<double> h[2];
  for (int i = 0; i < j; ++i) {
    const cpx<double> hi = ldz(H, (int64_t)i * m + j), hi1 = ldz(H, (int64_t)(i + 1) * m + j);
    const double c = cs[i];
    const cpx<double> s = ldz(sn, i);
    stz(H, (int64_t)i * m + j, c * hi + s * hi1);
    stz(H, (int64_t)(i + 1) * m + j, c * hi1 - conj(s) * hi);
  }
  h[0] = ldz(H, (int64_t)j * m + j);
  h[1] = cpx<double>{hn, 0.0};
  double c;
  cpx<double> s;
  const double na = sqrt(norm2(h[0])), nb = hn;
  if (nb == 0.0) { c = 1.0; s = czero<double>(); }
  else if (na == 0.0) { c = 0.0; s = cpx<double>{1.0, 0.0}; }
  else {
    const double rho = sqrt(na * na + nb * nb);
    c = na / rho;
    s = (1.0 / (na * rho)) * (h[0] * conj(h[1]));
  }
  cs[j] = c;
  stz(sn, j, s);
  stz(H, (int64_t)j * m + j, c * h[0] + s * h[1]);
  const cpx<double> gj = ldz(g, j);
  stz(g, j + 1, -(conj(s) * gj));
  stz(g, j, c * gj);
}

// y = R^{-1} g (R: the rotated Hessenberg, kk columns) -> coef[k][0..kk)
__global__ void k_gm_solve(GmState st, double* coef, int kk, int nrhs) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nrhs) return;
  const int m = st.m;
  const double* H = st.H + (int64_t)k * (m + 1) * m * 2;
  const double* g = st.g + (int64_t)k * (m + 1) * 2;
  for (int i = kk - 1; i >= 0; --i) {
    cpx<double> t = ldz(g, i);
    for (int l = i + 1; l < kk; ++l) t = t - ldz(H, (int64_t)i * m + l) * ldz(coef, (int64_t)k * kk + l);
    const cpx<double> d = ldz(H, (int64_t)i * m + i);
    const double dd = norm2(d);
    // a zero pivot only follows an exact breakdown; that column adds nothing
    stz(coef, (int64_t)k * kk + i, dd > 0 ? cpx<double>{(t.re * d.re + t.im * d.im) / dd, (t.im * d.re - t.re * d.im) / dd}
                                         : czero<double>());
  }
  // y_i multiplies v_i = sig_i W_i (or M v_i = sig_i Z_i): coefficients of the stored vectors
  const double* sg = st.sig + (int64_t)k * (m + 1);
  for (int i = 0; i < kk; ++i) stz(coef, (int64_t)k * kk + i, sg[i] * ldz(coef, (int64_t)k * kk + i));
}

}  // namespace

// The operator of a device GMRES run: n complex elements per right-hand side
// in storage precision cp; prec set: flexible GMRES, right-preconditioned by
// prec (the preconditioned directions are kept and form the update).
struct DevOp {
  int64_t n;
  int cp;
  std::string tag;  // workspace name prefix (nested runs need distinct tags)
  std::function<hipError_t(void* out, const void* in)> apply;
  std::function<qmg_status(void* z, const void* v)> prec;
};

// Fixed-step (F)GMRES from zero with every scalar on the device
// (graph-capturable).  Work buffers come from ws (allocate them before a
// capture with the same sizes).
static qmg_status gmres_device(qmg_ctx* c, const DevOp& op, void* y, const void* r, int nrhs, int iters,
                               hipStream_t s) {
  const int cp = op.cp;
  const int64_t n = op.n;
  const size_t vb = (size_t)n * cbytes(cp);
  const size_t bb = vb * nrhs;
  const int m = iters;
  const std::string& tag = op.tag;
  const bool flex = (bool)op.prec;
  void* V = ws_get(c, tag + "_V", bb * (m + 1));
  void* Z = flex ? ws_get(c, tag + "_Z", bb * m) : nullptr;
  double* dots = (double*)ws_get(c, tag + "_dots", sizeof(double) * 2 * (m + 2) * nrhs);
  double* part = (double*)ws_get(c, tag + "_part", sizeof(double) * multidot_partial_doubles(n, m + 2, nrhs));
  double* coef = (double*)ws_get(c, tag + "_coef", sizeof(double) * 2 * (m + 1) * nrhs);
  double* a = (double*)ws_get(c, tag + "_a", sizeof(double) * 2 * nrhs);
  double* nrm = (double*)ws_get(c, tag + "_nrm", sizeof(double) * 2 * nrhs);
  GmState st;
  st.m = m;
  st.H = (double*)ws_get(c, tag + "_H", sizeof(double) * 2 * (m + 1) * m * nrhs);
  st.g = (double*)ws_get(c, tag + "_g", sizeof(double) * 2 * (m + 1) * nrhs);
  st.cs = (double*)ws_get(c, tag + "_cs", sizeof(double) * m * nrhs);
  st.sn = (double*)ws_get(c, tag + "_sn", sizeof(double) * 2 * m * nrhs);
  st.beta = (double*)ws_get(c, tag + "_beta", sizeof(double) * nrhs);
  st.sig = (double*)ws_get(c, tag + "_sig", sizeof(double) * (m + 1) * nrhs);
  if (!V || (flex && !Z) || !dots || !part || !coef || !a || !nrm || !st.H || !st.g || !st.cs || !st.sn ||
      !st.beta || !st.sig)
    return set_err(c, QMG_E_NOMEM, "out of device memory (device GMRES)");
  const dim3 g1((nrhs + 63) / 64), b1(64);
  const int64_t vs = n * nrhs;
  hipError_t e = launch_multidot(cp, nrm, r, 0, 0, r, n, n, nrhs, part, s, 1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gm_init, g1, b1, 0, s, st, nrm, a, nrhs);
    e = launch_scale(cp, V, r, a, n, n, nrhs, s);
  }
  for (int j = 0; j < m && e == hipSuccess; ++j) {
    char* Vj = (char*)V + (size_t)j * bb;
    char* w = Vj + bb;  // the product is orthogonalised in place in slot j + 1
    const int last = j + 1 == m ? 1 : 0;
    if (flex) {
      char* Zj = (char*)Z + (size_t)j * bb;
      qmg_status ps = op.prec(Zj, Vj);
      if (ps != QMG_OK) return ps;
      e = op.apply(w, Zj);
    } else {
      e = op.apply(w, Vj);
    }
    if (e == hipSuccess) e = launch_multidot(cp, dots, V, vs, j + 1, w, n, n, nrhs, part, s, last);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_gm_coef, g1, b1, 0, s, st, dots, coef, j, nrhs, last, nrm);
      if (!last) e = launch_axpy_norm(cp, w, V, vs, j + 1, coef, n, n, nrhs, nrm, part, s);
    }
    if (e == hipSuccess) hipLaunchKernelGGL(k_gm_col, g1, b1, 0, s, st, nrm, j, nrhs);
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_gm_solve, g1, b1, 0, s, st, coef, m, nrhs);
    e = launch_fill_zero(y, bb, s);
  }
  if (e == hipSuccess) e = launch_multiaxpy(cp, y, flex ? Z : V, vs, m, coef, n, n, nrhs, s);
  if (e != hipSuccess) return hip_err(c, e, "device GMRES");
  return QMG_OK;
}

// GMRES on the coarse operator (coarse precision of p); shares its basis
// buffers with the host-driven coarse GMRES (never live at the same time)
qmg_status coarse_gmres_device(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int iters,
                               hipStream_t s, int qform) {
  DevOp op{(int64_t)coarse_elems(c), coarse_prec(p), "cg",
           [=](void* out, const void* in) { return launch_coarse_apply(c, p, out, in, tau, nrhs, s, qform); }, {}};
  return gmres_device(c, op, y, r, nrhs, iters, s);
}

// GMRES on the fine stencil in precision p (the smoother of Sec. 2's GMRES option)
qmg_status fine_gmres_device(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int iters,
                             hipStream_t s, int qform) {
  DevOp op{(int64_t)field_elems(c), p, "fs",
           [=](void* out, const void* in) { return launch_dslash(c, p, out, in, tau, nrhs, qform ? 1 : 0, s); }, {}};
  return gmres_device(c, op, y, r, nrhs, iters, s);
}

// ---- third level.  M2 r2 = z: P2 y3 with y3 from k3 GMRES steps on
// A3(tau) y3 = P2^H r2, then s2 GMRES steps from zero on A_c e = r2 - A_c z
// and z + e.  Level-2 and level-3 vectors are in the coarse precision of p.
qmg_status level2_cycle(qmg_ctx* c, int p, void* z, const void* r, const double* tau, int nrhs, int k3, int s2,
                        hipStream_t s, int qform) {
  const int cp = coarse_prec(p);
  const int64_t n2 = (int64_t)coarse_elems(c), n3 = (int64_t)l3_elems(c);
  void* r3 = ws_get(c, "l3_r", (size_t)n3 * nrhs * cbytes(cp));
  void* y3 = ws_get(c, "l3_y", (size_t)n3 * nrhs * cbytes(cp));
  if (!r3 || !y3) return set_err(c, QMG_E_NOMEM, "out of device memory (level-2 cycle)");
  hipError_t e = launch_restrict_l3(c, p, r3, r, nrhs, s);
  if (e != hipSuccess) return hip_err(c, e, "restrict to level 3");
  DevOp op3{n3, cp, "l3g",
            [=](void* out, const void* in) { return launch_apply_l3(c, p, out, in, tau, nrhs, s, qform); }, {}};
  qmg_status st = gmres_device(c, op3, y3, r3, nrhs, k3, s);
  if (st != QMG_OK) return st;
  e = launch_prolong_l3(c, p, z, y3, nrhs, s);
  if (e != hipSuccess) return hip_err(c, e, "prolong from level 3");
  if (s2 > 0) {
    void* az = ws_get(c, "l2_az", (size_t)n2 * nrhs * cbytes(cp));
    void* ez = ws_get(c, "l2_ez", (size_t)n2 * nrhs * cbytes(cp));
    if (!az || !ez) return set_err(c, QMG_E_NOMEM, "out of device memory (level-2 smoothing)");
    e = launch_coarse_apply(c, p, az, z, tau, nrhs, s, qform);
    if (e == hipSuccess) e = launch_xmy(cp, az, r, n2, n2, nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "level-2 smoothing residual");
    st = coarse_gmres_device(c, p, ez, az, tau, nrhs, s2, s, qform);
    if (st != QMG_OK) return st;
    e = launch_add(cp, z, ez, n2, n2, nrhs, s);
    if (e != hipSuccess) return hip_err(c, e, "level-2 smoothing update");
  }
  return QMG_OK;
}

// k2 FGMRES steps from zero on A_c(tau) y = r, right-preconditioned by M2
// (a K-cycle on level 2)
qmg_status level2_kcycle(qmg_ctx* c, int p, void* y, const void* r, const double* tau, int nrhs, int k2, int k3,
                         int s2, hipStream_t s, int qform) {
  DevOp op{(int64_t)coarse_elems(c), coarse_prec(p), "kc",
           [=](void* out, const void* in) { return launch_coarse_apply(c, p, out, in, tau, nrhs, s, qform); },
           [=](void* z, const void* v) { return level2_cycle(c, p, z, v, tau, nrhs, k3, s2, s, qform); }};
  return gmres_device(c, op, y, r, nrhs, k2, s);
}
