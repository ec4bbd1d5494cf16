// Gauge-field derivative of L = phi^H Q x (Wilson hops of eq. (2.5)).
// L holds each link U_mu(y) linearly in the forward hop at y and conjugated in
// the backward hop at y + mu, so per link
//   G[y,mu]_{ab}    = -1/2 sum_s conj(phi(y)_{s,a})    (g5 (I - g_mu) x(y+mu))_{s,b}
//   Gbar[y,mu]_{ab} = -1/2 sum_s conj(phi(y+mu)_{s,b}) (g5 (I + g_mu) x(y))_{s,a}
// written in canonical order [site][mu][a][b] (complex128).
#include "qmg_ctx.h"

namespace {

__device__ Spinor<double> spin_proj_full(const Spinor<double>& p, int mu, bool fwd) {
  // (I -/+ gamma_mu) p, colour untouched, then gamma5
  Half<double> h = project(p, mu, fwd);
  Spinor<double> o;
  for (int s = 0; s < 4; ++s)
    for (int c = 0; c < 3; ++c) o.s[s][c] = czero<double>();
  accum_recon(o, h, mu, fwd);
  for (int s = 2; s < 4; ++s)
    for (int c = 0; c < 3; ++c) o.s[s][c] = -o.s[s][c];
  return o;
}

__global__ __launch_bounds__(256) void k_force(Geom g, double2* G, double2* Gb, const double2* phi, const double2* x) {
  int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  const int b = (int)(site >> g.bs_log), l = (int)(site & ((1 << g.bs_log) - 1));
  const int64_t cs = canon_site(g, b, l);
  Spinor<double> ph = load_spinor<double>(phi, g, b, l);
  Spinor<double> xx = load_spinor<double>(x, g, b, l);
  for (int mu = 0; mu < 4; ++mu) {
    int bn, ln;
    nb_fwd(g, b, l, mu, bn, ln);
    Spinor<double> y = spin_proj_full(load_spinor<double>(x, g, bn, ln), mu, true);
    Spinor<double> phn = load_spinor<double>(phi, g, bn, ln);
    Spinor<double> z = spin_proj_full(xx, mu, false);
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c) {
        cpx<double> s1 = czero<double>(), s2 = czero<double>();
        for (int s = 0; s < 4; ++s) {
          s1 = s1 + cmul_conj(ph.s[s][a], y.s[s][c]);
          s2 = s2 + cmul_conj(phn.s[s][c], z.s[s][a]);
        }
        const int64_t o = (cs * 4 + mu) * 9 + 3 * a + c;
        G[o] = make_double2(-0.5 * s1.re, -0.5 * s1.im);
        Gb[o] = make_double2(-0.5 * s2.re, -0.5 * s2.im);
      }
  }
}

__global__ void k_unit_coarse(double2* y, int nb, int nc, int col) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (int64_t)nb * nc) return;
  y[i] = make_double2((i % nc) == col ? 1.0 : 0.0, 0.0);
}

}  // namespace

hipError_t launch_force(const qmg_ctx* c, double* dU, double* dUb, const void* phi, const void* x, hipStream_t s) {
  hipLaunchKernelGGL(k_force, dim3((unsigned)((c->g.V + 255) / 256)), dim3(256), 0, s, c->g, (double2*)dU,
                     (double2*)dUb, (const double2*)phi, (const double2*)x);
  return hipGetLastError();
}

hipError_t launch_unit_coarse(void* y, int nb, int nc, int col, hipStream_t s) {
  const int64_t n = (int64_t)nb * nc;
  hipLaunchKernelGGL(k_unit_coarse, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (double2*)y, nb, nc, col);
  return hipGetLastError();
}
