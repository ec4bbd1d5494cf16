// Gauge field packing and the clover term (plus mass) per site.
//
// The clover term follows the Sheikholeslami-Wohlert form the paper cites for
// its large configurations (Sec. 4): C = csw (i/4) sum_{mu,nu} sigma_{mu nu}
// (x) Fhat_{mu nu}, with Fhat = (Q_{mu nu} - Q_{mu nu}^H)/8 from the four
// counter-clockwise plaquettes ("leaves") at x, made traceless.  In the chiral
// basis sigma_{mu nu} is block diagonal; writing the chirality +/- blocks as
// sigma_l (x) M_l gives, per chirality, the 6x6 matrix
//   [[M3, M1 - i M2], [M1 + i M2, -M3]],  M_l = (i csw / 2) B_l,
//   B1 = +-F01 - F23,  B2 = +-F02 + F13,  B3 = +-F03 - F12,
// and (m0 + 4) is added on the diagonal.
#include "qmg_ctx.h"

namespace {

struct M3 { cpx<double> m[3][3]; };

__device__ M3 mmul(const M3& a, const M3& b) {
  M3 o;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      o.m[i][j] = a.m[i][0] * b.m[0][j] + a.m[i][1] * b.m[1][j] + a.m[i][2] * b.m[2][j];
  return o;
}
__device__ M3 mdag(const M3& a) {
  M3 o;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o.m[i][j] = conj(a.m[j][i]);
  return o;
}
__device__ M3 madd(const M3& a, const M3& b) {
  M3 o;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) o.m[i][j] = a.m[i][j] + b.m[i][j];
  return o;
}
__device__ M3 ldl(const double2* U, const Geom& g, int b, int mu, int l) {
  M3 o;
  for (int a = 0; a < 3; ++a)
    for (int c = 0; c < 3; ++c) o.m[a][c] = ldc(U, uidx(g, b, mu, 3 * a + c, l));
  return o;
}

__global__ __launch_bounds__(256) void k_pack_gauge(Geom g, double2* U, const double2* canon) {
  int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  int b = (int)(site >> g.bs_log), l = (int)(site & ((1 << g.bs_log) - 1));
  int64_t cs = canon_site(g, b, l);
  for (int mu = 0; mu < 4; ++mu)
    for (int ab = 0; ab < 9; ++ab) U[uidx(g, b, mu, ab, l)] = canon[(cs * 4 + mu) * 9 + ab];
}

// Fhat_{mu nu}(x), traceless
__device__ M3 fhat(const double2* U, const Geom& g, int b, int l, int mu, int nu) {
  int bpm, lpm, bpn, lpn, bmm, lmm, bmn, lmn, bx, lx;
  nb_fwd(g, b, l, mu, bpm, lpm);   // x+mu
  nb_fwd(g, b, l, nu, bpn, lpn);   // x+nu
  nb_bwd(g, b, l, mu, bmm, lmm);   // x-mu
  nb_bwd(g, b, l, nu, bmn, lmn);   // x-nu
  M3 umu = ldl(U, g, b, mu, l), unu = ldl(U, g, b, nu, l);
  // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H
  M3 q = mmul(mmul(umu, ldl(U, g, bpm, nu, lpm)), mmul(mdag(ldl(U, g, bpn, mu, lpn)), mdag(unu)));
  // leaf 2: U_nu(x) U_mu(x-mu+nu)^H U_nu(x-mu)^H U_mu(x-mu)
  nb_fwd(g, bmm, lmm, nu, bx, lx);  // x-mu+nu
  M3 umu_m = ldl(U, g, bmm, mu, lmm);
  q = madd(q, mmul(mmul(unu, mdag(ldl(U, g, bx, mu, lx))), mmul(mdag(ldl(U, g, bmm, nu, lmm)), umu_m)));
  // leaf 3: U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu)
  nb_bwd(g, bmm, lmm, nu, bx, lx);  // x-mu-nu
  M3 unu_m = ldl(U, g, bmn, nu, lmn);
  q = madd(q, mmul(mmul(mdag(umu_m), mdag(ldl(U, g, bx, nu, lx))), mmul(ldl(U, g, bx, mu, lx), unu_m)));
  // leaf 4: U_nu(x-nu)^H U_mu(x-nu) U_nu(x-nu+mu) U_mu(x)^H
  nb_fwd(g, bmn, lmn, mu, bx, lx);  // x-nu+mu
  q = madd(q, mmul(mmul(mdag(unu_m), ldl(U, g, bmn, mu, lmn)), mmul(ldl(U, g, bx, nu, lx), mdag(umu))));
  M3 f;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) f.m[i][j] = 0.125 * (q.m[i][j] - conj(q.m[j][i]));
  cpx<double> tr = (1.0 / 3.0) * (f.m[0][0] + f.m[1][1] + f.m[2][2]);
  for (int i = 0; i < 3; ++i) f.m[i][i] = f.m[i][i] - tr;
  return f;
}

__global__ __launch_bounds__(128) void k_clover(Geom g, double2* Dg, const double2* U, double mass4,
                                                double csw) {
  int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  int b = (int)(site >> g.bs_log), l = (int)(site & ((1 << g.bs_log) - 1));
  M3 F01 = fhat(U, g, b, l, 0, 1), F02 = fhat(U, g, b, l, 0, 2), F03 = fhat(U, g, b, l, 0, 3);
  M3 F12 = fhat(U, g, b, l, 1, 2), F13 = fhat(U, g, b, l, 1, 3), F23 = fhat(U, g, b, l, 2, 3);
  for (int h = 0; h < 2; ++h) {
    double sg = h == 0 ? 1.0 : -1.0;
    cpx<double> A[6][6];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cpx<double> b1 = sg * F01.m[i][j] - F23.m[i][j];
        cpx<double> b2 = sg * F02.m[i][j] + F13.m[i][j];
        cpx<double> b3 = sg * F03.m[i][j] - F12.m[i][j];
        // M_l = (i csw/2) B_l
        cpx<double> m1 = (0.5 * csw) * ti(b1), m2 = (0.5 * csw) * ti(b2), m3 = (0.5 * csw) * ti(b3);
        A[i][j] = m3;
        A[3 + i][3 + j] = -m3;
        A[i][3 + j] = m1 - ti(m2);
        A[3 + i][j] = m1 + ti(m2);
      }
    for (int i = 0; i < 6; ++i) A[i][i].re += mass4;
    for (int k = 0; k < 3; ++k)
      Dg[didx(g, b, h, k, l)] = make_double2(A[2 * k][2 * k].re, A[2 * k + 1][2 * k + 1].re);
    int k = 3;
    for (int i = 1; i < 6; ++i)
      for (int j = 0; j < i; ++j) Dg[didx(g, b, h, k++, l)] = make_double2(A[i][j].re, A[i][j].im);
  }
}

}  // namespace

hipError_t launch_pack_gauge(const Geom& g, void* U64, const double* canon, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_gauge, dim3((unsigned)((g.V + 255) / 256)), dim3(256), 0, s, g, (double2*)U64,
                     (const double2*)canon);
  return hipGetLastError();
}

hipError_t launch_clover(const Geom& g, void* diag64, const void* U64, double m0, double csw, hipStream_t s) {
  hipLaunchKernelGGL(k_clover, dim3((unsigned)((g.V + 127) / 128)), dim3(128), 0, s, g, (double2*)diag64,
                     (const double2*)U64, m0 + 4.0, csw);
  return hipGetLastError();
}
