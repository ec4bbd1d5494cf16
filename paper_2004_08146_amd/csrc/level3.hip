// Third multigrid level: aggregates of level-2 sites (the lattice blocks),
// the interpolation P2 from level-2 test vectors, the Galerkin level-3
// operator D3 = P2^H D_c P2 and the level-2 <-> level-3 transfers.  The
// construction repeats the first coarse level's one level down (Sec. 2 on
// aggregation, Sec. 3.1 on P from test vectors): every aggregate is split by
// coarse chirality (components 0..ntv-1 of a level-2 site have Gamma5^c = +1,
// the others -1, so Gamma5^c P2 = P2 Gamma5^cc), and the ntv2 columns of each
// (aggregate, chirality) are the test vectors restricted to it, orthonormalised
// by modified Gram-Schmidt in column order, twice per column.
//
// Layouts: level-2 vectors [nrhs][nb][2 ntv] (the first coarse level's);
// level-3 vectors [nrhs][n3][2 ntv2], index h*ntv2 + j; P2 complex
// [n3][2][bs2*ntv][ntv2], row q*ntv + i = component i of the chirality half of
// the aggregate's q-th level-2 site, columns fastest.  Aggregates are numbered
// lexicographically by aggregate coordinate, the sites inside one
// lexicographically too.  D3 is stored like D_c: D3T[a][d][j][i] = D3[a][d]_{ij},
// d = 0 self, 1 + 2 mu the aggregate at A + mu, 2 + 2 mu at A - mu.
#include <vector>

#include "qmg_ctx.h"
#include "reduce.h"

namespace {

constexpr int kMaxRows = 4;  // P2 rows per thread of the 256-thread build kernel
constexpr int kMaxOut = 9;   // D3 entries per thread of the assembly kernel (2 ntv2 <= 48)

struct L3Tab {
  const int* sites;
  const int* agg;
  const int* qloc;
  const int* keep;
  const int* nbr2;
  int n3, bs2, ntv, ntv2, nb;
};

L3Tab tab_of(const qmg_ctx* c) {
  const Level3& l = c->l3;
  return L3Tab{l.sites, l.agg, l.qloc, l.keep, c->g.nbr, l.n3, l.bs2, c->ntv, l.ntv2, c->g.nb};
}

// one work-group per (aggregate, chirality)
__global__ __launch_bounds__(256) void k_build_P2(L3Tab t, double2* P2, const double2* W2, int64_t wstride,
                                                  int* fail) {
  __shared__ double red[8];
  const int a = blockIdx.x >> 1, h = blockIdx.x & 1;
  const int L = t.bs2 * t.ntv, nc = 2 * t.ntv;
  double2* P = P2 + ((int64_t)a * 2 + h) * L * t.ntv2;
  for (int j = 0; j < t.ntv2; ++j) {
    cpx<double> v[kMaxRows];
    double n0[1] = {0.0};
#pragma unroll
    for (int m = 0; m < kMaxRows; ++m) {
      const int e = threadIdx.x + 256 * m;
      v[m] = czero<double>();
      if (e < L) {
        const int q = e / t.ntv, i = e - q * t.ntv;
        v[m] = ldc(W2 + j * wstride, (int64_t)t.sites[a * t.bs2 + q] * nc + h * t.ntv + i);
        n0[0] += norm2(v[m]);
      }
    }
    wg_sum<double, 1>(n0, red);
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        double cf[2] = {0.0, 0.0};
#pragma unroll
        for (int m = 0; m < kMaxRows; ++m) {
          const int e = threadIdx.x + 256 * m;
          if (e < L) {
            const cpx<double> s = cmul_conj(ldc(P, (int64_t)e * t.ntv2 + i), v[m]);
            cf[0] += s.re;
            cf[1] += s.im;
          }
        }
        wg_sum<double, 2>(cf, red);
        const cpx<double> cc = {cf[0], cf[1]};
#pragma unroll
        for (int m = 0; m < kMaxRows; ++m) {
          const int e = threadIdx.x + 256 * m;
          if (e < L) v[m] = v[m] - cc * ldc(P, (int64_t)e * t.ntv2 + i);
        }
      }
    double n1[1] = {0.0};
#pragma unroll
    for (int m = 0; m < kMaxRows; ++m) n1[0] += norm2(v[m]);
    wg_sum<double, 1>(n1, red);
    double nn = sqrt(n1[0]);
    if (!(nn >= 1e-12 * sqrt(n0[0]))) {
      if (threadIdx.x == 0) fail[0] = 1;
      nn = 1.0;
    }
    const double inv = 1.0 / nn;
#pragma unroll
    for (int m = 0; m < kMaxRows; ++m) {
      const int e = threadIdx.x + 256 * m;
      if (e < L) stc(P, (int64_t)e * t.ntv2 + j, inv * v[m]);
    }
  }
}

// D3[a][e] = sum over the (q, d) with site b = sites[a][q] and stencil entry d
// landing in block e of P2_b^H D_c[b][d] P2_{b'}, b' = nbr(b, d); one
// work-group per (aggregate, stored block), T = D_c[b][d] P2_{b'} staged in LDS.
// Like D_c, D3 keeps the self block and the 4 forward blocks (stored index
// blockIdx.y = 0 self, 1 + mu forward; stencil entry eblk = 0 or 1 + 2 mu): the
// backward ones follow from Gamma5^cc D3 Gamma5^cc = D3^H.  D_c's backward
// blocks are rebuilt from the forward block of the neighbour at X - mu:
// D_c[b][2 + 2 mu]_{r,col} = g_r g_col conj(F_{col,r}).
__global__ __launch_bounds__(256) void k_assemble_D3(L3Tab t, double2* D3T, const double2* DcT, const double2* P2) {
  extern __shared__ unsigned char smem_d3[];
  cpx<double>* T = reinterpret_cast<cpx<double>*>(smem_d3);  // [nc3][nc2]
  const int a = blockIdx.x, eout = blockIdx.y, eblk = eout == 0 ? 0 : 2 * eout - 1;
  const int ntv = t.ntv, ntv2 = t.ntv2, nc2 = 2 * ntv, nc3 = 2 * ntv2, L = t.bs2 * ntv;
  cpx<double> acc[kMaxOut];
#pragma unroll
  for (int m = 0; m < kMaxOut; ++m) acc[m] = czero<double>();
  for (int q = 0; q < t.bs2; ++q) {
    const int b = t.sites[a * t.bs2 + q];
    for (int d = 0; d < 9; ++d) {
      // uniform over the work-group: the same (b, d) for every thread
      if ((t.keep[b * 9 + d] ? 0 : d) != eblk) continue;
      const int bn = d == 0 ? b : t.nbr2[b * 8 + d - 1];
      const int an = t.agg[bn], qn = t.qloc[bn];
      const bool back = d > 0 && (d & 1) == 0;
      // forward/self: D_c[b][d]_{r,col} at col * nc2 + r; backward: F_{col,r} of the
      // forward block of bn at r * nc2 + col
      const double2* Dm = back ? DcT + ((int64_t)bn * 5 + d / 2) * nc2 * nc2
                               : DcT + ((int64_t)b * 5 + (d + 1) / 2) * nc2 * nc2;
      __syncthreads();
      for (int idx = threadIdx.x; idx < nc2 * nc3; idx += 256) {
        const int r = idx % nc2, cc = idx / nc2;
        const int hn = cc / ntv2, jn = cc - hn * ntv2;
        const double2* Pn = P2 + (((int64_t)an * 2 + hn) * L + (int64_t)qn * ntv) * ntv2 + jn;
        cpx<double> s = czero<double>();
        if (back) {
          // g_r g_col with col = hn ntv + i2: the sign of col is that of hn
          const double g = ((r < ntv) == (hn == 0)) ? 1.0 : -1.0;
          for (int i2 = 0; i2 < ntv; ++i2)
            cfma(s, g * conj(ldc(Dm, (int64_t)r * nc2 + hn * ntv + i2)), ldc(Pn, (int64_t)i2 * ntv2));
        } else {
          for (int i2 = 0; i2 < ntv; ++i2)
            cfma(s, ldc(Dm, (int64_t)(hn * ntv + i2) * nc2 + r), ldc(Pn, (int64_t)i2 * ntv2));
        }
        T[idx] = s;
      }
      __syncthreads();
#pragma unroll
      for (int m = 0; m < kMaxOut; ++m) {
        const int o = threadIdx.x + 256 * m;
        if (o < nc3 * nc3) {
          const int row = o % nc3, cc = o / nc3;
          const int h = row / ntv2, j = row - h * ntv2;
          const double2* Pa = P2 + (((int64_t)a * 2 + h) * L + (int64_t)q * ntv) * ntv2 + j;
          cpx<double> s = acc[m];
          for (int i = 0; i < ntv; ++i) cfma_conj(s, ldc(Pa, (int64_t)i * ntv2), T[cc * nc2 + h * ntv + i]);
          acc[m] = s;
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < kMaxOut; ++m) {
    const int o = threadIdx.x + 256 * m;
    if (o < nc3 * nc3) stc(D3T, ((int64_t)a * 5 + eout) * nc3 * nc3 + o, acc[m]);
  }
}

// y3[k][a][h ntv2 + j] = sum_{q, i} conj(P2[a][h][q ntv + i][j]) y2[k][sites[a][q]][h ntv + i]
template <typename R>
__global__ __launch_bounds__(64) void k_restrict_l3(L3Tab t, typename PT<R>::stor* y3, const typename PT<R>::stor* P2,
                                                    const typename PT<R>::stor* y2) {
  extern __shared__ unsigned char smem_r3[];
  cpx<R>* ys = reinterpret_cast<cpx<R>*>(smem_r3);  // [2][L]
  const int a = blockIdx.x, k = blockIdx.y;
  const int L = t.bs2 * t.ntv, nc = 2 * t.ntv;
  for (int idx = threadIdx.x; idx < 2 * L; idx += blockDim.x) {
    const int h = idx / L, e = idx - h * L, q = e / t.ntv, i = e - q * t.ntv;
    ys[idx] = ldcv<R>(y2, ((int64_t)k * t.nb + t.sites[a * t.bs2 + q]) * nc + h * t.ntv + i);
  }
  __syncthreads();
  const int o = threadIdx.x;
  if (o >= 2 * t.ntv2) return;
  const int h = o / t.ntv2, j = o - h * t.ntv2;
  const auto* P = P2 + ((int64_t)a * 2 + h) * L * t.ntv2 + j;
  cpx<R> acc = czero<R>();
  for (int e = 0; e < L; ++e) cfma_conj(acc, ldcv<R>(P, (int64_t)e * t.ntv2), ys[h * L + e]);
  stcv(y3, ((int64_t)k * t.n3 + a) * 2 * t.ntv2 + o, acc);
}

// y2[k][sites[a][q]][h ntv + i] = sum_j P2[a][h][q ntv + i][j] y3[k][a][h ntv2 + j]
template <typename R>
__global__ __launch_bounds__(256) void k_prolong_l3(L3Tab t, typename PT<R>::stor* y2, const typename PT<R>::stor* P2,
                                                   const typename PT<R>::stor* y3) {
  __shared__ cpx<R> ys[64];
  const int a = blockIdx.x, k = blockIdx.y;
  const int L = t.bs2 * t.ntv, nc = 2 * t.ntv;
  if (threadIdx.x < 2 * t.ntv2) ys[threadIdx.x] = ldcv<R>(y3, ((int64_t)k * t.n3 + a) * 2 * t.ntv2 + threadIdx.x);
  __syncthreads();
  for (int idx = threadIdx.x; idx < 2 * L; idx += blockDim.x) {
    const int h = idx / L, e = idx - h * L, q = e / t.ntv, i = e - q * t.ntv;
    const auto* P = P2 + (((int64_t)a * 2 + h) * L + e) * t.ntv2;
    cpx<R> acc = czero<R>();
    for (int j = 0; j < t.ntv2; ++j) cfma(acc, ldcv<R>(P, j), ys[h * t.ntv2 + j]);
    stcv(y2, ((int64_t)k * t.nb + t.sites[a * t.bs2 + q]) * nc + h * t.ntv + i, acc);
  }
}

int lex4(const int x[4], const int n[4]) { return ((x[0] * n[1] + x[1]) * n[2] + x[2]) * n[3] + x[3]; }

}  // namespace

size_t l3_elems(const qmg_ctx* c) { return (size_t)c->l3.n3 * 2 * c->l3.ntv2; }

hipError_t launch_restrict_l3(const qmg_ctx* c, int p, void* y3, const void* y2, int nrhs, hipStream_t s) {
  const L3Tab t = tab_of(c);
  const dim3 grid(t.n3, nrhs);
  const int L = t.bs2 * t.ntv;
  if (p == QMG_F64)
    hipLaunchKernelGGL(k_restrict_l3<double>, grid, dim3(64), 2 * L * sizeof(cpx<double>), s, t, (double2*)y3,
                       (const double2*)c->l3.P2[0], (const double2*)y2);
  else
    hipLaunchKernelGGL(k_restrict_l3<float>, grid, dim3(64), 2 * L * sizeof(cpx<float>), s, t, (float2*)y3,
                       (const float2*)c->l3.P2[1], (const float2*)y2);
  return hipGetLastError();
}

hipError_t launch_prolong_l3(const qmg_ctx* c, int p, void* y2, const void* y3, int nrhs, hipStream_t s) {
  const L3Tab t = tab_of(c);
  const dim3 grid(t.n3, nrhs);
  if (p == QMG_F64)
    hipLaunchKernelGGL(k_prolong_l3<double>, grid, dim3(256), 0, s, t, (double2*)y2, (const double2*)c->l3.P2[0],
                       (const double2*)y3);
  else
    hipLaunchKernelGGL(k_prolong_l3<float>, grid, dim3(256), 0, s, t, (float2*)y2, (const float2*)c->l3.P2[1],
                       (const float2*)y3);
  return hipGetLastError();
}

// Geometry tables, P2 from the ntv2 level-2 vectors W2 ([ntv2][nb][2 ntv] FP64)
// and D3 from the FP64 D_c; FP32 copies of both.  Synchronous.
qmg_status build_l3(qmg_ctx* c, const void* W2, int ntv2, const int block2[4], hipStream_t s) {
  Level3& l = c->l3;
  l.ok = false;
  drop_graphs(c);
  const Geom& g = c->g;
  int d3[4], bs2 = 1, n3 = 1;
  for (int mu = 0; mu < 4; ++mu) {
    d3[mu] = g.nbk[mu] / block2[mu];
    bs2 *= block2[mu];
    n3 *= d3[mu];
  }
  const int nb = g.nb;
  // tables: sites [n3 bs2] | agg [nb] | qloc [nb] | keep [9 nb] | nbr3 [8 n3]
  std::vector<int> tab((size_t)n3 * bs2 + 11 * (size_t)nb + 8 * (size_t)n3, 0);
  int* sites = tab.data();
  int* agg = sites + (size_t)n3 * bs2;
  int* qloc = agg + nb;
  int* keep = qloc + nb;
  int* nbr3 = keep + 9 * (size_t)nb;
  for (int b = 0; b < nb; ++b) {
    int A[4], q[4];
    for (int mu = 0; mu < 4; ++mu) {
      const int X = c->h_bcoord[b * 4 + mu];
      A[mu] = X / block2[mu];
      q[mu] = X % block2[mu];
    }
    const int a = lex4(A, d3), ql = lex4(q, block2);
    sites[(size_t)a * bs2 + ql] = b;
    agg[b] = a;
    qloc[b] = ql;
    keep[b * 9] = 1;
    for (int mu = 0; mu < 4; ++mu) {
      keep[b * 9 + 1 + 2 * mu] = q[mu] != block2[mu] - 1;
      keep[b * 9 + 2 + 2 * mu] = q[mu] != 0;
    }
  }
  for (int a = 0; a < n3; ++a) {
    int A[4], r = a;
    for (int mu = 3; mu >= 0; --mu) {
      A[mu] = r % d3[mu];
      r /= d3[mu];
    }
    for (int mu = 0; mu < 4; ++mu)
      for (int dir = 0; dir < 2; ++dir) {
        int B[4] = {A[0], A[1], A[2], A[3]};
        B[mu] = (A[mu] + (dir == 0 ? 1 : d3[mu] - 1)) % d3[mu];
        nbr3[a * 8 + 2 * mu + dir] = lex4(B, d3);
      }
  }
  int* dtab = (int*)ws_get(c, "l3_tab", tab.size() * sizeof(int));
  const int nc3 = 2 * ntv2, L = bs2 * c->ntv;
  const size_t pel = (size_t)n3 * 2 * L * ntv2, del = (size_t)n3 * 5 * nc3 * nc3;  // D3: self + 4 forward blocks
  for (int sp = 0; sp < 2; ++sp) {
    const int p = sp == 0 ? QMG_F64 : QMG_F32;
    l.P2[sp] = ws_get(c, "l3_P" + std::to_string(sp), pel * cbytes(p));
    l.D3[sp] = ws_get(c, "l3_D" + std::to_string(sp), del * cbytes(p));
    if (!l.P2[sp] || !l.D3[sp]) return set_err(c, QMG_E_NOMEM, "out of device memory (P2, D3)");
  }
  int* fail = (int*)ws_get(c, "l3_fail", sizeof(int));
  if (!dtab || !fail) return set_err(c, QMG_E_NOMEM, "out of device memory (level 3)");
  hipError_t e = hipMemcpy(dtab, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_err(c, e, "level-3 tables");
  l.ntv2 = ntv2;
  l.n3 = n3;
  l.bs2 = bs2;
  for (int mu = 0; mu < 4; ++mu) {
    l.block2[mu] = block2[mu];
    l.dims3[mu] = d3[mu];
  }
  l.sites = dtab;
  l.agg = dtab + (agg - sites);
  l.qloc = dtab + (qloc - sites);
  l.keep = dtab + (keep - sites);
  l.nbr3 = dtab + (nbr3 - sites);
  const L3Tab t = tab_of(c);
  e = hipMemsetAsync(fail, 0, sizeof(int), s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_build_P2, dim3(2 * n3), dim3(256), 0, s, t, (double2*)l.P2[0], (const double2*)W2,
                       (int64_t)coarse_elems(c), fail);
    e = hipGetLastError();
  }
  int hfail = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&hfail, fail, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "build P2");
  if (hfail) return set_err(c, QMG_E_NUMERIC, "level-2 test vectors are locally rank deficient");
  hipLaunchKernelGGL(k_assemble_D3, dim3(n3, 5), dim3(256), (size_t)nc3 * 2 * c->ntv * sizeof(cpx<double>), s, t,
                     (double2*)l.D3[0], (const double2*)c->Dc[QMG_F64], (const double2*)l.P2[0]);
  e = hipGetLastError();
  if (e == hipSuccess) e = launch_convert(l.P2[1], QMG_F32, l.P2[0], QMG_F64, (int64_t)pel, s);
  if (e == hipSuccess) e = launch_convert(l.D3[1], QMG_F32, l.D3[0], QMG_F64, (int64_t)del, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_err(c, e, "assemble D3");
  l.ok = true;
  return QMG_OK;
}

// Level-2 test vectors (reading: the paper's setup one level down): normalise
// W2, build the level, then iters - 1 rounds of inverse iteration w <- M2 w at
// tau = 0 in FP64, each followed by normalisation and a rebuild.
qmg_status solver_setup_l3(qmg_ctx* c, void* W2, int ntv2, const int block2[4], int iters, int s2, int k3,
                           hipStream_t s) {
  const int64_t n = (int64_t)coarse_elems(c);
  const size_t vb = (size_t)n * 16;
  std::vector<double> tau0(ntv2, 0.0);
  double* nrm = (double*)ws_get(c, "l3s_nrm", sizeof(double) * 2 * ntv2);
  double* sc = (double*)ws_get(c, "l3s_sc", sizeof(double) * 2 * ntv2);
  double* part = (double*)ws_get(c, "l3s_part", sizeof(double) * multidot_partial_doubles(n, 1, ntv2));
  void* Wn = ws_get(c, "l3s_new", vb * ntv2);
  if (!nrm || !sc || !part || !Wn) return set_err(c, QMG_E_NOMEM, "out of device memory (level-3 setup)");
  auto normalise = [&](void* X) -> qmg_status {
    hipError_t e = launch_multidot(QMG_F64, nrm, X, 0, 0, X, n, n, ntv2, part, s, 1);
    std::vector<double> h(2 * ntv2);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), nrm, sizeof(double) * 2 * ntv2, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_err(c, e, "level-3 setup norms");
    for (int k = 0; k < ntv2; ++k) {
      const double nn = std::sqrt(h[2 * k]);
      if (!(nn > 0) || !std::isfinite(nn)) return set_err(c, QMG_E_NUMERIC, "level-2 setup vector vanished");
      h[2 * k] = 1.0 / nn;
      h[2 * k + 1] = 0.0;
    }
    e = hipMemcpyAsync(sc, h.data(), sizeof(double) * 2 * ntv2, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = launch_scale(QMG_F64, X, X, sc, n, n, ntv2, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e == hipSuccess ? QMG_OK : hip_err(c, e, "level-3 setup scale");
  };
  qmg_status st = normalise(W2);
  if (st == QMG_OK) st = build_l3(c, W2, ntv2, block2, s);
  for (int it = 1; it < iters && st == QMG_OK; ++it) {
    st = level2_cycle(c, QMG_F64, Wn, W2, tau0.data(), ntv2, k3, s2, s);
    if (st == QMG_OK) st = normalise(Wn);
    if (st == QMG_OK) {
      hipError_t e = hipMemcpyAsync(W2, Wn, vb * ntv2, hipMemcpyDeviceToDevice, s);
      if (e != hipSuccess) return hip_err(c, e, "copy");
      st = build_l3(c, W2, ntv2, block2, s);
    }
  }
  ws_release(c, "l3s_new");
  return st;
}
