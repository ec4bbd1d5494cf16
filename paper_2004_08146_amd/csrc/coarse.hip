// Galerkin coarse operator D_c = P^H D P (Sec. 2) and its application
// out_k = (D_c - tau_k Gamma5^c) in_k.
//
// D_c couples each coarse site (lattice block) b to itself and to its 8
// neighbouring blocks.  Only the self block and the 4 forward blocks are
// stored: D is Gamma5-Hermitian and Gamma5 P = P Gamma5^c (text before
// eq. (2.9)), so Gamma5^c D_c Gamma5^c = D_c^H and, hop type by hop type, the
// block coupling b to X - mu is Gamma5^c (the block coupling X - mu to b)^H
// Gamma5^c.  The apply kernels rebuild those backward blocks on the fly.
// D_c is assembled column by column, a batch of columns at a time: prolong
// unit coarse vectors, split D applied to each into the block-local part
// (diagonal plus hops inside the block) and the 4 forward hop parts that leave
// the block, restrict all parts as one multi-rhs restriction (each part with
// the receiving block's P) and scatter them into the blocks.  Blocks are
// stored transposed, DcT[b][e][j][i] = D_c[b][e]_{ij}, e = 0 self, 1 + mu for
// the block at X + mu (kept apart from the -mu coupling even when the two
// neighbours coincide).  In the 9-entry stencil numbering used by the kernels,
// d = 0 is self, d = 1 + 2 mu the block at X + mu, d = 2 + 2 mu the one at
// X - mu.  The apply kernels serve every coarse level: they take the level's
// neighbour table, site count and blocks.
#include "qmg_ctx.h"

namespace {

// out5[0] = block-local part (diagonal, clover and the hops that stay inside
// the block), out5[1 + mu] = forward hop leaving the block (zero where it stays
// inside); the backward hops that leave the block are not needed
__global__ __launch_bounds__(256) void k_split(Geom g, double2* out5, const double2* in, const double2* U,
                                               const double2* diag, double mass4, int clover) {
  int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  const int b = (int)(site >> g.bs_log), l = (int)(site & ((1 << g.bs_log) - 1));
  const int64_t fs = g.V * 12;
  Spinor<double> self = load_spinor<double>(in, g, b, l);
  Spinor<double> loc0;
  if (clover) loc0 = apply_diag<double>(diag, g, b, l, self);
  else
    for (int s = 0; s < 4; ++s)
      for (int c = 0; c < 3; ++c) loc0.s[s][c] = mass4 * self.s[s][c];
  for (int mu = 0; mu < 4; ++mu) {
    for (int dir = 0; dir < 2; ++dir) {
      const bool fwd = dir == 0;
      int bn, ln;
      if (fwd) nb_fwd(g, b, l, mu, bn, ln);
      else nb_bwd(g, b, l, mu, bn, ln);
      Half<double> h = project(load_spinor<double>(in, g, bn, ln), mu, fwd);
      Half<double> w = fwd ? umul(load_link<double>(U, g, b, mu, l), h)
                           : udagmul(load_link<double>(U, g, bn, mu, ln), h);
      Spinor<double> t;
      for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 3; ++c) t.s[s][c] = czero<double>();
      accum_recon(t, w, mu, fwd);
      const bool inside = fwd ? (loc(g, l, mu) < g.msk[mu]) : (loc(g, l, mu) > 0);
      for (int s = 0; s < 4; ++s)
        for (int c = 0; c < 3; ++c)
          if (inside) loc0.s[s][c] = loc0.s[s][c] - 0.5 * t.s[s][c];
      if (fwd) {
        Spinor<double> o;
        for (int s = 0; s < 4; ++s)
          for (int c = 0; c < 3; ++c) o.s[s][c] = inside ? czero<double>() : (-0.5) * t.s[s][c];
        store_spinor(out5 + (1 + mu) * fs, g, b, l, o);
      }
    }
  }
  store_spinor(out5, g, b, l, loc0);
}

// DcT[b][e][c0 + kk][i] = part[kk * 5 + e][b][i]: restricted stencil parts of a
// batch of kb unit columns into the transposed blocks of D_c
__global__ __launch_bounds__(256) void k_scatter_dc(double2* DcT, const double2* part, int nb, int nc, int c0,
                                                  int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int i = (int)(idx % nc);
  const int64_t t = idx / nc;
  const int b = (int)(t % nb), n = (int)(t / nb);
  const int kk = n / 5, e = n - 5 * kk;
  DcT[(((int64_t)b * 5 + e) * nc + c0 + kk) * nc + i] = part[idx];
}

struct TauArr {
  double t[QMG_MAXRHS];
  int qform;  // 1: Gamma5^c (D_c - tau Gamma5^c) = Gamma5^c D_c - tau, the Galerkin P^H (Q - tau) P
};

template <typename S, typename C, int T>
__global__ __launch_bounds__(64) void k_coarse_apply(const int* nbr, int nb, typename PT<C>::stor* out,
                                                     const typename PT<S>::stor* DcT, const typename PT<C>::stor* in,
                                                     int nc, int nrhs, TauArr tau) {
  using R = typename PT<C>::real;
  __shared__ cpx<R> xin[9][T][64];
  const int b = blockIdx.x, k0 = blockIdx.y * T, tid = threadIdx.x;
  for (int idx = tid; idx < 9 * T * nc; idx += blockDim.x) {
    const int d = idx / (T * nc), t = (idx / nc) % T, j = idx % nc;
    const int nbk = d == 0 ? b : nbr[b * 8 + d - 1];
    const int k = k0 + t;
    xin[d][t][j] = k < nrhs ? ldcv<R>(in, ((int64_t)k * nb + nbk) * nc + j) : czero<R>();
  }
  __syncthreads();
  const int i = tid;
  if (i >= nc) return;
  cpx<R> acc[T];
#pragma unroll
  for (int t = 0; t < T; ++t) acc[t] = czero<R>();
  const R g5 = i < nc / 2 ? R(1) : R(-1);
  for (int d = 0; d < 9; ++d) {
    if (d == 0 || (d & 1)) {
      // self (e = 0) or forward block e = 1 + mu of this site: row j of the transposed block
      const auto* Dd = DcT + ((int64_t)b * 5 + (d + 1) / 2) * nc * nc;
      for (int j = 0; j < nc; ++j) {
        const cpx<R> a = ldcv<R>(Dd, (int64_t)j * nc + i);
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = acc[t] + a * xin[d][t][j];
      }
    } else {
      // backward block: D_c[b][X - mu]_{ij} = g_i g_j conj(F_{ji}), F the forward block of
      // the site at X - mu, whose transposed storage holds F_{ji} at i * nc + j
      const auto* Fd = DcT + ((int64_t)nbr[b * 8 + d - 1] * 5 + d / 2) * nc * nc + (int64_t)i * nc;
      for (int j = 0; j < nc; ++j) {
        const cpx<R> f = ldcv<R>(Fd, j);
        const R gg = j < nc / 2 ? g5 : -g5;
        const cpx<R> a = {gg * f.re, -gg * f.im};
#pragma unroll
        for (int t = 0; t < T; ++t) acc[t] = acc[t] + a * xin[d][t][j];
      }
    }
  }
#pragma unroll
  for (int t = 0; t < T; ++t) {
    const int k = k0 + t;
    if (k < nrhs) {
      const cpx<R> v = acc[t] - (R(tau.t[k]) * g5) * xin[0][t][i];
      stcv(out, ((int64_t)k * nb + b) * nc + i, tau.qform ? g5 * v : v);
    }
  }
}

// ---- MFMA coarse apply (many right-hand sides): per coarse site b and tile of
// 16 rhs, Out (2ntv x 16) = sum_d D_c[b][d] (2ntv x 2ntv) In_{nbr(b,d)} (2ntv x 16),
// a complex GEMM done as four real 16x16x4 MFMA products per k-step
// (C_re += A_re B_re - A_im B_im, C_im += A_re B_im + A_im B_re).  One wave
// per work-group; the 16 rhs of a neighbour block are staged in LDS.
typedef float mf4 __attribute__((ext_vector_type(4)));
typedef double md4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ mf4 mfma(float a, float b, mf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ md4 mfma(double a, double b, md4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }

template <typename R> struct MAcc;
template <> struct MAcc<float> { using T = mf4; };
template <> struct MAcc<double> { using T = md4; };

// row of output register r of lane l inside a 16x16 tile
template <typename R> __device__ __forceinline__ int mrow(int l, int r);
template <> __device__ __forceinline__ int mrow<float>(int l, int r) { return 4 * (l >> 4) + r; }
template <> __device__ __forceinline__ int mrow<double>(int l, int r) { return 4 * r + (l >> 4); }

template <typename S, typename C, int NT>
__global__ __launch_bounds__(64 * NT) void k_coarse_mfma(const int* nbr, int nb, typename PT<C>::stor* out,
                                                         const typename PT<S>::stor* DcT, const typename PT<C>::stor* in,
                                                         int nrhs, TauArr tau) {
  using R = typename PT<C>::real;
  using AT = typename MAcc<R>::T;
  constexpr int NC = 16 * NT;  // 2 ntv
  __shared__ cpx<R> Bs[NC][16];
  __shared__ cpx<R> Bself[NC][16];
  // one wave per 16-row tile t of the output; the waves share the staged inputs
  const int b = blockIdx.x, n0 = blockIdx.y * 16, tid = threadIdx.x;
  const int t = tid >> 6, l = tid & 63;
  const int ln = l & 15, lk = l >> 4;
  AT acc_re = AT{0, 0, 0, 0}, acc_im = AT{0, 0, 0, 0};
  // output row of this lane's A fragment
  const int irow = 16 * t + ln;
#pragma unroll 1
  for (int d = 0; d < 9; ++d) {
    const int nbk = d == 0 ? b : nbr[b * 8 + d - 1];
    __syncthreads();
    for (int idx = tid; idx < NC * 16; idx += 64 * NT) {
      const int j = idx % NC, n = idx / NC;
      const cpx<R> v = n0 + n < nrhs ? ldcv<R>(in, ((int64_t)(n0 + n) * nb + nbk) * NC + j) : czero<R>();
      Bs[j][n] = v;
      if (d == 0) Bself[j][n] = v;
    }
    __syncthreads();
    if (d == 0 || (d & 1)) {
      // self or forward block: A_{ij} at row j of the transposed block
      const auto* Dd = DcT + ((int64_t)b * 5 + (d + 1) / 2) * NC * NC + irow;
#pragma unroll 4
      for (int j0 = 0; j0 < NC; j0 += 4) {
        const cpx<R> bv = Bs[j0 + lk][ln];
        const cpx<R> av = ldcv<R>(Dd, (int64_t)(j0 + lk) * NC);
        acc_re = mfma(av.re, bv.re, acc_re);
        acc_re = mfma(-av.im, bv.im, acc_re);
        acc_im = mfma(av.re, bv.im, acc_im);
        acc_im = mfma(av.im, bv.re, acc_im);
      }
    } else {
      // backward block from the forward block F of the site at X - mu:
      // A_{ij} = g_i g_j conj(F_{ji}), F_{ji} stored at i * NC + j, i.e. along row i.
      // The contraction index is visited in a permuted order (A and B permuted
      // alike): in each run of 16 columns, MFMA step s takes j = jb + 4 lk + s, so
      // every lane reads its 4 consecutive entries of row i with one wide load
      const auto* Fd = DcT + ((int64_t)nbk * 5 + d / 2) * NC * NC + (int64_t)irow * NC;
      const R gi = irow < NC / 2 ? R(1) : R(-1);
#pragma unroll
      for (int jb = 0; jb < NC; jb += 16) {
        cpx<R> f[4];
        ld4c(Fd + jb + 4 * lk, f);
        const R gg = (jb + 4 * lk < NC / 2) ? gi : -gi;  // the 4 columns share a chirality half
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const cpx<R> bv = Bs[jb + 4 * lk + q][ln];
          const R are = gg * f[q].re, aim = -gg * f[q].im;
          acc_re = mfma(are, bv.re, acc_re);
          acc_re = mfma(-aim, bv.im, acc_re);
          acc_im = mfma(are, bv.im, acc_im);
          acc_im = mfma(aim, bv.re, acc_im);
        }
      }
    }
  }
  const int n = n0 + ln;
  if (n >= nrhs) return;
  const R tn = R(tau.t[n]);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = 16 * t + mrow<R>(l, r);
    const R g5 = i < NC / 2 ? R(1) : R(-1);
    const cpx<R> self = Bself[i][ln];
    cpx<R> v = {acc_re[r] - tn * g5 * self.re, acc_im[r] - tn * g5 * self.im};
    if (tau.qform) v = g5 * v;
    stcv(out, ((int64_t)n * nb + b) * NC + i, v);
  }
}

// one coarse level's stencil: nb sites, 2 ntv components each, blocks D
// (storage precision S) and the neighbour table
struct CLevel {
  const int* nbr;
  int nb, ntv;
  const void* D;
};

template <typename S>
void capply_mfma(const CLevel& lv, int p, void* out, const void* in, const TauArr& tau, int nrhs, hipStream_t s) {
  using P = typename PT<S>::stor;
  dim3 grid(lv.nb, (nrhs + 15) / 16);
  // 2 ntv = 48 (ntv = 24) -> 3 row tiles; 2 ntv = 32 -> 2; 2 ntv = 16 -> 1
  const int nt = (2 * lv.ntv) / 16;
  auto go = [&](auto ntc) {
    constexpr int NT = decltype(ntc)::value;
    if (p == QMG_F64)
      hipLaunchKernelGGL((k_coarse_mfma<S, double, NT>), grid, dim3(64 * NT), 0, s, lv.nbr, lv.nb, (double2*)out,
                         (const P*)lv.D, (const double2*)in, nrhs, tau);
    else
      hipLaunchKernelGGL((k_coarse_mfma<S, float, NT>), grid, dim3(64 * NT), 0, s, lv.nbr, lv.nb, (float2*)out,
                         (const P*)lv.D, (const float2*)in, nrhs, tau);
  };
  if (nt == 3) go(std::integral_constant<int, 3>{});
  else if (nt == 2) go(std::integral_constant<int, 2>{});
  else go(std::integral_constant<int, 1>{});
}

template <typename S, int T>
void capply_t(const CLevel& lv, int p, void* out, const void* in, const TauArr& tau, int nrhs, hipStream_t s) {
  using P = typename PT<S>::stor;
  const int nc = 2 * lv.ntv;
  dim3 grid(lv.nb, (nrhs + T - 1) / T);
  if (p == QMG_F64)
    hipLaunchKernelGGL((k_coarse_apply<S, double, T>), grid, dim3(64), 0, s, lv.nbr, lv.nb, (double2*)out,
                       (const P*)lv.D, (const double2*)in, nc, nrhs, tau);
  else
    hipLaunchKernelGGL((k_coarse_apply<S, float, T>), grid, dim3(64), 0, s, lv.nbr, lv.nb, (float2*)out,
                       (const P*)lv.D, (const float2*)in, nc, nrhs, tau);
}

template <typename S>
void capply_s(const qmg_ctx* c, const CLevel& lv, int p, void* out, const void* in, const double* htau, int nrhs,
              hipStream_t s, int qform) {
  TauArr t;
  for (int i = 0; i < QMG_MAXRHS; ++i) t.t[i] = i < nrhs ? htau[i] : 0.0;
  t.qform = qform;
  // MFMA path when the coarse dimension is a multiple of 16 (ntv = 8, 16, 24) and
  // enough right-hand sides share each matrix block
  if (c->tune.coarse_mfma && (2 * lv.ntv) % 16 == 0 && 2 * lv.ntv <= 48 && nrhs >= c->tune.coarse_mfma_min_rhs) {
    if constexpr (std::is_same<S, double>::value) {
      if (p == QMG_F64) { capply_mfma<S>(lv, p, out, in, t, nrhs, s); return; }
    } else {
      capply_mfma<S>(lv, p, out, in, t, nrhs, s);
      return;
    }
  }
  if (nrhs >= 4) capply_t<S, 4>(lv, p, out, in, t, nrhs, s);
  else if (nrhs == 2) capply_t<S, 2>(lv, p, out, in, t, nrhs, s);
  else capply_t<S, 1>(lv, p, out, in, t, nrhs, s);
}

}  // namespace

hipError_t launch_split_stencil(const qmg_ctx* c, void* out5, const void* in, hipStream_t s) {
  hipLaunchKernelGGL(k_split, dim3((unsigned)((c->g.V + 255) / 256)), dim3(256), 0, s, c->g, (double2*)out5,
                     (const double2*)in, (const double2*)c->U[QMG_F64], (const double2*)c->Dg[QMG_F64],
                     c->m0 + 4.0, c->clover ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_scatter_dc(const qmg_ctx* c, void* Dc64, const void* part, int c0, int kb, hipStream_t s) {
  const int nc = 2 * c->ntv;
  const int64_t total = (int64_t)kb * 5 * c->g.nb * nc;
  hipLaunchKernelGGL(k_scatter_dc, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, (double2*)Dc64,
                     (const double2*)part, c->g.nb, nc, c0, total);
  return hipGetLastError();
}

// tau: host array of nrhs shifts
hipError_t launch_coarse_apply(const qmg_ctx* c, int p, void* out, const void* in, const double* dtau, int nrhs,
                               hipStream_t s, int qform) {
  const CLevel lv{c->g.nbr, c->g.nb, c->ntv, c->Dc[p]};
  if (p == QMG_F64) capply_s<double>(c, lv, p, out, in, dtau, nrhs, s, qform);
  else if (p == QMG_F32) capply_s<float>(c, lv, p, out, in, dtau, nrhs, s, qform);
  else capply_s<bf16_t>(c, lv, p, out, in, dtau, nrhs, s, qform);
  return hipGetLastError();
}

// level-3 operator A3(tau) = D3 - tau Gamma5^cc (D3 stored in the coarse precision of p)
hipError_t launch_apply_l3(const qmg_ctx* c, int p, void* out, const void* in, const double* dtau, int nrhs,
                           hipStream_t s, int qform) {
  const int sp = p == QMG_F64 ? 0 : 1;
  const CLevel lv{c->l3.nbr3, c->l3.n3, c->l3.ntv2, c->l3.D3[sp]};
  if (p == QMG_F64) capply_s<double>(c, lv, p, out, in, dtau, nrhs, s, qform);
  else capply_s<float>(c, lv, p, out, in, dtau, nrhs, s, qform);
  return hipGetLastError();
}
