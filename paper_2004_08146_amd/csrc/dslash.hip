// Wilson(-clover) stencil, eq. (2.5):
//   (D psi)(x) = [(m0+4) + C(x)] psi(x) - 1/2 sum_mu (I - g_mu) U_mu(x) psi(x+mu)
//                                       - 1/2 sum_mu (I + g_mu) U_mu(x-mu)^H psi(x-mu)
// with the shift folded in: mode 0 gives (D - tau Gamma5) psi (eq. (3.7)),
// mode 1 gives (Gamma5 D - tau) psi = (Q - tau) psi (eq. (1.1)).
//
// One thread per site and right-hand side.  Work-groups are mapped to sites
// so that each XCD walks a contiguous slab of the block-major lattice and the
// right-hand sides of one site tile run back to back on the same XCD (their
// shared links then come from that XCD's L2).
#include "qmg_ctx.h"

namespace {

// SI: storage type of the input field (the output, links and clover use S); an
// FP64 apply may read a field stored in FP32 or BF16 with no change in its
// arithmetic, since every such value is exact in FP64.
template <typename S, typename SI = S>
struct DsArgs {
  typename PT<S>::stor* out;
  const typename PT<SI>::stor* in;
  const typename PT<S>::stor* U;
  const typename PT<S>::stor* diag;
  double mass4;
  int64_t fstride;  // complex elements per field
  int nrhs;
  int remap;
  const int* tord;  // block ids in work order: tiles of tb blocks, each tile's rhs groups back to back
  int tb;
  int nt_out;       // 1: the output is written with non-temporal stores (streamed past the caches)
  Geom g;
  double tau[QMG_MAXRHS];
};

// acc += (I - g_mu) U_mu(x) psi(x+mu) + (I + g_mu) U_mu(x-mu)^H psi(x-mu)
template <typename R, int MU, typename PI, typename P>
__device__ __forceinline__ void hop_pair(Spinor<R>& acc, const PI* in, const P* U, const Geom& g, int b, int l) {
  int bn, ln;
  nb_fwd(g, b, l, MU, bn, ln);
  {
    Half<R> h = project(load_spinor<R>(in, g, bn, ln), MU, true);
    accum_recon(acc, umul(load_link<R>(U, g, b, MU, l), h), MU, true);
  }
  nb_bwd(g, b, l, MU, bn, ln);
  {
    Half<R> h = project(load_spinor<R>(in, g, bn, ln), MU, false);
    accum_recon(acc, udagmul(load_link<R>(U, g, bn, MU, ln), h), MU, false);
  }
}

template <typename S, bool CLOVER, int MODE, bool UB, typename SI>
__global__ __launch_bounds__(256) void k_dslash(DsArgs<S, SI> a) {
  using R = typename PT<S>::real;
  const Geom& g = a.g;
  const int w = blockIdx.x, nw = gridDim.x;
  const int L = (a.remap && (nw & 7) == 0) ? (w & 7) * (nw >> 3) + (w >> 3) : w;
  const int k = L % a.nrhs;
  const int64_t site = (int64_t)(L / a.nrhs) * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  int b = (int)(site >> g.bs_log);
  if (UB) b = __builtin_amdgcn_readfirstlane(b);
  const int l = (int)(site & ((1 << g.bs_log) - 1));
  const auto* in = a.in + k * a.fstride;
  auto* out = a.out + k * a.fstride;

  Spinor<R> acc;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.s[s][c] = czero<R>();

  // one direction at a time keeps a single neighbour in flight per thread
#pragma unroll 1
  for (int mu = 0; mu < 4; ++mu) {
    switch (mu) {
      case 0: hop_pair<R, 0>(acc, in, a.U, g, b, l); break;
      case 1: hop_pair<R, 1>(acc, in, a.U, g, b, l); break;
      case 2: hop_pair<R, 2>(acc, in, a.U, g, b, l); break;
      default: hop_pair<R, 3>(acc, in, a.U, g, b, l); break;
    }
  }
  const Spinor<R> self = load_spinor<R>(in, g, b, l);
  Spinor<R> o;
  if (CLOVER) {
    o = apply_diag<R>(a.diag, g, b, l, self);
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) o.s[s][c] = R(a.mass4) * self.s[s][c];
  }
  const R tau = R(a.tau[k]);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      cpx<R> v = o.s[s][c] - R(0.5) * acc.s[s][c];
      if (MODE == 0) {
        // D - tau Gamma5
        v = (s < 2) ? v - tau * self.s[s][c] : v + tau * self.s[s][c];
      } else {
        // Gamma5 D - tau
        v = (s < 2) ? v - tau * self.s[s][c] : -v - tau * self.s[s][c];
      }
      o.s[s][c] = v;
    }
  store_spinor(out, g, b, l, o);
}

// ---- 4^4 blocks: compile-time geometry, 32-bit offsets, R right-hand sides per
// thread sharing every link load.  One work-group = one block x R rhs.
template <int MU> struct Sh44 { static constexpr int v = 6 - 2 * MU; };

template <typename C, typename P>
__device__ __forceinline__ Spinor<C> ld_spinor44(const P* f, uint32_t b, uint32_t l) {
  Spinor<C> p;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      auto v = cv(ldo(f, ((b * 12u + (uint32_t)(3 * s + c)) << 8) + l));
      p.s[s][c] = cpx<C>{C(v.re), C(v.im)};
    }
  return p;
}
template <typename C, typename P>
__device__ __forceinline__ Link<C> ld_link44(const P* U, uint32_t b, int mu, uint32_t l) {
  Link<C> u;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      auto v = cv(ldo(U, ((b * 36u + (uint32_t)(mu * 9 + 3 * a + c)) << 8) + l));
      u.u[a][c] = cpx<C>{C(v.re), C(v.im)};
    }
  return u;
}

// one hop (HOP = 2 mu for x + mu, 2 mu + 1 for x - mu) for R right-hand sides
template <typename C, int HOP, int R, typename PI, typename P>
__device__ __forceinline__ void hop44(Spinor<C> (&acc)[R], const PI* const (&in)[R], const P* U, const int* nbr,
                                      uint32_t b, uint32_t l, int nr) {
  constexpr int MU = HOP / 2;
  constexpr bool FWD = (HOP % 2) == 0;
  constexpr int SH = Sh44<MU>::v;
  const uint32_t lc = (l >> SH) & 3u;
  const uint32_t bo = (uint32_t)nbr[b * 8 + HOP];
  uint32_t bn, ln;
  if (FWD) {
    bn = lc < 3u ? b : bo;
    ln = lc < 3u ? l + (1u << SH) : l - (3u << SH);
  } else {
    bn = lc > 0u ? b : bo;
    ln = lc > 0u ? l - (1u << SH) : l + (3u << SH);
  }
  const Link<C> u = FWD ? ld_link44<C>(U, b, MU, l) : ld_link44<C>(U, bn, MU, ln);
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r < nr) {
      const Half<C> h = project(ld_spinor44<C>(in[r], bn, ln), MU, FWD);
      accum_recon(acc[r], FWD ? umul(u, h) : udagmul(u, h), MU, FWD);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename S, bool CLOVER, int MODE, int R, int W, bool LOOP, typename SI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(W > 0 ? W : 1))) void k_dslash44(DsArgs<S, SI> a) {
  using C = typename PT<S>::real;
  using P = typename PT<S>::stor;
  const int w = blockIdx.x, nw = gridDim.x;
  const int L = (a.remap && (nw & 7) == 0) ? (w & 7) * (nw >> 3) + (w >> 3) : w;
  const int ng = (a.nrhs + R - 1) / R;
  // blocks are visited in lexicographic order so that neighbouring blocks run
  // close together in time (and, with the XCD remap, on the same XCD).  With
  // LOOP one work-group walks all rhs groups of its block, so the block's
  // links are fetched from HBM once and re-read from cache.
  // Without LOOP, work-group L takes rhs group kg of one block, in tiles of tb
  // blocks whose rhs groups run back to back (tb = 1: one block at a time).
  uint32_t b;
  int kbeg, kend;
  if (LOOP) {
    b = (uint32_t)__builtin_amdgcn_readfirstlane(a.g.lexord[L]);
    kbeg = 0;
    kend = ng;
  } else {
    const int per = a.tb * ng, ti = L / per, rem = L - ti * per;
    kbeg = rem / a.tb;
    kend = kbeg + 1;
    b = (uint32_t)__builtin_amdgcn_readfirstlane(a.tord[ti * a.tb + (rem - kbeg * a.tb)]);
  }
  const uint32_t l = threadIdx.x;
#pragma unroll 1
  for (int kg = kbeg; kg < kend; ++kg) {
  const int k0 = kg * R;
  const int nr = a.nrhs - k0 < R ? a.nrhs - k0 : R;
  const typename PT<SI>::stor* in[R];
#pragma unroll
  for (int r = 0; r < R; ++r) in[r] = a.in + (size_t)(k0 + (r < nr ? r : 0)) * a.fstride;
  Spinor<C> acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc[r].s[s][c] = czero<C>();
#pragma unroll 1
  for (int hop = 0; hop < 8; ++hop) {
    switch (hop) {
      case 0: hop44<C, 0, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      case 1: hop44<C, 1, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      case 2: hop44<C, 2, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      case 3: hop44<C, 3, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      case 4: hop44<C, 4, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      case 5: hop44<C, 5, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      case 6: hop44<C, 6, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
      default: hop44<C, 7, R>(acc, in, a.U, a.g.nbr, b, l, nr); break;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r >= nr) break;
    const Spinor<C> self = ld_spinor44<C>(in[r], b, l);
    Spinor<C> o;
    if (CLOVER) {
      o = apply_diag<C>(a.diag, a.g, (int)b, (int)l, self);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) o.s[s][c] = C(a.mass4) * self.s[s][c];
    }
    const C tau = C(a.tau[k0 + r]);
    P* out = a.out + (size_t)(k0 + r) * a.fstride;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cpx<C> v = o.s[s][c] - C(0.5) * acc[r].s[s][c];
        if (MODE == 0) v = (s < 2) ? v - tau * self.s[s][c] : v + tau * self.s[s][c];
        else v = (s < 2) ? v - tau * self.s[s][c] : -v - tau * self.s[s][c];
        const uint32_t o = ((b * 12u + (uint32_t)(3 * s + c)) << 8) + l;
        if (a.nt_out) sto_nt(out, o, vc(v, (P*)nullptr));
        else sto(out, o, vc(v, (P*)nullptr));
      }
  }
  }
}

template <typename S, bool CLOVER, int MODE, int R, int W, bool LOOP = false, typename SI>
void launch44(const DsArgs<S, SI>& a, int nb, hipStream_t s) {
  const unsigned ng = LOOP ? 1u : (unsigned)((a.nrhs + R - 1) / R);
  hipLaunchKernelGGL((k_dslash44<S, CLOVER, MODE, R, W, LOOP, SI>), dim3((unsigned)nb * ng), dim3(256), 0, s, a);
}

template <typename S, bool CLOVER, int MODE, typename SI = S>
void launch_t(const qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, hipStream_t s,
              int p) {
  using P = typename PT<S>::stor;
  DsArgs<S, SI> a;
  a.out = (P*)out;
  a.in = (const typename PT<SI>::stor*)in;
  a.U = (const P*)c->U[p];
  a.diag = (const P*)c->Dg[p];
  a.mass4 = c->m0 + 4.0;
  a.fstride = (int64_t)field_elems(c);
  a.nrhs = nrhs;
  a.remap = c->tune.dslash_xcd_remap;
  a.tord = c->d_tord;
  a.tb = c->tile_blocks;
  a.nt_out = 0;
  a.g = c->g;
  for (int i = 0; i < QMG_MAXRHS; ++i) a.tau[i] = i < nrhs ? tau[i] : 0.0;
  const bool b44 = c->g.block[0] == 4 && c->g.block[1] == 4 && c->g.block[2] == 4 && c->g.block[3] == 4;
  const int var = c->tune.force_variant >= 0 ? c->tune.force_variant : c->tune.dslash[p][nrhs == 1 ? 0 : 1];
  if (b44 && var > 0 && var < kNumDsVariants) {
    switch (var) {
      case 1: launch44<S, CLOVER, MODE, 1, 0>(a, c->g.nb, s); break;
      case 2: launch44<S, CLOVER, MODE, 1, 2>(a, c->g.nb, s); break;
      case 3: launch44<S, CLOVER, MODE, 1, 3>(a, c->g.nb, s); break;
      case 4: launch44<S, CLOVER, MODE, 1, 4>(a, c->g.nb, s); break;
      case 5: launch44<S, CLOVER, MODE, 2, 0>(a, c->g.nb, s); break;
      case 6: launch44<S, CLOVER, MODE, 2, 2>(a, c->g.nb, s); break;
      case 7: launch44<S, CLOVER, MODE, 4, 0>(a, c->g.nb, s); break;
      case 8: launch44<S, CLOVER, MODE, 1, 2, true>(a, c->g.nb, s); break;
      case 9: launch44<S, CLOVER, MODE, 2, 0, true>(a, c->g.nb, s); break;
      case 10: launch44<S, CLOVER, MODE, 2, 2, true>(a, c->g.nb, s); break;
      default: {
        // variant 1 with the output streamed past the caches, which then keep the
        // neighbour spinors, links and clover for longer
        DsArgs<S, SI> an = a;
        an.nt_out = 1;
        launch44<S, CLOVER, MODE, 1, 0>(an, c->g.nb, s);
        break;
      }
    }
    return;
  }
  const int wg = 256;
  unsigned nwg = (unsigned)((c->g.V + wg - 1) / wg) * (unsigned)nrhs;
  if ((1 << c->g.bs_log) >= wg)
    hipLaunchKernelGGL((k_dslash<S, CLOVER, MODE, true, SI>), dim3(nwg), dim3(wg), 0, s, a);
  else
    hipLaunchKernelGGL((k_dslash<S, CLOVER, MODE, false, SI>), dim3(nwg), dim3(wg), 0, s, a);
}

template <typename S>
void launch_p(const qmg_ctx* c, void* out, const void* in, const double* tau, int nrhs, int mode,
              hipStream_t s, int p) {
  if (c->clover) {
    if (mode == 0) launch_t<S, true, 0>(c, out, in, tau, nrhs, s, p);
    else launch_t<S, true, 1>(c, out, in, tau, nrhs, s, p);
  } else {
    if (mode == 0) launch_t<S, false, 0>(c, out, in, tau, nrhs, s, p);
    else launch_t<S, false, 1>(c, out, in, tau, nrhs, s, p);
  }
}

}  // namespace

hipError_t launch_dslash(const qmg_ctx* c, int p, void* out, const void* in, const double* tau, int nrhs,
                         int mode, hipStream_t s) {
  if (p == QMG_F64) launch_p<double>(c, out, in, tau, nrhs, mode, s, p);
  else if (p == QMG_F32) launch_p<float>(c, out, in, tau, nrhs, mode, s, p);
  else launch_p<bf16_t>(c, out, in, tau, nrhs, mode, s, p);
  return hipGetLastError();
}

hipError_t launch_dslash_d_in(const qmg_ctx* c, void* out, const void* in, int in_prec, const double* tau,
                              int nrhs, hipStream_t s, int mode) {
  if (in_prec == QMG_F64) return launch_dslash(c, QMG_F64, out, in, tau, nrhs, mode, s);
  auto go = [&](auto mc) {
    constexpr int M = decltype(mc)::value;
    if (c->clover) {
      if (in_prec == QMG_F32) launch_t<double, true, M, float>(c, out, in, tau, nrhs, s, QMG_F64);
      else launch_t<double, true, M, bf16_t>(c, out, in, tau, nrhs, s, QMG_F64);
    } else {
      if (in_prec == QMG_F32) launch_t<double, false, M, float>(c, out, in, tau, nrhs, s, QMG_F64);
      else launch_t<double, false, M, bf16_t>(c, out, in, tau, nrhs, s, QMG_F64);
    }
  };
  if (mode == 0) go(std::integral_constant<int, 0>{});
  else go(std::integral_constant<int, 1>{});
  return hipGetLastError();
}
