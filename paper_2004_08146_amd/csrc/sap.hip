// One colour half-sweep of red-black SAP (Sec. 2, eq. (2.10)) on
// A_tau = D - tau Gamma5 (eq. (3.7)):
//   for every block i of the colour:  r_i = (f - A_tau x)_i,
//   e_i = n_mr minimal-residual steps on A_{tau,i} e = r_i from e = 0
//         (A_{tau,i}: A_tau restricted to block i, hops leaving it dropped),
//   x_i += e_i.
// Blocks of one colour do not touch each other, so each block is one
// work-group (one thread per site); the residual needs x of the neighbouring
// (other-colour) blocks, which this launch does not modify.  The block
// iterate rho lives in LDS so the block operator reads its neighbours there;
// block-wide dot products use a fixed reduction order (bitwise reproducible).
#include "qmg_ctx.h"

namespace {

template <typename S>
struct SapArgs {
  typename PT<S>::stor* x;
  const typename PT<S>::stor* f;
  const typename PT<S>::stor* U;
  const typename PT<S>::stor* diag;
  double mass4;
  int64_t fstride;
  int nrhs;
  int first_block;  // first block id of the colour
  int nblk;         // blocks of the colour
  int n_mr;
  Geom g;
  double tau[QMG_MAXRHS];
};

// sum of NV values over the work-group, same result in every thread
template <typename R, int NV>
__device__ __forceinline__ void block_sum(R (&v)[NV], R* red) {
  const int tid = threadIdx.x, nt = blockDim.x;
  if (nt >= 64) {
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
      for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R s = red[i];
      for (int w = 1; w < nw; ++w) s += red[w * NV + i];
      v[i] = s;
    }
  } else {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[i * nt + tid] = v[i];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      R s = red[i * nt];
      for (int t = 1; t < nt; ++t) s += red[i * nt + t];
      v[i] = s;
    }
  }
  __syncthreads();
}

template <typename R>
__device__ __forceinline__ Spinor<R> lds_spinor(const cpx<R>* sh, int l, int bs) {
  Spinor<R> p;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) p.s[s][c] = sh[(3 * s + c) * bs + l];
  return p;
}

template <typename R, typename P, bool CLOVER>
__device__ __forceinline__ Spinor<R> diag_part(const P* diag, R mass4, const Geom& g, int b, int l,
                                               const Spinor<R>& v, R tau) {
  Spinor<R> o;
  if (CLOVER) o = apply_diag<R>(diag, g, b, l, v);
  else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) o.s[s][c] = mass4 * v.s[s][c];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.s[s][c] = (s < 2) ? o.s[s][c] - tau * v.s[s][c] : o.s[s][c] + tau * v.s[s][c];
  return o;
}

// hops of the full lattice operator at (b, l), reading psi from global memory
template <typename R, int MU, typename P>
__device__ __forceinline__ void hop_global(Spinor<R>& acc, const P* in, const P* U, const Geom& g, int b, int l) {
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

// hops that stay inside the block, reading rho from LDS
template <typename R, int MU, typename P>
__device__ __forceinline__ void hop_block(Spinor<R>& acc, const cpx<R>* sh, const P* U, const Geom& g, int b,
                                          int l, int bs) {
  const int lc = loc(g, l, MU);
  const int st = 1 << g.sh[MU];
  if (lc < g.msk[MU]) {
    Half<R> h = project(lds_spinor(sh, l + st, bs), MU, true);
    accum_recon(acc, umul(load_link<R>(U, g, b, MU, l), h), MU, true);
  }
  if (lc > 0) {
    Half<R> h = project(lds_spinor(sh, l - st, bs), MU, false);
    accum_recon(acc, udagmul(load_link<R>(U, g, b, MU, l - st), h), MU, false);
  }
}

// QF: the procedure for Q - tau = Gamma5 A_tau itself (residual and block
// operator multiplied by Gamma5: lower two spins change sign)
template <typename S, bool CLOVER, bool QF>
__global__ __launch_bounds__(256) void k_sap(SapArgs<S> a) {
  using R = typename PT<S>::real;
  extern __shared__ unsigned char smem[];
  const Geom& g = a.g;
  const int bs = 1 << g.bs_log;
  cpx<R>* sh = reinterpret_cast<cpx<R>*>(smem);
  R* red = reinterpret_cast<R*>(smem + sizeof(cpx<R>) * 12 * bs);

  const int w = blockIdx.x, nw = gridDim.x;
  const int L = ((nw & 7) == 0) ? (w & 7) * (nw >> 3) + (w >> 3) : w;
  const int k = L % a.nrhs;
  const int b = a.first_block + L / a.nrhs;
  const int l = threadIdx.x;
  auto* x = a.x + k * a.fstride;
  const auto* f = a.f + k * a.fstride;
  const R tau = R(a.tau[k]);
  const R mass4 = R(a.mass4);

  // r = f - A_tau x at this site (full operator, neighbours from global x)
  Spinor<R> rho;
  {
    Spinor<R> acc;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.s[s][c] = czero<R>();
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      switch (mu) {
        case 0: hop_global<R, 0>(acc, x, a.U, g, b, l); break;
        case 1: hop_global<R, 1>(acc, x, a.U, g, b, l); break;
        case 2: hop_global<R, 2>(acc, x, a.U, g, b, l); break;
        default: hop_global<R, 3>(acc, x, a.U, g, b, l); break;
      }
    }
    Spinor<R> xs = load_spinor<R>(x, g, b, l);
    Spinor<R> d = diag_part<R, typename PT<S>::stor, CLOVER>(a.diag, mass4, g, b, l, xs, tau);
    Spinor<R> fs = load_spinor<R>(f, g, b, l);
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cpx<R> ax = d.s[s][c] - R(0.5) * acc.s[s][c];
        rho.s[s][c] = (QF && s >= 2) ? fs.s[s][c] + ax : fs.s[s][c] - ax;
      }
  }

  Spinor<R> e;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) e.s[s][c] = czero<R>();

  for (int it = 0; it < a.n_mr; ++it) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) sh[(3 * s + c) * bs + l] = rho.s[s][c];
    __syncthreads();
    // q = A_{tau,i} rho
    Spinor<R> acc;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.s[s][c] = czero<R>();
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      switch (mu) {
        case 0: hop_block<R, 0>(acc, sh, a.U, g, b, l, bs); break;
        case 1: hop_block<R, 1>(acc, sh, a.U, g, b, l, bs); break;
        case 2: hop_block<R, 2>(acc, sh, a.U, g, b, l, bs); break;
        default: hop_block<R, 3>(acc, sh, a.U, g, b, l, bs); break;
      }
    }
    Spinor<R> q = diag_part<R, typename PT<S>::stor, CLOVER>(a.diag, mass4, g, b, l, rho, tau);
    R v[3] = {R(0), R(0), R(0)};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        q.s[s][c] = q.s[s][c] - R(0.5) * acc.s[s][c];
        if (QF && s >= 2) q.s[s][c] = -q.s[s][c];
        cpx<R> t = cmul_conj(q.s[s][c], rho.s[s][c]);
        v[0] += t.re;
        v[1] += t.im;
        v[2] += norm2(q.s[s][c]);
      }
    block_sum<R, 3>(v, red);
    cpx<R> alpha = czero<R>();
    if (v[2] > R(0)) alpha = cpx<R>{v[0] / v[2], v[1] / v[2]};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e.s[s][c] = e.s[s][c] + alpha * rho.s[s][c];
        rho.s[s][c] = rho.s[s][c] - alpha * q.s[s][c];
      }
  }
  Spinor<R> xs = load_spinor<R>(x, g, b, l);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) xs.s[s][c] = xs.s[s][c] + e.s[s][c];
  store_spinor(x, g, b, l, xs);
}

// ---- 4^4 blocks, FP32 arithmetic (FP32 or BF16 storage): one work-group per
// block walks all right-hand sides.  The block's forward links are staged in
// LDS once (the block operator only needs links inside the block) and the
// clover blocks stay in registers, so the minimal-residual iterations touch
// no global memory; only the residual's faces and the update go to HBM.
constexpr int kSh44[4] = {6, 4, 2, 0};

template <int MU>
__device__ __forceinline__ void nb44(uint32_t b, uint32_t l, bool fwd, const int* nbr, uint32_t& bn, uint32_t& ln,
                                     bool& inside) {
  constexpr int SH = kSh44[MU];
  const uint32_t lc = (l >> SH) & 3u;
  if (fwd) {
    inside = lc < 3u;
    bn = inside ? b : (uint32_t)nbr[b * 8 + 2 * MU];
    ln = inside ? l + (1u << SH) : l - (3u << SH);
  } else {
    inside = lc > 0u;
    bn = inside ? b : (uint32_t)nbr[b * 8 + 2 * MU + 1];
    ln = inside ? l - (1u << SH) : l + (3u << SH);
  }
}

__device__ __forceinline__ Link<float> lds_link(const cpx<float>* Ul, int mu, uint32_t l) {
  Link<float> u;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) u.u[a][c] = Ul[(mu * 9 + 3 * a + c) * 256 + l];
  return u;
}

template <typename P>
__device__ __forceinline__ Spinor<float> gl_spinor(const P* f, uint32_t b, uint32_t l) {
  Spinor<float> p;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      auto v = cv(ldo(f, ((b * 12u + (uint32_t)(3 * s + c)) << 8) + l));
      p.s[s][c] = cpx<float>{float(v.re), float(v.im)};
    }
  return p;
}

// residual hop: neighbour spinor from global x, link from LDS when inside the block
template <int HOP, typename P>
__device__ __forceinline__ void res_hop44(Spinor<float>& acc, const P* x, const P* U, const cpx<float>* Ul,
                                          const int* nbr, uint32_t b, uint32_t l) {
  constexpr int MU = HOP / 2;
  constexpr bool FWD = HOP % 2 == 0;
  uint32_t bn, ln;
  bool inside;
  nb44<MU>(b, l, FWD, nbr, bn, ln, inside);
  const Half<float> h = project(gl_spinor(x, bn, ln), MU, FWD);
  if (FWD) {
    accum_recon(acc, umul(lds_link(Ul, MU, l), h), MU, true);
  } else {
    Link<float> u;
    if (inside) u = lds_link(Ul, MU, ln);
    else {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          auto v = cv(ldo(U, ((bn * 36u + (uint32_t)(MU * 9 + 3 * a + c)) << 8) + ln));
          u.u[a][c] = cpx<float>{float(v.re), float(v.im)};
        }
    }
    accum_recon(acc, udagmul(u, h), MU, false);
  }
}

// block-restricted hop: neighbour from LDS rho, link from LDS.  Branch free: a
// lane whose neighbour lies outside the block reads the zero pad (sites
// 256..319 of each component row, stride kRhStride) and so adds nothing.
constexpr int kRhStride = 320;
template <int HOP>
__device__ __forceinline__ void blk_hop44(Spinor<float>& acc, const cpx<float>* rh, const cpx<float>* Ul, uint32_t l) {
  constexpr int MU = HOP / 2;
  constexpr bool FWD = HOP % 2 == 0;
  constexpr int SH = kSh44[MU];
  const uint32_t lc = (l >> SH) & 3u;
  const bool in = FWD ? lc < 3u : lc > 0u;
  const uint32_t ln = FWD ? l + (1u << SH) : l - (1u << SH);
  const uint32_t ls = in ? ln : 256u + (l & 63u);
  const Half<float> h = project(lds_spinor(rh, (int)ls, kRhStride), MU, FWD);
  const Link<float> u = lds_link(Ul, MU, (FWD || !in) ? l : ln);
  accum_recon(acc, FWD ? umul(u, h) : udagmul(u, h), MU, FWD);
}

// (m0+4 + C) v - tau Gamma5 v with the clover blocks held in registers
template <bool CLOVER>
__device__ __forceinline__ Spinor<float> diag_reg(const cpx<float> (&dg)[2][18], float mass4, const Spinor<float>& v,
                                                  float tau) {
  Spinor<float> o;
  if (CLOVER) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      cpx<float> in[6], w[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) in[i] = v.s[2 * h + i / 3][i % 3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        w[2 * k] = dg[h][k].re * in[2 * k];
        w[2 * k + 1] = dg[h][k].im * in[2 * k + 1];
      }
      int k = 3;
#pragma unroll
      for (int i = 1; i < 6; ++i)
#pragma unroll
        for (int j = 0; j < i; ++j) {
          cfma(w[i], dg[h][k], in[j]);
          cfma_conj(w[j], dg[h][k], in[i]);
          ++k;
        }
#pragma unroll
      for (int i = 0; i < 6; ++i) o.s[2 * h + i / 3][i % 3] = w[i];
    }
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) o.s[s][c] = mass4 * v.s[s][c];
  }
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) o.s[s][c] = (s < 2) ? o.s[s][c] - tau * v.s[s][c] : o.s[s][c] + tau * v.s[s][c];
  return o;
}

// sum of 3 values over the 256 threads of one rhs slot (waves 4q..4q+3).
// red is double buffered by the caller (alternate halves on successive calls),
// so one barrier suffices: a half is rewritten only two calls later, after
// every thread has passed the next call's barrier.
__device__ __forceinline__ void slot_sum3(float (&v)[3], float* red, int slot) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < 3; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0)
#pragma unroll
    for (int i = 0; i < 3; ++i) red[wave * 3 + i] = v[i];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    float t = red[(4 * slot) * 3 + i];
#pragma unroll
    for (int q = 1; q < 4; ++q) t += red[(4 * slot + q) * 3 + i];
    v[i] = t;
  }
}

template <typename S, bool CLOVER, int NS, bool QF>
__global__ __launch_bounds__(256 * NS) void k_sap44(SapArgs<S> a) {
  using P = typename PT<S>::stor;
  __shared__ cpx<float> Ul[36 * 256];
  __shared__ cpx<float> rhs_lds[NS][12 * kRhStride];
  __shared__ float red[2][4 * NS * 3];
  int rb = 0;
  const int w = blockIdx.x, nw = gridDim.x;
  const int L = ((nw & 7) == 0) ? (w & 7) * (nw >> 3) + (w >> 3) : w;
  const uint32_t b = (uint32_t)__builtin_amdgcn_readfirstlane(a.first_block + L);
  const uint32_t l = threadIdx.x & 255u;
  const int slot = (int)(threadIdx.x >> 8);
  cpx<float>* rh = rhs_lds[slot];
  const int* nbr = a.g.nbr;
  for (int i = (int)l; i < 12 * 64; i += 256) rh[(i >> 6) * kRhStride + 256 + (i & 63)] = czero<float>();
  for (int i = slot; i < 36; i += NS) {
    auto v = cv(ldo(a.U, ((b * 36u + (uint32_t)i) << 8) + l));
    Ul[i * 256 + l] = cpx<float>{float(v.re), float(v.im)};
  }
  cpx<float> dg[2][18];
  if (CLOVER) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int k = 0; k < 18; ++k) {
        auto v = cv(ldo(a.diag, ((b * 36u + (uint32_t)(h * 18 + k)) << 8) + l));
        dg[h][k] = cpx<float>{float(v.re), float(v.im)};
      }
  }
  const float mass4 = float(a.mass4);
  __syncthreads();
#pragma unroll 1
  for (int k0 = 0; k0 < a.nrhs; k0 += NS) {
    // both slots run every iteration (the barriers are work-group wide); a
    // slot past the last rhs recomputes rhs k0 and does not store
    const bool active = k0 + slot < a.nrhs;
    const int k = active ? k0 + slot : k0;
    P* x = a.x + (size_t)k * a.fstride;
    const P* f = a.f + (size_t)k * a.fstride;
    const float tau = float(a.tau[k]);
    Spinor<float> acc;
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.s[s][c] = czero<float>();
    // forward and backward hop of one direction together: their neighbour
    // loads are in flight at the same time (a full unroll spills)
#pragma unroll 1
    for (int mu = 0; mu < 4; ++mu) {
      switch (mu) {
        case 0: res_hop44<0>(acc, x, a.U, Ul, nbr, b, l); res_hop44<1>(acc, x, a.U, Ul, nbr, b, l); break;
        case 1: res_hop44<2>(acc, x, a.U, Ul, nbr, b, l); res_hop44<3>(acc, x, a.U, Ul, nbr, b, l); break;
        case 2: res_hop44<4>(acc, x, a.U, Ul, nbr, b, l); res_hop44<5>(acc, x, a.U, Ul, nbr, b, l); break;
        default: res_hop44<6>(acc, x, a.U, Ul, nbr, b, l); res_hop44<7>(acc, x, a.U, Ul, nbr, b, l); break;
      }
    }
    Spinor<float> xs = gl_spinor(x, b, l);
    Spinor<float> rho;
    {
      const Spinor<float> d = diag_reg<CLOVER>(dg, mass4, xs, tau);
      const Spinor<float> fs = gl_spinor(f, b, l);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const cpx<float> ax = d.s[s][c] - 0.5f * acc.s[s][c];
          rho.s[s][c] = (QF && s >= 2) ? fs.s[s][c] + ax : fs.s[s][c] - ax;
        }
    }
#pragma unroll 1
    for (int it = 0; it < a.n_mr; ++it) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) rh[(3 * s + c) * kRhStride + l] = rho.s[s][c];
      __syncthreads();
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) acc.s[s][c] = czero<float>();
#pragma unroll 1
      for (int hop = 0; hop < 8; ++hop) {
        switch (hop) {
          case 0: blk_hop44<0>(acc, rh, Ul, l); break;
          case 1: blk_hop44<1>(acc, rh, Ul, l); break;
          case 2: blk_hop44<2>(acc, rh, Ul, l); break;
          case 3: blk_hop44<3>(acc, rh, Ul, l); break;
          case 4: blk_hop44<4>(acc, rh, Ul, l); break;
          case 5: blk_hop44<5>(acc, rh, Ul, l); break;
          case 6: blk_hop44<6>(acc, rh, Ul, l); break;
          default: blk_hop44<7>(acc, rh, Ul, l); break;
        }
      }
      Spinor<float> q = diag_reg<CLOVER>(dg, mass4, rho, tau);
      float v[3] = {0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          q.s[s][c] = q.s[s][c] - 0.5f * acc.s[s][c];
          if (QF && s >= 2) q.s[s][c] = -q.s[s][c];
          const cpx<float> t = cmul_conj(q.s[s][c], rho.s[s][c]);
          v[0] += t.re;
          v[1] += t.im;
          v[2] += norm2(q.s[s][c]);
        }
      slot_sum3(v, red[rb], slot);
      rb ^= 1;
      cpx<float> alpha = czero<float>();
      if (v[2] > 0.f) alpha = cpx<float>{v[0] / v[2], v[1] / v[2]};
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xs.s[s][c] = xs.s[s][c] + alpha * rho.s[s][c];
          rho.s[s][c] = rho.s[s][c] - alpha * q.s[s][c];
        }
    }
    if (active) {
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int c = 0; c < 3; ++c)
          sto(x, ((b * 12u + (uint32_t)(3 * s + c)) << 8) + l, vc(xs.s[s][c], (P*)nullptr));
    }
    // the residual of the next rhs reads x of neighbouring blocks only, and
    // this work-group's own block is rewritten by this work-group alone
  }
}

template <typename S>
void launch_s(const qmg_ctx* c, int p, void* x, const void* f, const double* tau, int nrhs, int colour,
              int n_mr, hipStream_t s, bool qf) {
  using P = typename PT<S>::stor;
  using R = typename PT<S>::real;
  SapArgs<S> a;
  a.x = (P*)x;
  a.f = (const P*)f;
  a.U = (const P*)c->U[p];
  a.diag = (const P*)c->Dg[p];
  a.mass4 = c->m0 + 4.0;
  a.fstride = (int64_t)field_elems(c);
  a.nrhs = nrhs;
  a.first_block = colour == 0 ? 0 : c->g.ncol0;
  a.nblk = colour == 0 ? c->g.ncol0 : c->g.nb - c->g.ncol0;
  a.n_mr = n_mr;
  a.g = c->g;
  for (int i = 0; i < QMG_MAXRHS; ++i) a.tau[i] = i < nrhs ? tau[i] : 0.0;
  const int bs = 1 << c->g.bs_log;
  size_t lds = sizeof(cpx<R>) * 12 * bs + sizeof(R) * 3 * std::max(bs, 8);
  const bool b44 = c->g.block[0] == 4 && c->g.block[1] == 4 && c->g.block[2] == 4 && c->g.block[3] == 4;
  if constexpr (!std::is_same<S, double>::value) {
    if (b44 && c->tune.sap_variant >= 1) {
      dim3 grid((unsigned)a.nblk);
      if (c->tune.sap_variant == 2) {
        if (qf) {
          if (c->clover) hipLaunchKernelGGL((k_sap44<S, true, 2, true>), grid, dim3(512), 0, s, a);
          else hipLaunchKernelGGL((k_sap44<S, false, 2, true>), grid, dim3(512), 0, s, a);
        } else {
          if (c->clover) hipLaunchKernelGGL((k_sap44<S, true, 2, false>), grid, dim3(512), 0, s, a);
          else hipLaunchKernelGGL((k_sap44<S, false, 2, false>), grid, dim3(512), 0, s, a);
        }
      } else {
        if (qf) {
          if (c->clover) hipLaunchKernelGGL((k_sap44<S, true, 1, true>), grid, dim3(256), 0, s, a);
          else hipLaunchKernelGGL((k_sap44<S, false, 1, true>), grid, dim3(256), 0, s, a);
        } else {
          if (c->clover) hipLaunchKernelGGL((k_sap44<S, true, 1, false>), grid, dim3(256), 0, s, a);
          else hipLaunchKernelGGL((k_sap44<S, false, 1, false>), grid, dim3(256), 0, s, a);
        }
      }
      return;
    }
  }
  dim3 grid((unsigned)(a.nblk * nrhs));
  if (qf) {
    if (c->clover) hipLaunchKernelGGL((k_sap<S, true, true>), grid, dim3(bs), lds, s, a);
    else hipLaunchKernelGGL((k_sap<S, false, true>), grid, dim3(bs), lds, s, a);
  } else {
    if (c->clover) hipLaunchKernelGGL((k_sap<S, true, false>), grid, dim3(bs), lds, s, a);
    else hipLaunchKernelGGL((k_sap<S, false, false>), grid, dim3(bs), lds, s, a);
  }
}

}  // namespace

hipError_t launch_sap_colour(const qmg_ctx* c, int p, void* x, const void* f, const double* tau, int nrhs,
                             int colour, int n_mr, hipStream_t s, int qform) {
  if (p == QMG_F64) launch_s<double>(c, p, x, f, tau, nrhs, colour, n_mr, s, qform != 0);
  else if (p == QMG_F32) launch_s<float>(c, p, x, f, tau, nrhs, colour, n_mr, s, qform != 0);
  else launch_s<bf16_t>(c, p, x, f, tau, nrhs, colour, n_mr, s, qform != 0);
  return hipGetLastError();
}
