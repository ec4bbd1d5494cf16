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

template <typename S, bool CLOVER>
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
      for (int c = 0; c < 3; ++c) rho.s[s][c] = fs.s[s][c] - (d.s[s][c] - R(0.5) * acc.s[s][c]);
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

template <typename S>
void launch_s(const qmg_ctx* c, int p, void* x, const void* f, const double* tau, int nrhs, int colour,
              int n_mr, hipStream_t s) {
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
  dim3 grid((unsigned)(a.nblk * nrhs));
  if (c->clover) hipLaunchKernelGGL((k_sap<S, true>), grid, dim3(bs), lds, s, a);
  else hipLaunchKernelGGL((k_sap<S, false>), grid, dim3(bs), lds, s, a);
}

}  // namespace

hipError_t launch_sap_colour(const qmg_ctx* c, int p, void* x, const void* f, const double* tau, int nrhs,
                             int colour, int n_mr, hipStream_t s) {
  if (p == QMG_F64) launch_s<double>(c, p, x, f, tau, nrhs, colour, n_mr, s);
  else if (p == QMG_F32) launch_s<float>(c, p, x, f, tau, nrhs, colour, n_mr, s);
  else launch_s<bf16_t>(c, p, x, f, tau, nrhs, colour, n_mr, s);
  return hipGetLastError();
}
