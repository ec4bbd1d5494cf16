// Interpolation P from test vectors, restriction y = P^H v and prolongation
// v = P y (Sec. 2: aggregation-based P, R = P^H; Sec. 3.1 on building P).
//
// Aggregates are (lattice block) x (chirality half): spins {0,1} and {2,3},
// so Gamma5 P = P Gamma5^c (text before eq. (2.9)).  P is stored complex
// [nb][2][ntv][6][bs]: column j of aggregate (b, h), entry (spin-in-half,
// colour) d at site l.  Coarse vectors are [nrhs][nb][2*ntv], index h*ntv + j.
// Columns of each aggregate are orthonormalised in column order, twice per
// column, by Gram-Schmidt over chunks of eight earlier columns (modified
// Gram-Schmidt in exact arithmetic).
#include "qmg_ctx.h"
#include "reduce.h"

namespace {

QMG_HD int64_t pidx(const Geom& g, int ntv, int b, int h, int j, int d, int l) {
  return ((((int64_t)b * 2 + h) * ntv + j) * 6 + d) * ((int64_t)1 << g.bs_log) + l;
}

// Column j of both chirality halves: orthogonalised against columns 0..j-1
// twice, eight columns at a time (the dot products of a chunk are reduced
// together, then the chunk is subtracted), then normalised.  Equal to
// modified Gram-Schmidt in exact arithmetic; one work-group reduction per
// chunk instead of one per column pair.
constexpr int kGsChunk = 8;
__global__ __launch_bounds__(256) void k_build_P(Geom g, double2* P, const double2* W, int ntv, int* fail) {
  extern __shared__ double red[];
  const int b = blockIdx.x, l = threadIdx.x;
  const int64_t fs = g.V * 12;
  for (int j = 0; j < ntv; ++j) {
    cpx<double> v[2][6];
    for (int h = 0; h < 2; ++h)
      for (int d = 0; d < 6; ++d) v[h][d] = ldc(W + j * fs, sidx(g, b, 6 * h + d, l));
    double n0[2] = {0, 0};
    for (int h = 0; h < 2; ++h)
      for (int d = 0; d < 6; ++d) n0[h] += norm2(v[h][d]);
    wg_sum<double, 2>(n0, red);
    for (int pass = 0; pass < 2; ++pass)
      for (int i0 = 0; i0 < j; i0 += kGsChunk) {
        // cf[4 t + 2 h + (0 re, 1 im)] = <P_{i0+t}, v> on chirality h
        double cf[4 * kGsChunk];
#pragma unroll
        for (int t = 0; t < kGsChunk; ++t) {
          const int i = i0 + t;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            cpx<double> a = czero<double>();
            if (i < j)
              for (int d = 0; d < 6; ++d) cfma_conj(a, ldc(P, pidx(g, ntv, b, h, i, d, l)), v[h][d]);
            cf[4 * t + 2 * h] = a.re;
            cf[4 * t + 2 * h + 1] = a.im;
          }
        }
        wg_sum<double, 4 * kGsChunk>(cf, red);
#pragma unroll
        for (int t = 0; t < kGsChunk; ++t) {
          const int i = i0 + t;
          if (i < j)
            for (int h = 0; h < 2; ++h) {
              const cpx<double> c = {cf[4 * t + 2 * h], cf[4 * t + 2 * h + 1]};
              for (int d = 0; d < 6; ++d) v[h][d] = v[h][d] - c * ldc(P, pidx(g, ntv, b, h, i, d, l));
            }
        }
      }
    double n1[2] = {0, 0};
    for (int h = 0; h < 2; ++h)
      for (int d = 0; d < 6; ++d) n1[h] += norm2(v[h][d]);
    wg_sum<double, 2>(n1, red);
    for (int h = 0; h < 2; ++h) {
      double nn = sqrt(n1[h]);
      if (!(nn >= 1e-12 * sqrt(n0[h]))) {
        if (l == 0) fail[0] = 1;
        nn = 1.0;
      }
      double inv = 1.0 / nn;
      for (int d = 0; d < 6; ++d) stc(P, pidx(g, ntv, b, h, j, d, l), inv * v[h][d]);
    }
  }
}

// y[k][b][o] = sum_{l,d} conj(P[b][h][j][d][l]) v[k][b][6h+d][l], o = h*ntv + j
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_restrict(Geom g, typename PT<C>::stor* y, const typename PT<S>::stor* P,
                                                  const typename PT<S>::stor* v, int ntv, int nrhs,
                                                  int64_t fstride, int64_t ysk, int64_t ysb) {
  using R = typename PT<S>::real;
  extern __shared__ unsigned char smem_r[];
  R* red = reinterpret_cast<R*>(smem_r);
  const int b = blockIdx.x / nrhs, k = blockIdx.x % nrhs, l = threadIdx.x;
  const int nc = 2 * ntv;
  cpx<R> vv[12];
  for (int c = 0; c < 12; ++c) vv[c] = ldcv<R>(v + k * fstride, sidx(g, b, c, l));
  auto* yo = y + k * ysk + b * ysb;
#pragma unroll
  for (int h = 0; h < 2; ++h)
    for (int j0 = 0; j0 < ntv; j0 += 8) {
      R acc[16];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int j = j0 + t;
        cpx<R> s = czero<R>();
        if (j < ntv)
#pragma unroll
          for (int d = 0; d < 6; ++d) s = s + cmul_conj(ldcv<R>(P, pidx(g, ntv, b, h, j, d, l)), vv[6 * h + d]);
        acc[2 * t] = s.re;
        acc[2 * t + 1] = s.im;
      }
      wg_sum<R, 16>(acc, red);
      if (l < 8 && j0 + l < ntv) {
        R re = acc[0], im = acc[1];
#pragma unroll
        for (int t = 1; t < 8; ++t)
          if (t == l) { re = acc[2 * t]; im = acc[2 * t + 1]; }
        stcv(yo, h * ntv + j0 + l, cpx<R>{re, im});
      }
    }
}

// v[k][b][6h+d][l] = sum_j P[b][h][j][d][l] y[k][b][h*ntv+j]
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_prolong(Geom g, typename PT<S>::stor* v, const typename PT<S>::stor* P,
                                                 const typename PT<C>::stor* y, int ntv, int nrhs,
                                                 int64_t fstride) {
  using R = typename PT<S>::real;
  __shared__ cpx<R> ys[64];
  const int b = blockIdx.x / nrhs, k = blockIdx.x % nrhs, l = threadIdx.x;
  const int nc = 2 * ntv;
  const auto* yi = y + ((int64_t)k * g.nb + b) * nc;
  for (int o = l; o < nc; o += blockDim.x) ys[o] = ldcv<R>(yi, o);
  __syncthreads();
  for (int h = 0; h < 2; ++h)
    for (int d = 0; d < 6; ++d) {
      cpx<R> s = czero<R>();
      for (int j = 0; j < ntv; ++j) s = s + ldcv<R>(P, pidx(g, ntv, b, h, j, d, l)) * ys[h * ntv + j];
      stcv(v + k * fstride, sidx(g, b, 6 * h + d, l), s);
    }
}

// ---- many right-hand sides: R rhs per work-group share every P load
template <typename S, typename C, int R>
__global__ __launch_bounds__(256) void k_restrict_mr(Geom g, typename PT<C>::stor* y, const typename PT<S>::stor* P,
                                                     const typename PT<S>::stor* v, int ntv, int nrhs,
                                                     int64_t fstride) {
  using Rr = typename PT<S>::real;
  extern __shared__ unsigned char smem_r[];
  Rr* red = reinterpret_cast<Rr*>(smem_r);
  const int ng = (nrhs + R - 1) / R;
  const int b = blockIdx.x / ng, k0 = (blockIdx.x % ng) * R, l = threadIdx.x;
  const int nr = nrhs - k0 < R ? nrhs - k0 : R;
  const int nc = 2 * ntv;
  cpx<Rr> vv[R][12];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int c = 0; c < 12; ++c)
      vv[r][c] = r < nr ? ldcv<Rr>(v + (int64_t)(k0 + r) * fstride, sidx(g, b, c, l)) : czero<Rr>();
#pragma unroll
  for (int h = 0; h < 2; ++h)
    for (int j0 = 0; j0 < ntv; j0 += 4) {
      Rr acc[8 * R];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int j = j0 + t;
        cpx<Rr> pv[6];
#pragma unroll
        for (int d = 0; d < 6; ++d) pv[d] = j < ntv ? ldcv<Rr>(P, pidx(g, ntv, b, h, j, d, l)) : czero<Rr>();
#pragma unroll
        for (int r = 0; r < R; ++r) {
          cpx<Rr> sum = czero<Rr>();
#pragma unroll
          for (int d = 0; d < 6; ++d) sum = sum + cmul_conj(pv[d], vv[r][6 * h + d]);
          acc[(r * 4 + t) * 2] = sum.re;
          acc[(r * 4 + t) * 2 + 1] = sum.im;
        }
      }
      wg_sum<Rr, 8 * R>(acc, red);
      if (l < 4 * R) {
        const int r = l / 4, t = l % 4;
        Rr re = acc[0], im = acc[1];
#pragma unroll
        for (int q = 1; q < 4 * R; ++q)
          if (q == l) { re = acc[2 * q]; im = acc[2 * q + 1]; }
        if (r < nr && j0 + t < ntv) stcv(y + ((int64_t)(k0 + r) * g.nb + b) * nc, h * ntv + j0 + t, cpx<Rr>{re, im});
      }
    }
}

// P read once per site for every rhs: the coarse inputs of the block live in LDS
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_prolong_mr(Geom g, typename PT<S>::stor* v, const typename PT<S>::stor* P,
                                                    const typename PT<C>::stor* y, int ntv, int nrhs, int64_t fstride) {
  using R = typename PT<S>::real;
  __shared__ cpx<R> ys[QMG_MAXRHS * 64];
  const int b = blockIdx.x, l = threadIdx.x;
  const int nc = 2 * ntv;
  for (int o = l; o < nrhs * nc; o += blockDim.x) {
    const int k = o / nc, i = o % nc;
    ys[k * 64 + i] = ldcv<R>(y + ((int64_t)k * g.nb + b) * nc, i);
  }
  __syncthreads();
  for (int h = 0; h < 2; ++h)
    for (int d = 0; d < 6; ++d) {
      cpx<R> pc[32];
#pragma unroll
      for (int j = 0; j < 32; ++j) pc[j] = j < ntv ? ldcv<R>(P, pidx(g, ntv, b, h, j, d, l)) : czero<R>();
      for (int k = 0; k < nrhs; ++k) {
        cpx<R> s = czero<R>();
#pragma unroll
        for (int j = 0; j < 32; ++j)
          if (j < ntv) s = s + pc[j] * ys[k * 64 + h * ntv + j];
        stcv(v + (int64_t)k * fstride, sidx(g, b, 6 * h + d, l), s);
      }
    }
}

// ---- restriction on MFMA: per block and chirality h, Y_h (ntv x 16 rhs) =
// P_h^H (ntv x K) V_h (K x 16), K = 6 * 256 (spin-in-half, colour, site),
// as four real 16x16x4 products per k-step.  One wave per chirality; the 4 k
// values of a step are 4 sites (stride 4) with the same (spin, colour).
typedef float tf4 __attribute__((ext_vector_type(4)));
typedef double td4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ tf4 tmfma(float a, float b, tf4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
__device__ __forceinline__ td4 tmfma(double a, double b, td4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
template <typename R> struct TAcc;
template <> struct TAcc<float> { using T = tf4; };
template <> struct TAcc<double> { using T = td4; };
template <typename R> __device__ __forceinline__ int trow(int l, int r);
template <> __device__ __forceinline__ int trow<float>(int l, int r) { return 4 * (l >> 4) + r; }
template <> __device__ __forceinline__ int trow<double>(int l, int r) { return 4 * r + (l >> 4); }

template <typename S, typename C, int MT>
__global__ __launch_bounds__(128) void k_restrict_mfma(Geom g, typename PT<C>::stor* y, const typename PT<S>::stor* P,
                                                       const typename PT<S>::stor* v, int ntv, int nrhs, int64_t fstride) {
  using R = typename PT<S>::real;
  using AT = typename TAcc<R>::T;
  const int b = blockIdx.x, n0 = blockIdx.y * 16;
  const int h = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ln = lane & 15, lk = lane >> 4;
  const int n = n0 + ln;
  const bool nok = n < nrhs;
  const auto* vn = v + (int64_t)(nok ? n : 0) * fstride;
  AT acc_re[MT], acc_im[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) {
    acc_re[t] = AT{0, 0, 0, 0};
    acc_im[t] = AT{0, 0, 0, 0};
  }
  // each (spin, colour) row of 256 sites is summed in a fresh accumulator and
  // then added to the total: accumulation depth 64 + 6 instead of 384
#pragma unroll 1
  for (int d = 0; d < 6; ++d) {
    AT part_re[MT], part_im[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      part_re[t] = AT{0, 0, 0, 0};
      part_im[t] = AT{0, 0, 0, 0};
    }
    // 16 sites per step: lane (ln, lk) loads sites l0 + 4 lk .. l0 + 4 lk + 3 of
    // its P row and rhs with two wide loads; MFMA q takes site l0 + 4 lk + q in
    // k-slot lk (the same site order in A and B, so the sum is unchanged)
#pragma unroll 2
    for (int l0 = 0; l0 < 256; l0 += 16) {
      const int l = l0 + 4 * lk;
      cpx<R> bv[4];
      ld4c(vn + sidx(g, b, 6 * h + d, l), bv);
      if (!nok)
#pragma unroll
        for (int q = 0; q < 4; ++q) bv[q] = czero<R>();
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        const int i = 16 * t + ln;
        cpx<R> p[4];
        if (i < ntv) ld4c(P + pidx(g, ntv, b, h, i, d, l), p);
        else
#pragma unroll
          for (int q = 0; q < 4; ++q) p[q] = czero<R>();
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // A = conj(P): (p.re, -p.im)
          part_re[t] = tmfma(p[q].re, bv[q].re, part_re[t]);
          part_re[t] = tmfma(p[q].im, bv[q].im, part_re[t]);
          part_im[t] = tmfma(p[q].re, bv[q].im, part_im[t]);
          part_im[t] = tmfma(-p[q].im, bv[q].re, part_im[t]);
        }
      }
    }
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      acc_re[t] += part_re[t];
      acc_im[t] += part_im[t];
    }
  }
  if (!nok) return;
  const int nc = 2 * ntv;
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * t + trow<R>(lane, r);
      if (i < ntv) stcv(y + ((int64_t)n * g.nb + b) * nc, h * ntv + i, cpx<R>{acc_re[t][r], acc_im[t][r]});
    }
}

// ---- prolongation on MFMA: per block b, chirality h and spin-colour row d,
// the tile v[n0..n0+15][6h+d][16 sites] = Y^T (16 rhs x ntv) P_hd (ntv x 16
// sites); Y^T stays in registers for the 96 tiles of (b, h), four waves share them.
template <typename S, typename C>
__global__ __launch_bounds__(256) void k_prolong_mfma(Geom g, typename PT<S>::stor* v, const typename PT<S>::stor* P,
                                                      const typename PT<C>::stor* y, int ntv, int nrhs,
                                                      int64_t fstride) {
  using R = typename PT<S>::real;
  using AT = typename TAcc<R>::T;
  const int b = blockIdx.x, h = blockIdx.y, n0 = blockIdx.z * 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int ln = lane & 15, lk = lane >> 4;
  const int nc = 2 * ntv, nks = (ntv + 3) >> 2;
  const bool nok = n0 + ln < nrhs;
  cpx<R> ya[8];
#pragma unroll
  for (int st = 0; st < 8; ++st) {
    const int j = 4 * st + lk;
    ya[st] = (st < nks && nok && j < ntv) ? ldcv<R>(y, ((int64_t)(n0 + ln) * g.nb + b) * nc + h * ntv + j)
                                          : czero<R>();
  }
#pragma unroll 1
  for (int tile = wave; tile < 96; tile += 4) {
    const int d = tile >> 4, s0 = (tile & 15) << 4;
    AT cre = AT{0, 0, 0, 0}, cim = AT{0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < 8; ++st) {
      if (st < nks) {
        const int j = 4 * st + lk;
        const cpx<R> pb = j < ntv ? ldcv<R>(P, pidx(g, ntv, b, h, j, d, s0 + ln)) : czero<R>();
        cre = tmfma(ya[st].re, pb.re, cre);
        cre = tmfma(-ya[st].im, pb.im, cre);
        cim = tmfma(ya[st].re, pb.im, cim);
        cim = tmfma(ya[st].im, pb.re, cim);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int n = n0 + trow<R>(lane, r);
      if (n < nrhs) stcv(v + (int64_t)n * fstride, sidx(g, b, 6 * h + d, s0 + ln), cpx<R>{cre[r], cim[r]});
    }
  }
}

template <typename S>
void restrict_t(const qmg_ctx* c, void* yc, const void* v, int nrhs, hipStream_t s, int p) {
  using P = typename PT<S>::stor;
  using R = typename PT<S>::real;
  const int bs = 1 << c->g.bs_log;
  size_t lds = sizeof(R) * 16 * std::max(bs, 4);
  if (nrhs >= c->tune.restrict_mfma_min_rhs && bs == 256 && c->ntv <= 32) {
    dim3 grid(c->g.nb, (nrhs + 15) / 16);
    const int mt = (c->ntv + 15) / 16;
    auto go = [&](auto mtc) {
      constexpr int MT = decltype(mtc)::value;
      if (p == QMG_F64)
        hipLaunchKernelGGL((k_restrict_mfma<S, double, MT>), grid, dim3(128), 0, s, c->g, (double2*)yc,
                           (const P*)c->P[p], (const P*)v, c->ntv, nrhs, (int64_t)field_elems(c));
      else
        hipLaunchKernelGGL((k_restrict_mfma<S, float, MT>), grid, dim3(128), 0, s, c->g, (float2*)yc,
                           (const P*)c->P[p], (const P*)v, c->ntv, nrhs, (int64_t)field_elems(c));
    };
    if (mt == 1) go(std::integral_constant<int, 1>{});
    else go(std::integral_constant<int, 2>{});
    return;
  }
  if (nrhs > 1 && c->tune.transfer_mr) {
    constexpr int RR = std::is_same<S, double>::value ? 2 : 4;
    const int ng = (nrhs + RR - 1) / RR;
    const size_t lds2 = sizeof(R) * 8 * RR * std::max(bs, 4);
    if (p == QMG_F64)
      hipLaunchKernelGGL((k_restrict_mr<S, double, RR>), dim3(c->g.nb * ng), dim3(bs), lds2, s, c->g, (double2*)yc,
                         (const P*)c->P[p], (const P*)v, c->ntv, nrhs, (int64_t)field_elems(c));
    else
      hipLaunchKernelGGL((k_restrict_mr<S, float, RR>), dim3(c->g.nb * ng), dim3(bs), lds2, s, c->g, (float2*)yc,
                         (const P*)c->P[p], (const P*)v, c->ntv, nrhs, (int64_t)field_elems(c));
    return;
  }
  if (p == QMG_F64)
    hipLaunchKernelGGL((k_restrict<S, double>), dim3(c->g.nb * nrhs), dim3(bs), lds, s, c->g, (double2*)yc,
                       (const P*)c->P[p], (const P*)v, c->ntv, nrhs, (int64_t)field_elems(c),
                       (int64_t)c->g.nb * 2 * c->ntv, (int64_t)2 * c->ntv);
  else
    hipLaunchKernelGGL((k_restrict<S, float>), dim3(c->g.nb * nrhs), dim3(bs), lds, s, c->g, (float2*)yc,
                       (const P*)c->P[p], (const P*)v, c->ntv, nrhs, (int64_t)field_elems(c),
                       (int64_t)c->g.nb * 2 * c->ntv, (int64_t)2 * c->ntv);
}

template <typename S>
void prolong_t(const qmg_ctx* c, void* v, const void* yc, int nrhs, hipStream_t s, int p) {
  using P = typename PT<S>::stor;
  const int bs = 1 << c->g.bs_log;
  if (nrhs >= c->tune.restrict_mfma_min_rhs && bs == 256 && c->ntv <= 32) {
    dim3 grid(c->g.nb, 2, (nrhs + 15) / 16);
    if (p == QMG_F64)
      hipLaunchKernelGGL((k_prolong_mfma<S, double>), grid, dim3(256), 0, s, c->g, (P*)v, (const P*)c->P[p],
                         (const double2*)yc, c->ntv, nrhs, (int64_t)field_elems(c));
    else
      hipLaunchKernelGGL((k_prolong_mfma<S, float>), grid, dim3(256), 0, s, c->g, (P*)v, (const P*)c->P[p],
                         (const float2*)yc, c->ntv, nrhs, (int64_t)field_elems(c));
    return;
  }
  if (nrhs > 1 && c->tune.transfer_mr) {
    if (p == QMG_F64)
      hipLaunchKernelGGL((k_prolong_mr<S, double>), dim3(c->g.nb), dim3(bs), 0, s, c->g, (P*)v, (const P*)c->P[p],
                         (const double2*)yc, c->ntv, nrhs, (int64_t)field_elems(c));
    else
      hipLaunchKernelGGL((k_prolong_mr<S, float>), dim3(c->g.nb), dim3(bs), 0, s, c->g, (P*)v, (const P*)c->P[p],
                         (const float2*)yc, c->ntv, nrhs, (int64_t)field_elems(c));
    return;
  }
  if (p == QMG_F64)
    hipLaunchKernelGGL((k_prolong<S, double>), dim3(c->g.nb * nrhs), dim3(bs), 0, s, c->g, (P*)v,
                       (const P*)c->P[p], (const double2*)yc, c->ntv, nrhs, (int64_t)field_elems(c));
  else
    hipLaunchKernelGGL((k_prolong<S, float>), dim3(c->g.nb * nrhs), dim3(bs), 0, s, c->g, (P*)v,
                       (const P*)c->P[p], (const float2*)yc, c->ntv, nrhs, (int64_t)field_elems(c));
}

}  // namespace

hipError_t launch_build_P(const qmg_ctx* c, void* P64, const void* W, int ntv, int* d_fail, hipStream_t s) {
  const int bs = 1 << c->g.bs_log;
  // wg_sum scratch: 4 kGsChunk values per wave (per lane below 64 lanes)
  size_t lds = sizeof(double) * 4 * kGsChunk * (bs >= 64 ? bs / 64 : bs);
  hipLaunchKernelGGL(k_build_P, dim3(c->g.nb), dim3(bs), lds, s, c->g, (double2*)P64, (const double2*)W, ntv,
                     d_fail);
  return hipGetLastError();
}

hipError_t launch_restrict(const qmg_ctx* c, int p, void* yc, const void* v, int nrhs, hipStream_t s) {
  if (p == QMG_F64) restrict_t<double>(c, yc, v, nrhs, s, p);
  else if (p == QMG_F32) restrict_t<float>(c, yc, v, nrhs, s, p);
  else restrict_t<bf16_t>(c, yc, v, nrhs, s, p);
  return hipGetLastError();
}

hipError_t launch_prolong(const qmg_ctx* c, int p, void* v, const void* yc, int nrhs, hipStream_t s) {
  if (p == QMG_F64) prolong_t<double>(c, v, yc, nrhs, s, p);
  else if (p == QMG_F32) prolong_t<float>(c, v, yc, nrhs, s, p);
  else prolong_t<bf16_t>(c, v, yc, nrhs, s, p);
  return hipGetLastError();
}
