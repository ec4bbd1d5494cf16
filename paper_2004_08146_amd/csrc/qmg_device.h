// Device-side building blocks shared by the qmg kernels: complex arithmetic,
// storage precisions, the block-major field layout, the Wilson spin projectors
// and SU(3) colour products.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define QMG_HD __host__ __device__ __forceinline__

// ---------------------------------------------------------------- complex --
template <typename T>
struct cpx {
  T re, im;
};
template <typename T> QMG_HD cpx<T> mk(T r, T i) { return cpx<T>{r, i}; }
template <typename T> QMG_HD cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T> QMG_HD cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <typename T> QMG_HD cpx<T> operator-(cpx<T> a) { return {-a.re, -a.im}; }
template <typename T> QMG_HD cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T> QMG_HD cpx<T> operator*(T s, cpx<T> a) { return {s * a.re, s * a.im}; }
template <typename T> QMG_HD cpx<T> conj(cpx<T> a) { return {a.re, -a.im}; }
// i*a and -i*a
template <typename T> QMG_HD cpx<T> ti(cpx<T> a) { return {-a.im, a.re}; }
template <typename T> QMG_HD cpx<T> tmi(cpx<T> a) { return {a.im, -a.re}; }
// conj(a) * b
template <typename T> QMG_HD cpx<T> cmul_conj(cpx<T> a, cpx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <typename T> QMG_HD T norm2(cpx<T> a) { return a.re * a.re + a.im * a.im; }
// fused multiply-add chains (the compiler does not contract a + (b*c - d*e))
QMG_HD float fmar(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
QMG_HD double fmar(double a, double b, double c) { return __builtin_fma(a, b, c); }
// acc += a * b
template <typename T> QMG_HD void cfma(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fmar(a.re, b.re, acc.re);
  acc.re = fmar(-a.im, b.im, acc.re);
  acc.im = fmar(a.re, b.im, acc.im);
  acc.im = fmar(a.im, b.re, acc.im);
}
// acc += conj(a) * b
template <typename T> QMG_HD void cfma_conj(cpx<T>& acc, cpx<T> a, cpx<T> b) {
  acc.re = fmar(a.re, b.re, acc.re);
  acc.re = fmar(a.im, b.im, acc.re);
  acc.im = fmar(a.re, b.im, acc.im);
  acc.im = fmar(-a.im, b.re, acc.im);
}
template <typename T> QMG_HD cpx<T> czero() { return {T(0), T(0)}; }

// ------------------------------------------------------------- precisions --
// Storage precisions: double, float, and bf16 (tag type; arithmetic in float).
struct bf16_t {};

template <typename S> struct PT;
template <> struct PT<double> { using real = double; using stor = double2; };
template <> struct PT<float> { using real = float; using stor = float2; };
template <> struct PT<bf16_t> { using real = float; using stor = uint32_t; };

// float -> bfloat16 bits, round to nearest even (NaN kept quiet).
QMG_HD uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
QMG_HD float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }

QMG_HD cpx<double> ldc(const double2* p, int64_t i) { double2 v = p[i]; return {v.x, v.y}; }
QMG_HD cpx<float> ldc(const float2* p, int64_t i) { float2 v = p[i]; return {v.x, v.y}; }
QMG_HD cpx<float> ldc(const uint32_t* p, int64_t i) {
  uint32_t v = p[i];
  return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)};
}
QMG_HD void stc(double2* p, int64_t i, cpx<double> a) { p[i] = make_double2(a.re, a.im); }
QMG_HD void stc(float2* p, int64_t i, cpx<float> a) { p[i] = make_float2(a.re, a.im); }
QMG_HD void stc(uint32_t* p, int64_t i, cpx<float> a) {
  p[i] = f32_to_bf16_bits(a.re) | (f32_to_bf16_bits(a.im) << 16);
}
// generic converting load into compute type R
template <typename R, typename P> QMG_HD cpx<R> ldcv(const P* p, int64_t i) {
  auto v = ldc(p, i);
  return {R(v.re), R(v.im)};
}
template <typename P, typename R> QMG_HD void stcv(P* p, int64_t i, cpx<R> a) {
  using T = decltype(ldc(p, 0).re);
  stc(p, i, cpx<T>{T(a.re), T(a.im)});
}

// load / store with a 32-bit element offset from a uniform base pointer (the
// compiler then addresses with an SGPR base and one VGPR offset)
template <typename P> QMG_HD P ldo(const P* base, uint32_t elem) {
  return *reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) + (size_t)(elem * (uint32_t)sizeof(P)));
}
template <typename P> QMG_HD void sto(P* base, uint32_t elem, P v) {
  *reinterpret_cast<P*>(reinterpret_cast<char*>(base) + (size_t)(elem * (uint32_t)sizeof(P))) = v;
}
// store through the non-temporal path (the line is not kept in the caches)
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
QMG_HD void sto_nt(double2* base, uint32_t elem, double2 v) {
  __builtin_nontemporal_store(nt_d2{v.x, v.y}, reinterpret_cast<nt_d2*>(reinterpret_cast<char*>(base) +
                                                                       (size_t)(elem * (uint32_t)sizeof(double2))));
}
QMG_HD void sto_nt(float2* base, uint32_t elem, float2 v) {
  __builtin_nontemporal_store(nt_f2{v.x, v.y}, reinterpret_cast<nt_f2*>(reinterpret_cast<char*>(base) +
                                                                      (size_t)(elem * (uint32_t)sizeof(float2))));
}
QMG_HD void sto_nt(uint32_t* base, uint32_t elem, uint32_t v) {
  __builtin_nontemporal_store(v, reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(base) +
                                                            (size_t)(elem * (uint32_t)sizeof(uint32_t))));
}
QMG_HD cpx<double> cv(double2 v) { return {v.x, v.y}; }
QMG_HD cpx<float> cv(float2 v) { return {v.x, v.y}; }
QMG_HD cpx<float> cv(uint32_t v) { return {__uint_as_float(v << 16), __uint_as_float(v & 0xffff0000u)}; }
QMG_HD double2 vc(cpx<double> a, double2*) { return make_double2(a.re, a.im); }
QMG_HD float2 vc(cpx<float> a, float2*) { return make_float2(a.re, a.im); }
QMG_HD uint32_t vc(cpx<float> a, uint32_t*) { return f32_to_bf16_bits(a.re) | (f32_to_bf16_bits(a.im) << 16); }

// 4 consecutive complex entries (16-byte aligned) with wide loads, converted to R
template <typename R>
__device__ __forceinline__ void ld4c(const double2* p, cpx<R> (&f)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double2 v = p[q];
    f[q] = {R(v.x), R(v.y)};
  }
}
template <typename R>
__device__ __forceinline__ void ld4c(const float2* p, cpx<R> (&f)[4]) {
  const float4 a = reinterpret_cast<const float4*>(p)[0], b = reinterpret_cast<const float4*>(p)[1];
  f[0] = {R(a.x), R(a.y)};
  f[1] = {R(a.z), R(a.w)};
  f[2] = {R(b.x), R(b.y)};
  f[3] = {R(b.z), R(b.w)};
}
template <typename R>
__device__ __forceinline__ void ld4c(const uint32_t* p, cpx<R> (&f)[4]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const cpx<float> v = cv(w[q]);
    f[q] = {R(v.re), R(v.im)};
  }
}


// ------------------------------------------------------------------ layout --
// Sites are grouped in blocks of B0 x B1 x B2 x B3 (powers of two), numbered
// colour-major (all red blocks, then all black blocks).  A site is (b, l) with
// l the lexicographic index inside its block.  One spinor field is complex
// [nb][12][bs] (component 3*spin + colour); the gauge field is complex
// [nb][4][9][bs]; the clover-plus-mass diagonal is complex [nb][2][18][bs]
// (per chirality: 3 pairs of real diagonal entries, then the 15 lower
// off-diagonal entries (i > j) row by row).
struct Geom {
  int dims[4];
  int block[4];
  int nbk[4];     // blocks per direction
  int sh[4];      // bit shift of local coordinate mu inside l
  int msk[4];     // block[mu] - 1
  int bs_log;     // log2(sites per block)
  int nb;         // number of blocks
  int ncol0;      // number of colour-0 blocks (ids 0..ncol0-1)
  int64_t V;
  const int* nbr;     // [nb][8] neighbour block: 2*mu forward, 2*mu+1 backward
  const int* bcoord;  // [nb][4] block coordinates
  const int* lexord;  // [nb] block id of the i-th block in lexicographic order
};

QMG_HD int loc(const Geom& g, int l, int mu) { return (l >> g.sh[mu]) & g.msk[mu]; }

// neighbour (b', l') of site (b, l) in direction +mu / -mu (periodic)
QMG_HD void nb_fwd(const Geom& g, int b, int l, int mu, int& bo, int& lo) {
  if (loc(g, l, mu) < g.msk[mu]) { bo = b; lo = l + (1 << g.sh[mu]); }
  else { bo = g.nbr[b * 8 + 2 * mu]; lo = l - (g.msk[mu] << g.sh[mu]); }
}
QMG_HD void nb_bwd(const Geom& g, int b, int l, int mu, int& bo, int& lo) {
  if (loc(g, l, mu) > 0) { bo = b; lo = l - (1 << g.sh[mu]); }
  else { bo = g.nbr[b * 8 + 2 * mu + 1]; lo = l + (g.msk[mu] << g.sh[mu]); }
}
// index (in complex elements) of component c of site (b, l) in a field
QMG_HD int64_t sidx(const Geom& g, int b, int c, int l) {
  return (((int64_t)b * 12 + c) << g.bs_log) + l;
}
QMG_HD int64_t uidx(const Geom& g, int b, int mu, int ab, int l) {
  return (((int64_t)b * 36 + mu * 9 + ab) << g.bs_log) + l;
}
QMG_HD int64_t didx(const Geom& g, int b, int h, int k, int l) {
  return (((int64_t)b * 36 + h * 18 + k) << g.bs_log) + l;
}
// canonical site index of (b, l)
QMG_HD int64_t canon_site(const Geom& g, int b, int l) {
  int64_t s = 0;
  for (int mu = 0; mu < 4; ++mu)
    s = s * g.dims[mu] + (int64_t)g.bcoord[b * 4 + mu] * g.block[mu] + loc(g, l, mu);
  return s;
}

// ------------------------------------------------------------ spin algebra --
// A spinor at one site: 4 spins x 3 colours.  Gamma basis (chiral):
// gamma0 = [[0,-I],[-I,0]], gamma_k = [[0,-i sigma_k],[i sigma_k,0]],
// gamma5 = diag(1,1,-1,-1).  For the hop terms (I -/+ gamma_mu) only two spin
// combinations h0, h1 (a half spinor) are independent; the lower two spins
// are recovered from the colour-rotated half spinor.
template <typename R> struct Spinor { cpx<R> s[4][3]; };
template <typename R> struct Half { cpx<R> h[2][3]; };

// project with (I - gamma_mu) (fwd = true) or (I + gamma_mu) (fwd = false)
template <typename R>
QMG_HD Half<R> project(const Spinor<R>& p, int mu, bool fwd) {
  Half<R> o;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cpx<R> p0 = p.s[0][c], p1 = p.s[1][c], p2 = p.s[2][c], p3 = p.s[3][c];
    switch (mu) {
      case 0:
        if (fwd) { o.h[0][c] = p0 + p2; o.h[1][c] = p1 + p3; }
        else { o.h[0][c] = p0 - p2; o.h[1][c] = p1 - p3; }
        break;
      case 1:
        if (fwd) { o.h[0][c] = p0 + ti(p3); o.h[1][c] = p1 + ti(p2); }
        else { o.h[0][c] = p0 - ti(p3); o.h[1][c] = p1 - ti(p2); }
        break;
      case 2:
        if (fwd) { o.h[0][c] = p0 + p3; o.h[1][c] = p1 - p2; }
        else { o.h[0][c] = p0 - p3; o.h[1][c] = p1 + p2; }
        break;
      default:
        if (fwd) { o.h[0][c] = p0 + ti(p2); o.h[1][c] = p1 - ti(p3); }
        else { o.h[0][c] = p0 - ti(p2); o.h[1][c] = p1 + ti(p3); }
        break;
    }
  }
  return o;
}

// acc += full spinor rebuilt from the colour-rotated half spinor w
template <typename R>
QMG_HD void accum_recon(Spinor<R>& acc, const Half<R>& w, int mu, bool fwd) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cpx<R> h0 = w.h[0][c], h1 = w.h[1][c];
    acc.s[0][c] = acc.s[0][c] + h0;
    acc.s[1][c] = acc.s[1][c] + h1;
    switch (mu) {
      case 0:
        if (fwd) { acc.s[2][c] = acc.s[2][c] + h0; acc.s[3][c] = acc.s[3][c] + h1; }
        else { acc.s[2][c] = acc.s[2][c] - h0; acc.s[3][c] = acc.s[3][c] - h1; }
        break;
      case 1:
        if (fwd) { acc.s[2][c] = acc.s[2][c] + tmi(h1); acc.s[3][c] = acc.s[3][c] + tmi(h0); }
        else { acc.s[2][c] = acc.s[2][c] + ti(h1); acc.s[3][c] = acc.s[3][c] + ti(h0); }
        break;
      case 2:
        if (fwd) { acc.s[2][c] = acc.s[2][c] - h1; acc.s[3][c] = acc.s[3][c] + h0; }
        else { acc.s[2][c] = acc.s[2][c] + h1; acc.s[3][c] = acc.s[3][c] - h0; }
        break;
      default:
        if (fwd) { acc.s[2][c] = acc.s[2][c] + tmi(h0); acc.s[3][c] = acc.s[3][c] + ti(h1); }
        else { acc.s[2][c] = acc.s[2][c] + ti(h0); acc.s[3][c] = acc.s[3][c] + tmi(h1); }
        break;
    }
  }
}

template <typename R> struct Link { cpx<R> u[3][3]; };

// w = U h (per spin row of the half spinor)
template <typename R>
QMG_HD Half<R> umul(const Link<R>& U, const Half<R>& h) {
  Half<R> o;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a)
    {
      cpx<R> t = U.u[a][0] * h.h[s][0];
      cfma(t, U.u[a][1], h.h[s][1]);
      cfma(t, U.u[a][2], h.h[s][2]);
      o.h[s][a] = t;
    }
  return o;
}
// w = U^H h
template <typename R>
QMG_HD Half<R> udagmul(const Link<R>& U, const Half<R>& h) {
  Half<R> o;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a)
    {
      cpx<R> t = cmul_conj(U.u[0][a], h.h[s][0]);
      cfma_conj(t, U.u[1][a], h.h[s][1]);
      cfma_conj(t, U.u[2][a], h.h[s][2]);
      o.h[s][a] = t;
    }
  return o;
}

template <typename R, typename P>
QMG_HD Spinor<R> load_spinor(const P* f, const Geom& g, int b, int l) {
  Spinor<R> p;
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) p.s[s][c] = ldcv<R>(f, sidx(g, b, 3 * s + c, l));
  return p;
}
template <typename R, typename P>
QMG_HD void store_spinor(P* f, const Geom& g, int b, int l, const Spinor<R>& p) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) stcv(f, sidx(g, b, 3 * s + c, l), p.s[s][c]);
}
template <typename R, typename P>
QMG_HD Link<R> load_link(const P* U, const Geom& g, int b, int mu, int l) {
  Link<R> u;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int c = 0; c < 3; ++c) u.u[a][c] = ldcv<R>(U, uidx(g, b, mu, 3 * a + c, l));
  return u;
}

// out = A psi with A the two Hermitian 6x6 chirality blocks stored at (b, l)
template <typename R, typename P>
QMG_HD Spinor<R> apply_diag(const P* D, const Geom& g, int b, int l, const Spinor<R>& p) {
  Spinor<R> o;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    cpx<R> v[6], w[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) v[i] = p.s[2 * h + i / 3][i % 3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      cpx<R> d = ldcv<R>(D, didx(g, b, h, k, l));
      w[2 * k] = d.re * v[2 * k];
      w[2 * k + 1] = d.im * v[2 * k + 1];
    }
    int k = 3;
#pragma unroll
    for (int i = 1; i < 6; ++i)
#pragma unroll
      for (int j = 0; j < i; ++j) {
        cpx<R> a = ldcv<R>(D, didx(g, b, h, k, l));
        ++k;
        w[i] = w[i] + a * v[j];
        w[j] = w[j] + cmul_conj(a, v[i]);
      }
#pragma unroll
    for (int i = 0; i < 6; ++i) o.s[2 * h + i / 3][i % 3] = w[i];
  }
  return o;
}

// ------------------------------------------------------- wave reductions --
// Deterministic sum over the 64 lanes of a wave (fixed butterfly order).
QMG_HD double wave_sum(double v) {
#ifdef __HIP_DEVICE_COMPILE__
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
#endif
  return v;
}
QMG_HD float wave_sum(float v) {
#ifdef __HIP_DEVICE_COMPILE__
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
#endif
  return v;
}
