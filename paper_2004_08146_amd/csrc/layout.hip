// Canonical <-> block-major field layout and precision conversion.
#include "qmg_ctx.h"

namespace {

template <typename S>
__global__ __launch_bounds__(256) void k_pack(Geom g, typename PT<S>::stor* out, const double2* canon) {
  int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  int k = blockIdx.y;
  int b = (int)(site >> g.bs_log), l = (int)(site & ((1 << g.bs_log) - 1));
  int64_t cs = canon_site(g, b, l);
  const double2* src = canon + ((int64_t)k * g.V + cs) * 12;
  auto* dst = out + (int64_t)k * g.V * 12;
  for (int c = 0; c < 12; ++c) {
    double2 v = src[c];
    stcv(dst, sidx(g, b, c, l), cpx<double>{v.x, v.y});
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_unpack(Geom g, double2* canon, const typename PT<S>::stor* in) {
  int64_t site = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (site >= g.V) return;
  int k = blockIdx.y;
  int b = (int)(site >> g.bs_log), l = (int)(site & ((1 << g.bs_log) - 1));
  int64_t cs = canon_site(g, b, l);
  double2* dst = canon + ((int64_t)k * g.V + cs) * 12;
  const auto* src = in + (int64_t)k * g.V * 12;
  for (int c = 0; c < 12; ++c) {
    cpx<double> v = ldcv<double>(src, sidx(g, b, c, l));
    dst[c] = make_double2(v.re, v.im);
  }
}

template <typename D, typename S>
__global__ __launch_bounds__(256) void k_convert(typename PT<D>::stor* dst, const typename PT<S>::stor* src,
                                                 int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += step) {
    if constexpr (std::is_same<D, double>::value) stcv(dst, i, ldcv<double>(src, i));
    else stcv(dst, i, ldcv<float>(src, i));
  }
}

dim3 site_grid(const Geom& g, int nrhs) { return dim3((unsigned)((g.V + 255) / 256), (unsigned)nrhs); }

}  // namespace

hipError_t launch_pack(const Geom& g, void* out, int p, const double* canon, int nrhs, hipStream_t s) {
  auto c = reinterpret_cast<const double2*>(canon);
  if (p == QMG_F64) hipLaunchKernelGGL(k_pack<double>, site_grid(g, nrhs), dim3(256), 0, s, g, (double2*)out, c);
  else if (p == QMG_F32) hipLaunchKernelGGL(k_pack<float>, site_grid(g, nrhs), dim3(256), 0, s, g, (float2*)out, c);
  else hipLaunchKernelGGL(k_pack<bf16_t>, site_grid(g, nrhs), dim3(256), 0, s, g, (uint32_t*)out, c);
  return hipGetLastError();
}

hipError_t launch_unpack(const Geom& g, double* canon, const void* in, int p, int nrhs, hipStream_t s) {
  auto c = reinterpret_cast<double2*>(canon);
  if (p == QMG_F64) hipLaunchKernelGGL(k_unpack<double>, site_grid(g, nrhs), dim3(256), 0, s, g, c, (const double2*)in);
  else if (p == QMG_F32) hipLaunchKernelGGL(k_unpack<float>, site_grid(g, nrhs), dim3(256), 0, s, g, c, (const float2*)in);
  else hipLaunchKernelGGL(k_unpack<bf16_t>, site_grid(g, nrhs), dim3(256), 0, s, g, c, (const uint32_t*)in);
  return hipGetLastError();
}

template <typename D>
static void conv_from(void* dst, const void* src, int ps, int64_t n, hipStream_t s) {
  using DS = typename PT<D>::stor;
  unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
  if (grid == 0) return;
  if (ps == QMG_F64) hipLaunchKernelGGL((k_convert<D, double>), dim3(grid), dim3(256), 0, s, (DS*)dst, (const double2*)src, n);
  else if (ps == QMG_F32) hipLaunchKernelGGL((k_convert<D, float>), dim3(grid), dim3(256), 0, s, (DS*)dst, (const float2*)src, n);
  else hipLaunchKernelGGL((k_convert<D, bf16_t>), dim3(grid), dim3(256), 0, s, (DS*)dst, (const uint32_t*)src, n);
}

hipError_t launch_convert(void* dst, int pd, const void* src, int ps, int64_t n, hipStream_t s) {
  if (pd == QMG_F64) conv_from<double>(dst, src, ps, n, s);
  else if (pd == QMG_F32) conv_from<float>(dst, src, ps, n, s);
  else conv_from<bf16_t>(dst, src, ps, n, s);
  return hipGetLastError();
}
