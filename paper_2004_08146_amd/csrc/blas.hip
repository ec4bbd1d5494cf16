// Vector kernels for the Krylov solvers: batched dot products (two stages,
// fixed summation order, results bitwise reproducible), batched axpy, scaling.
// A batch is nrhs vectors of n complex numbers, vector k at offset k*stride;
// a basis V_j (j < J) is at offset j*vstride.  Dot products accumulate in
// double whatever the storage precision.
#include <type_traits>

#include "qmg_ctx.h"
#include "reduce.h"

namespace {

constexpr int kDotWG = 256;
constexpr int kDotPerThread = 8;
constexpr int64_t kChunk = (int64_t)kDotWG * kDotPerThread;

// partial[(k*J + j)*nchunk + chunk] = sum over the chunk of conj(V_j,k) w_k
template <typename S>
__global__ __launch_bounds__(kDotWG) void k_dot_stage1(double* partial, const typename PT<S>::stor* V, int64_t vstride,
                                                      int J, const typename PT<S>::stor* w, int64_t n,
                                                      int64_t stride, int nchunk, int with_self,
                                                      int64_t vkstride) {
  __shared__ double red[2 * (kDotWG / 64)];
  const int chunk = blockIdx.x, k = blockIdx.y;
  const int64_t i0 = chunk * kChunk + threadIdx.x;
  const auto* wk = w + k * stride;
  cpx<double> wl[kDotPerThread];
#pragma unroll
  for (int t = 0; t < kDotPerThread; ++t) {
    const int64_t i = i0 + (int64_t)t * kDotWG;
    wl[t] = i < n ? ldcv<double>(wk, i) : czero<double>();
  }
  for (int j = 0; j < J; ++j) {
    const auto* vj = V + j * vstride + k * vkstride;
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kDotPerThread; ++t) {
      const int64_t i = i0 + (int64_t)t * kDotWG;
      if (i < n) {
        cpx<double> p = cmul_conj(ldcv<double>(vj, i), wl[t]);
        acc[0] += p.re;
        acc[1] += p.im;
      }
    }
    wg_sum<double, 2>(acc, red);
    if (threadIdx.x == 0) {
      double* o = partial + (((int64_t)k * (J + with_self) + j) * nchunk + chunk) * 2;
      o[0] = acc[0];
      o[1] = acc[1];
    }
  }
  if (with_self) {
    double acc[2] = {0.0, 0.0};
#pragma unroll
    for (int t = 0; t < kDotPerThread; ++t) acc[0] += norm2(wl[t]);
    wg_sum<double, 2>(acc, red);
    if (threadIdx.x == 0) {
      double* o = partial + (((int64_t)k * (J + 1) + J) * nchunk + chunk) * 2;
      o[0] = acc[0];
      o[1] = 0.0;
    }
  }
}

// w_k += sum_j coef[k*J+j] V_j,k over one chunk, and partial[k][chunk] = ||new w_k||^2 there.
// With a copy type C (FP32 or BF16 storage), the new w is also written to cp in
// that storage, rounded through FP32 exactly as the conversion kernel rounds it.
template <typename S, typename C = void>
__global__ __launch_bounds__(kDotWG) void k_axpy_norm(typename PT<S>::stor* w, const typename PT<S>::stor* V,
                                                     int64_t vstride, int J, const double* coef, int64_t n,
                                                     int64_t stride, int nchunk, double* partial, C* cp) {
  using R = typename PT<S>::real;
  __shared__ double red[2 * (kDotWG / 64)];
  const int chunk = blockIdx.x, k = blockIdx.y;
  const int64_t i0 = chunk * kChunk + threadIdx.x;
  auto* wk = w + k * stride;
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int t = 0; t < kDotPerThread; ++t) {
    const int64_t i = i0 + (int64_t)t * kDotWG;
    if (i < n) {
      cpx<double> v = ldcv<double>(wk, i);
      for (int j = 0; j < J; ++j) {
        const cpx<double> c = {coef[((int64_t)k * J + j) * 2], coef[((int64_t)k * J + j) * 2 + 1]};
        v = v + c * ldcv<double>(V + j * vstride + k * stride, i);
      }
      const cpx<R> vr = {R(v.re), R(v.im)};
      stcv(wk, i, vr);
      if constexpr (!std::is_void<C>::value) stcv(cp + k * stride, i, cpx<float>{float(vr.re), float(vr.im)});
      acc[0] += norm2(ldcv<double>(wk, i));
    }
  }
  wg_sum<double, 2>(acc, red);
  if (threadIdx.x == 0) {
    partial[((int64_t)k * nchunk + chunk) * 2] = acc[0];
    partial[((int64_t)k * nchunk + chunk) * 2 + 1] = 0.0;
  }
}

// dots[k*J + j] = ordered tree sum of the partials
__global__ __launch_bounds__(256) void k_dot_stage2(double* dots, const double* partial, int J, int nchunk) {
  __shared__ double red[2 * 4];
  const int j = blockIdx.x, k = blockIdx.y;
  const double* p = partial + ((int64_t)k * J + j) * nchunk * 2;
  double acc[2] = {0.0, 0.0};
  for (int c = threadIdx.x; c < nchunk; c += blockDim.x) {
    acc[0] += p[2 * c];
    acc[1] += p[2 * c + 1];
  }
  wg_sum<double, 2>(acc, red);
  if (threadIdx.x == 0) {
    dots[((int64_t)k * J + j) * 2] = acc[0];
    dots[((int64_t)k * J + j) * 2 + 1] = acc[1];
  }
}

template <typename S, typename SV = S>
__global__ __launch_bounds__(256) void k_multiaxpy(typename PT<S>::stor* w, const typename PT<SV>::stor* V,
                                                   int64_t vstride, int J, const double* coef, int64_t n,
                                                   int64_t stride) {
  using R = typename PT<S>::real;
  const int k = blockIdx.y;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  auto* wk = w + k * stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    cpx<double> acc = ldcv<double>(wk, i);
    for (int j = 0; j < J; ++j) {
      cpx<double> c = {coef[((int64_t)k * J + j) * 2], coef[((int64_t)k * J + j) * 2 + 1]};
      acc = acc + c * ldcv<double>(V + j * vstride + k * stride, i);
    }
    stcv(wk, i, cpx<R>{R(acc.re), R(acc.im)});
  }
}

// y_k = a_k x_k; with a copy type C (FP32 or BF16 storage) the result is also
// written to cp, rounded through FP32 as the conversion kernel rounds it
template <typename S, typename C = void>
__global__ __launch_bounds__(256) void k_scale(typename PT<S>::stor* y, const typename PT<S>::stor* x, const double* a,
                                               int64_t n, int64_t stride, C* cp) {
  using R = typename PT<S>::real;
  const int k = blockIdx.y;
  const cpx<double> ak = {a[2 * k], a[2 * k + 1]};
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    cpx<double> v = ak * ldcv<double>(x + k * stride, i);
    const cpx<R> vr = {R(v.re), R(v.im)};
    stcv(y + k * stride, i, vr);
    if constexpr (!std::is_void<C>::value) stcv(cp + k * stride, i, cpx<float>{float(vr.re), float(vr.im)});
  }
}

template <typename S>
__global__ __launch_bounds__(256) void k_xmy(typename PT<S>::stor* y, const typename PT<S>::stor* x, int64_t n,
                                             int64_t stride) {
  using R = typename PT<S>::real;
  const int k = blockIdx.y;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    cpx<R> v = ldcv<R>(x + k * stride, i) - ldcv<R>(y + k * stride, i);
    stcv(y + k * stride, i, v);
  }
}

// y = Gamma5 x on fine fields (spins 2, 3 change sign); n = total complex elements
template <typename S>
__global__ __launch_bounds__(256) void k_gamma5(typename PT<S>::stor* y, const typename PT<S>::stor* x, int64_t n,
                                                int bs_log) {
  using R = typename PT<S>::real;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const int comp = (int)((i >> bs_log) % 12);
    cpx<R> v = ldcv<R>(x, i);
    stcv(y, i, comp >= 6 ? -v : v);
  }
}

// plain streaming copy, 16 B per lane per step (bandwidth probe)
__global__ __launch_bounds__(256) void k_stream_copy(uint4* dst, const uint4* src, int64_t n) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) dst[i] = src[i];
}

__global__ void k_zero(uint32_t* p, int64_t n) {
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) p[i] = 0u;
}

unsigned ew_grid(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192)); }

template <typename F>
void by_prec(int p, F&& f) {
  if (p == QMG_F64) f(double{});
  else if (p == QMG_F32) f(float{});
  else f(bf16_t{});
}

}  // namespace

hipError_t launch_multidot(int p, double* dots, const void* V, int64_t vstride, int J, const void* w, int64_t n,
                           int64_t stride, int nrhs, double* partial, hipStream_t s, int with_self) {
  const int nchunk = (int)((n + kChunk - 1) / kChunk);
  by_prec(p, [&](auto tag) {
    using S = decltype(tag);
    using P = typename PT<S>::stor;
    hipLaunchKernelGGL(k_dot_stage1<S>, dim3(nchunk, nrhs), dim3(kDotWG), 0, s, partial, (const P*)V, vstride, J,
                       (const P*)w, n, stride, nchunk, with_self, stride);
  });
  hipLaunchKernelGGL(k_dot_stage2, dim3(J + with_self, nrhs), dim3(256), 0, s, dots, partial, J + with_self, nchunk);
  return hipGetLastError();
}

// dots[(k*J + j)*2] = <V_j, w_k> for nw vectors w_k (offset k*wstride) against
// one shared basis: the work-groups of all w_k read a basis chunk together
hipError_t launch_multidot_shared(int p, double* dots, const void* V, int64_t vstride, int J, const void* w,
                                  int64_t wstride, int nw, int64_t n, double* partial, hipStream_t s) {
  const int nchunk = (int)((n + kChunk - 1) / kChunk);
  by_prec(p, [&](auto tag) {
    using S = decltype(tag);
    using P = typename PT<S>::stor;
    hipLaunchKernelGGL(k_dot_stage1<S>, dim3(nchunk, nw), dim3(kDotWG), 0, s, partial, (const P*)V, vstride, J,
                       (const P*)w, n, wstride, nchunk, 0, (int64_t)0);
  });
  hipLaunchKernelGGL(k_dot_stage2, dim3(J, nw), dim3(256), 0, s, dots, partial, J, nchunk);
  return hipGetLastError();
}

// w_k += sum_j coef V_j,k; norms[2k] = ||w_k||^2 afterwards (fixed summation order)
hipError_t launch_axpy_norm(int p, void* w, const void* V, int64_t vstride, int J, const double* coef, int64_t n,
                            int64_t stride, int nrhs, double* norms, double* partial, hipStream_t s, void* copy,
                            int copy_prec) {
  const int nchunk = (int)((n + kChunk - 1) / kChunk);
  const dim3 grid(nchunk, nrhs), blk(kDotWG);
  if (copy && p == QMG_F64 && copy_prec == QMG_F32) {
    hipLaunchKernelGGL((k_axpy_norm<double, float2>), grid, blk, 0, s, (double2*)w, (const double2*)V, vstride, J,
                       coef, n, stride, nchunk, partial, (float2*)copy);
  } else if (copy && p == QMG_F64 && copy_prec == QMG_BF16) {
    hipLaunchKernelGGL((k_axpy_norm<double, uint32_t>), grid, blk, 0, s, (double2*)w, (const double2*)V, vstride, J,
                       coef, n, stride, nchunk, partial, (uint32_t*)copy);
  } else {
    if (copy) return hipErrorInvalidValue;  // only FP64 vectors are copied to FP32 / BF16
    by_prec(p, [&](auto tag) {
      using S = decltype(tag);
      using P = typename PT<S>::stor;
      hipLaunchKernelGGL((k_axpy_norm<S, void>), grid, blk, 0, s, (P*)w, (const P*)V, vstride, J, coef, n, stride,
                         nchunk, partial, (void*)nullptr);
    });
  }
  hipLaunchKernelGGL(k_dot_stage2, dim3(1, nrhs), dim3(256), 0, s, norms, partial, 1, nchunk);
  return hipGetLastError();
}

// scratch needed by launch_multidot / launch_axpy_norm: doubles
size_t multidot_partial_doubles(int64_t n, int J, int nrhs) {
  return (size_t)((n + kChunk - 1) / kChunk) * (J + 1) * nrhs * 2;
}

hipError_t launch_multiaxpy(int p, void* w, const void* V, int64_t vstride, int J, const double* coef, int64_t n,
                            int64_t stride, int nrhs, hipStream_t s) {
  by_prec(p, [&](auto tag) {
    using S = decltype(tag);
    using P = typename PT<S>::stor;
    hipLaunchKernelGGL(k_multiaxpy<S>, dim3(ew_grid(n), nrhs), dim3(256), 0, s, (P*)w, (const P*)V, vstride, J,
                       coef, n, stride);
  });
  return hipGetLastError();
}

hipError_t launch_multiaxpy_d(void* w, const void* V, int vprec, int64_t vstride, int J, const double* coef,
                              int64_t n, int64_t stride, int nrhs, hipStream_t s) {
  by_prec(vprec, [&](auto tag) {
    using SV = decltype(tag);
    using PV = typename PT<SV>::stor;
    hipLaunchKernelGGL((k_multiaxpy<double, SV>), dim3(ew_grid(n), nrhs), dim3(256), 0, s, (double2*)w, (const PV*)V,
                       vstride, J, coef, n, stride);
  });
  return hipGetLastError();
}

hipError_t launch_scale(int p, void* y, const void* x, const double* a, int64_t n, int64_t stride, int nrhs,
                        hipStream_t s, void* copy, int copy_prec) {
  const dim3 grid(ew_grid(n), nrhs), blk(256);
  if (copy && p == QMG_F64 && copy_prec == QMG_F32) {
    hipLaunchKernelGGL((k_scale<double, float2>), grid, blk, 0, s, (double2*)y, (const double2*)x, a, n, stride,
                       (float2*)copy);
  } else if (copy && p == QMG_F64 && copy_prec == QMG_BF16) {
    hipLaunchKernelGGL((k_scale<double, uint32_t>), grid, blk, 0, s, (double2*)y, (const double2*)x, a, n, stride,
                       (uint32_t*)copy);
  } else {
    if (copy) return hipErrorInvalidValue;  // only FP64 vectors are copied to FP32 / BF16
    by_prec(p, [&](auto tag) {
      using S = decltype(tag);
      using P = typename PT<S>::stor;
      hipLaunchKernelGGL((k_scale<S, void>), grid, blk, 0, s, (P*)y, (const P*)x, a, n, stride, (void*)nullptr);
    });
  }
  return hipGetLastError();
}

template <typename S>
__global__ __launch_bounds__(256) void k_add(typename PT<S>::stor* y, const typename PT<S>::stor* x, int64_t n,
                                             int64_t stride) {
  using R = typename PT<S>::real;
  const int k = blockIdx.y;
  const int64_t step = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += step) {
    const cpx<R> v = ldcv<R>(y + k * stride, i) + ldcv<R>(x + k * stride, i);
    stcv(y + k * stride, i, v);
  }
}

hipError_t launch_add(int p, void* y, const void* x, int64_t n, int64_t stride, int nrhs, hipStream_t s) {
  by_prec(p, [&](auto tag) {
    using S = decltype(tag);
    using P = typename PT<S>::stor;
    hipLaunchKernelGGL(k_add<S>, dim3(ew_grid(n), nrhs), dim3(256), 0, s, (P*)y, (const P*)x, n, stride);
  });
  return hipGetLastError();
}

hipError_t launch_xmy(int p, void* y, const void* x, int64_t n, int64_t stride, int nrhs, hipStream_t s) {
  by_prec(p, [&](auto tag) {
    using S = decltype(tag);
    using P = typename PT<S>::stor;
    hipLaunchKernelGGL(k_xmy<S>, dim3(ew_grid(n), nrhs), dim3(256), 0, s, (P*)y, (const P*)x, n, stride);
  });
  return hipGetLastError();
}

hipError_t launch_gamma5_bs(int p, void* y, const void* x, int64_t n, int bs_log, hipStream_t s) {
  by_prec(p, [&](auto tag) {
    using S = decltype(tag);
    using P = typename PT<S>::stor;
    hipLaunchKernelGGL(k_gamma5<S>, dim3(ew_grid(n)), dim3(256), 0, s, (P*)y, (const P*)x, n, bs_log);
  });
  return hipGetLastError();
}

hipError_t launch_stream_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 16);
  // 4 work-groups per CU of 256 threads: enough loads in flight to saturate HBM
  // with each lane streaming a long contiguous range of 16-B chunks
  if (n > 0) hipLaunchKernelGGL(k_stream_copy, dim3(1024), dim3(256), 0, s, (uint4*)dst, (const uint4*)src, n);
  return hipGetLastError();
}

hipError_t launch_fill_zero(void* y, size_t bytes, hipStream_t s) {
  const int64_t n = (int64_t)(bytes / 4);
  if (n > 0) hipLaunchKernelGGL(k_zero, dim3(ew_grid(n)), dim3(256), 0, s, (uint32_t*)y, n);
  return hipGetLastError();
}
