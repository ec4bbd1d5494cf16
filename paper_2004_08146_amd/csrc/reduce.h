// Work-group reductions with a fixed summation order.
#pragma once
#include "qmg_device.h"

// sum of NV values over the work-group (power-of-two size), same result in
// every thread.  red: LDS scratch of at least NV * max(blockDim.x/64, blockDim.x) (for
// blockDim.x < 64) elements.  Ends with a barrier so red can be reused.
template <typename R, int NV>
__device__ __forceinline__ void wg_sum(R (&v)[NV], R* red) {
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
