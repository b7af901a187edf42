// Wavefront (64-lane) and workgroup prefix-sum / reduction helpers.
#pragma once
#include <hip/hip_runtime.h>

namespace ap {

// Orders LDS traffic between the lanes of one wavefront.
__device__ __forceinline__ void __syncwarp_ap() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_incl_scan_i32(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Fixed-order butterfly sum over the 64 lanes (same order every run).
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ float wave_sum_f32(float v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Sum over a workgroup of NW wavefronts; result valid in every thread.
template <int NW>
__device__ __forceinline__ double block_sum_f64(double v, double* lds /* NW doubles */) {
  v = wave_sum_f64(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int k = 0; k < NW; ++k) t += lds[k];
  return t;
}

}  // namespace ap
