// Small device helpers shared by the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace lbm {

// Compile-time loop: f(std::integral_constant<int, I>) for I in [B, E).
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<I + 1, N>(f);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum (fx, fy) over a workgroup of BS threads in a fixed order (lanes, then
// waves) and store the pair at partials[2*slot].  Every thread must call it.
template <int BS>
__device__ __forceinline__ void block_force_partial(double fx, double fy, double* partials,
                                                    int slot) {
  __shared__ double red[2][BS / 64];
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = fx;
    red[1][wave] = fy;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sx = 0.0, sy = 0.0;
#pragma unroll
    for (int k = 0; k < BS / 64; ++k) {
      sx += red[0][k];
      sy += red[1][k];
    }
    partials[2 * slot] = sx;
    partials[2 * slot + 1] = sy;
  }
}

}  // namespace lbm
