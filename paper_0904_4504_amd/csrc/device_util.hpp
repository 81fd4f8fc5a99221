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

}  // namespace lbm
