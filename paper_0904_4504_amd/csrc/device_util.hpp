// Small device helpers shared by the kernels.
#pragma once

#include <hip/hip_ext.h>
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

// Launch kernel k; with events, through the extended launch that has the
// dispatch record them at the kernel's start and end.
template <typename K, typename E, typename... A>
inline void launch_kernel(K k, dim3 grid, dim3 block, hipStream_t stream, const E& ev,
                          A... args) {
  if (ev.start)
    hipExtLaunchKernelGGL(k, grid, block, 0, stream, ev.start, ev.stop, 0u, args...);
  else
    hipLaunchKernelGGL(k, grid, block, 0, stream, args...);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace lbm
