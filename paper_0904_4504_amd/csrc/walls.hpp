// Diffuse-scattering wall (Sec. 4, eq. DS) of the plate, shared by the
// population and the coefficient kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "solver.hpp"

namespace lbm {

// Deviation from w_q rho0 of the population of direction q (v_qy > 0) that
// the moving wall emits into column x: w_q [rho_w(x) E_q(U) - rho0], with
// E_q(U) = 1 + vx U/th + (vx U)^2/2th^2 - U^2/2th the H2 equilibrium factor
// at the wall velocity (eq. feq_h2) and rho_w(x) = (rho0 A1 + cm)/emit(U) the
// wall density of zero normal mass flux: cm is the deviation of the mass of
// the populations of column x that cross the wall, emit(U) = A1 + U^2 A2 the
// mass the wall emits per unit density.  Written without the O(1)
// cancellation: rho_w E - rho0 = rho0 (A1 e - U^2 A2)/emit + cm (1 + e)/emit,
// e = E - 1.
template <int vx>
__device__ __forceinline__ double ds_arrival(const SolveDesc& d, double U, double cm, double wq,
                                             double theta) {
  const double uu = U * U;
  const double e = vx * U / theta + uu * (vx * vx / (2 * theta * theta) - 1 / (2 * theta));
  const double emit = d.ds[0] + uu * d.ds[1];
  return wq * (d.rho0 * (d.ds[0] * e - uu * d.ds[1]) + cm * (1 + e)) / emit;
}

}  // namespace lbm
