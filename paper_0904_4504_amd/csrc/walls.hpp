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

// Box with diffuse or Maxwell faces: face of a fluid cell (x, y) within R
// cells of the body, by the axis on which the cell lies outside the body's
// range: 0 below the body, 1 above, 2 left, 3 right; -1 if outside on both
// axes (its links are corner links) or out of reach.
template <int R>
__device__ __forceinline__ int box_face(const SolveDesc& d, int x, int y) {
  const bool inx = x >= d.bx0 && x < d.bx1, iny = y >= d.by0 && y < d.by1;
  if (inx && !iny) {
    if (y < d.by0) return y >= d.by0 - R ? 0 : -1;
    return y < d.by1 + R ? 1 : -1;
  }
  if (iny && !inx) {
    if (x < d.bx0) return x >= d.bx0 - R ? 2 : -1;
    return x < d.bx1 + R ? 3 : -1;
  }
  return -1;
}

// Column of a face cell (numbering of WallCol).
__device__ __forceinline__ int box_column(const SolveDesc& d, int face, int x, int y) {
  const int lx = d.bx1 - d.bx0, ly = d.by1 - d.by0;
  switch (face) {
    case 0: return x - d.bx0;
    case 1: return lx + x - d.bx0;
    case 2: return 2 * lx + y - d.by0;
    default: return 2 * lx + ly + y - d.by0;
  }
}

// Deviation from w_l rho0 of the diffuse arrival on link l of a face column
// with constants c: w_l [rho_w E_l(U) - rho0], the wall density rho_w
// returning the mass bounce-back would return through the column,
// rho_w = (rho0 (Mr + L1 U) + cm) / (Mr + Z1 U + Z2 U^2), cm the deviation
// of the column's crossing mass; written without the O(1) cancellation
// (e = E_l - 1).
__device__ __forceinline__ double ds_box_arrival(const WallCol& c, double rho0, double U,
                                                 double cm, double wl, double vx,
                                                 double theta) {
  const double uu = U * U;
  const double e = vx * U / theta + uu * (vx * vx / (2 * theta * theta) - 1 / (2 * theta));
  const double z = c.Mr + c.Z1 * U + c.Z2 * uu;
  return wl * (rho0 * (c.Mr * e + c.L1 * U * (1 + e) - c.Z1 * U - c.Z2 * uu) + cm * (1 + e)) /
         z;
}

}  // namespace lbm
