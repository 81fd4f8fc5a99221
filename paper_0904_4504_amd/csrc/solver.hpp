// Internal data structures shared by the kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts of 64)
constexpr int kMomTileW = 64;    // coefficient kernel: tile width (one wavefront per row)
constexpr int kMomTileH = 8;     // coefficient kernel: tile height (two rows per thread)
constexpr int kMaxSlots = 1 << 20;

enum Geom : int32_t { GEOM_PLATE = 0, GEOM_BOX = 1, GEOM_PERIODIC = 2 };
enum Far : int32_t { FAR_WALL = 0, FAR_EQ = 1 };

// Per-step drive sample: wall velocity and lock-in basis at t_n = n + 1/2.
struct Drive {
  double u;    // U_w(t_n) = u0 sin(omega t_n)
  double s;    // sin(omega t_n)
  double c;    // cos(omega t_n)
};

// Device-resident counters and accumulators of one solve.
struct SolveState {
  int64_t step;        // steps completed; selects the input buffer (parity) and drive[step]
  int32_t unstable;    // set by the step kernel when a cell has rho <= 0 or non-finite
  int32_t pad;
  double lockin[6];    // x: sum F sin, sum F cos, sum F; then the same for y
};

// Everything a kernel needs to advance one solve; lives in device memory.
// Pointers are device addresses.
struct SolveDesc {
  void* buf[2];              // populations A, B: population q of cell (x, y) at q*qs + y*ys + x
  const Drive* drive;        // [max_steps]
  double* hist;              // force ring [hist_cap][2]
  SolveState* state;
  double* partials;          // [nslots][2] per-tile force partial sums
  const int32_t* slot;       // [ntiles] tile -> partial slot, -1 if the tile has no wall link
  void* mbuf[2];             // H2 coefficients (a0, bx, by, cxx, cxy, cyy) of the state, step
                             // n reads mbuf[n & 1]; coefficient k of cell (x, y) at
                             // k*mks + y*mys + x (null when the solver keeps populations)
  const int32_t* mslot;      // [tiles_x*tiles_y] coefficient-kernel tile -> partial slot
  int64_t mks, mys;
  int32_t tiles_x, mnslots;
  int64_t qs;                // elements between the populations of one cell
  int64_t ys;                // elements between rows
  int64_t max_steps;
  int64_t hist_cap;
  int64_t lockin_first, lockin_count;
  int32_t nx, ny, ncells, pad1;    // ncells = nx * ny (row-major cell index y*nx + x)
  int32_t geom, far;
  int32_t bx0, by0, bx1, by1;      // solid cells [bx0,bx1) x [by0,by1) (box only)
  int32_t ntiles, nslots;
  int32_t cells_per_tile;
  int32_t pad0;
  double inv_tau;                  // 1/tau (0 for tau = +inf)
  double rho0;
  double ladd_scale;               // 2 rho0 / theta: moving-wall term per unit (w_i v_i.U)
  double fstatic[2];               // rest-state part of the wall force (geometry constant)
};

// One entry of the launch work list: a tile of one solve.
struct WorkItem {
  int32_t solve;
  int32_t tile;
};

// Lattice constants passed by value to the kernels.
struct KernelLattice {
  double w[8];        // weights per orbit
  double theta;
};

}  // namespace lbm
