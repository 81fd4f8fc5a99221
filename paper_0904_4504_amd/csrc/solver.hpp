// Internal data structures shared by the kernels and the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

// Events a kernel launch records itself at its start and end (the dispatch
// timestamps, as a profiler's trace sees them); null: none.
struct KernelEvents {
  hipEvent_t start = nullptr, stop = nullptr;
};

constexpr int kBlock = 256;      // threads per workgroup (4 wavefronts of 64)
constexpr int kCoefTileW = 64;   // coefficient kernel: tile width (one column per lane)
constexpr int kCoefKMax = 3;     // coefficient kernel: tile variants K = 1..3
constexpr int kCoefKDefault = 3;

// Rows of a coefficient-kernel tile of variant K: four wavefronts of K rows
// each (K cells per thread).
constexpr int kCoefWaves = 4;    // coefficient kernel: wavefronts per workgroup
__host__ __device__ constexpr int coef_tile_rows(int K) { return kCoefWaves * K; }
constexpr int kMaxSlots = 1 << 20;

enum Geom : int32_t { GEOM_PLATE = 0, GEOM_BOX = 1, GEOM_PERIODIC = 2 };
enum Far : int32_t { FAR_WALL = 0, FAR_EQ = 1 };
enum Wall : int32_t { WALL_BB = 0, WALL_DS = 1 };

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

// Momentum exchange of the wall force, precomputed per solve on the host.
// Population state: F += (wx, wy) * buf[off] for every wall link (off = the
// population at the mirror cell that crosses the wall), and M += wm * buf[off]
// (the crossing mass, diffuse wall only), the weights those of the link's
// pattern (they depend on its direction only, so a solve has at most Q).
struct ForceLink {
  int64_t off;
  int32_t pat, pad;
};
struct LinkWeights {
  double wx, wy, wm, pad;
};
// Coefficient state: F += (wx . c, wy . c) and M += wm . c per mirror cell,
// c_k = mbuf[k*mks + off] (the cell's links folded into 6-vectors; cells with
// the same set of links share one pattern of weights).
struct ForceCell {
  int64_t off;
  int32_t pat, pad;
};
struct CellWeights {
  double wx[6], wy[6], wm[6];
};

// Box with diffuse or Maxwell faces.  A link (arrival cell, direction whose
// source lies in the body) belongs to the face on whose axis its arrival cell
// lies outside the body's range; faces are cut into columns (one per arrival
// coordinate along the face: faces below, above the body by x, left, right of
// it by y; numbered in that order).  Per column, over its links l: Mr = sum
// w_l, Z1 = sum w_l vx_l / theta, Z2 = sum w_l (vx_l^2 / 2 theta^2 -
// 1 / 2 theta) (the mass emitted per unit wall density is Mr + Z1 U + Z2 U^2),
// L1 = sum 2 w_l vx_l / theta (the moving-wall terms bounce-back would add,
// per unit rho0 U); the column's links are [first, first + count) of the link
// table.  For a solve kept as H2 coefficients: cell[k] is the coefficient
// offset (y pitch + x) of the column's cell k + 1 cells from the face, and
// the column's crossing mass is sum_k sum_j mc[k][j] c_j(cell[k]) (every
// partner population df_{-v}(x_p) = w (a0 - vx bx - vy by + vx^2 cxx +
// vx vy cxy + vy^2 cyy) is linear in the coefficients of its cell).
struct WallCol {
  double Mr, Z1, Z2, L1;
  int32_t first, count;
  int64_t cell[3];
  double mc[3][6];
};
// One link of such a box: its bounce-back partner (the opposite population at
// the mirror cell) and, on a face, its specular source (the population of
// the velocity mirrored in the face's normal, at the source point mirrored
// through the face plane), as element offsets into a population buffer
// (off_*) and as the cells' coefficient offsets (cell_*); its column (-1: a
// corner link, which keeps bounce-back); normal: the face is normal to the
// motion (x faces); the arrival direction's weight and velocity.
struct WallLink {
  int64_t off_partner, off_spec;
  int64_t cell_partner, cell_spec;
  int32_t col, normal;
  double w, vx, vy;
};
// Most face columns a diffuse or Maxwell box may have (2 (box_lx + box_ly)).
constexpr int kMaxWallCols = 1024;

// Everything a kernel needs to advance one solve; lives in device memory.
// Pointers are device addresses.
struct SolveDesc {
  void* buf[2];              // populations A, B: population q of cell (x, y) at q*qs + y*ys + x
  const Drive* drive;        // [max_steps]
  double* hist;              // force ring [hist_cap][2]
  SolveState* state;
  const ForceLink* links;    // [nlinks]
  const ForceCell* fcells;   // [nfcells] (coefficient state only)
  const LinkWeights* lweights;  // weight patterns of the links
  const CellWeights* cweights;  // weight patterns of the cells
  void* mbuf[2];             // H2 coefficients (a0, bx, by, cxx, cxy, cyy) of the state, step
                             // n reads mbuf[n & 1]; coefficient k of cell (x, y) at
                             // k*mks + y*mys + x (null when the solver keeps populations)
  int64_t mks, mys;
  int32_t tiles_x, pad2;          // coefficient kernel: tiles per row of tiles
  int64_t qs;                // elements between the populations of one cell
  int64_t ys;                // elements between rows
  int64_t max_steps;
  int64_t hist_cap;
  int64_t lockin_first, lockin_count;
  int32_t nx, ny, ncells, pad1;    // ncells = nx * ny (row-major cell index y*nx + x)
  int32_t geom, far;
  int32_t bx0, by0, bx1, by1;      // solid cells [bx0,bx1) x [by0,by1) (box only)
  int32_t nlinks, nfcells;
  double inv_tau;                  // 1/tau (0 for tau = +inf)
  double rho0;
  double ladd_scale;               // 2 rho0 / theta: moving-wall term per unit (w_i v_i.U)
  double fstatic[2];               // rest-state part of the wall force (geometry constant)
  double kladd[2];                 // force of the moving-wall terms per unit U_w
  int32_t wall, pad3;              // WALL_BB or WALL_DS (diffuse share sigma, rest specular)
  double sigma;                    // accommodation: 1 diffuse .. 0 specular
  // diffuse wall: A1 = sum_{vy>0} vy w, A2 = sum_{vy>0} vy w (vx^2/2th^2 - 1/2th),
  // Bx = sum_{vy>0} vy vx^2 w / th, By0 = sum_{vy>0} vy^2 w,
  // By2 = sum_{vy>0} vy^2 w (vx^2/2th^2 - 1/2th), nx rho0
  double ds[6];
  // box with diffuse or Maxwell faces (null otherwise)
  const WallCol* wcols;      // [nwcols]
  const WallLink* wlinks;    // [nwlinks]
  int32_t nwcols, nwlinks;
  double theta;              // lattice theta (the finalize's diffuse emission)
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
