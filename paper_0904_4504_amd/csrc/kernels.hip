// Lattice-BGK hot path for gfx950: fused pull-stream + regularized collision
// with moving-wall bounce-back and FP64 momentum-exchange force, and the
// per-step force finalisation with lock-in accumulation.
//
// Method (Sec. 5): advection f_i^adv(x) = f_i(x - v_i) (eq. advection);
// moments rho, rho u, Pi of f^adv (eq. MME_lbgk); H2 equilibrium (eq.
// feq_h2); regularized non-equilibrium part (eq. fne) relaxed by (1 - 1/tau)
// (eq. regularization).  Bounce-back (Sec. 4, eq. BB) in its linearised
// half-way lattice form with the moving-wall term 2 w_i rho0 (v_i.U_w)/theta;
// wall drive U_w = U0 sin(omega t) along x (Sec. 6).  The force on the body is
// the momentum exchanged by the bounced populations; its dissipative and
// inertial parts (Sec. 2, F_f = -m(gamma x_t + beta x_tt)) come from the
// lock-in sums.
//
// Storage: deviations delta f_i = f_i - w_i rho0 in FP64 or FP32, structure
// of arrays: population q of cell (x, y) at q*qs + y*ys + x.  Wide lattices
// interleave the Q rows of each lattice row (qs = row pitch, ys = Q*pitch), so
// the Q streams of a workgroup stay within a few hundred KB; narrow lattices
// use whole-lattice planes (qs = plane, ys = nx).  Written in
// deviation form the regularized collision needs only six sums of the pulled
// populations (delta rho, j, P = sum delta f v v); its output is
//   delta f_i^post = w_i [ a0 + v_i . b + c_xx vx^2 + c_xy vx vy + c_yy vy^2 ]
// with B = A' - omega_r (A' - j j / rho), A' = P - delta rho theta I,
//   a0 = delta rho - tr(B)/(2 theta), b = j/theta, c_xx = B_xx/(2 theta^2),
//   c_xy = B_xy/theta^2, c_yy = B_yy/(2 theta^2),
// which equals f^eq + (1 - 1/tau) fne of the paper minus w_i rho0 (the H2
// equilibrium and the projected non-equilibrium part expand in the same
// Hermite basis).  omega_r = 1/tau is kept separate from 1 - 1/tau so that
// large tau loses no precision in FP32.
#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "device_util.hpp"
#include "lattice.hpp"
#include "solver.hpp"
#include "walls.hpp"

namespace lbm {

// Pull of population q into fluid cell (x, y) when the cell lies within R
// cells of the domain edge or of the body: periodic wrap, bounce-back at the
// moving wall / body (with the moving-wall term), stationary far wall or
// rest-equilibrium far field (delta f = 0).  The wall force is computed from
// the same input state by the finalize kernel.  DSW: the plate's moving wall
// may be diffuse (else it is bounce-back).
template <class L, typename S, bool DSW, int q>
__device__ __forceinline__ S pull_edge(const SolveDesc& d, const S* __restrict__ fin, int x,
                                       int y, double ladd, double wq, double U, double cm,
                                       double theta, int face, int col) {
  constexpr int vx = L::vx[q], vy = L::vy[q];
  constexpr int o = opposite<L>(q);
  const int nx = d.nx, ny = d.ny;
  const int64_t qs = d.qs, ys = d.ys;
  int sx = x - vx, sy = y - vy;
  if (d.geom == GEOM_PERIODIC) {
    sx += sx < 0 ? nx : 0;
    sx -= sx >= nx ? nx : 0;
    sy += sy < 0 ? ny : 0;
    sy -= sy >= ny ? ny : 0;
    return fin[q * qs + sy * ys + sx];
  }
  if (d.geom == GEOM_PLATE) {
    sx += sx < 0 ? nx : 0;
    sx -= sx >= nx ? nx : 0;
    if constexpr (vy > 0) {
      if (sy < 0) {
        // from the moving wall at y = -1/2: diffuse emission (a share sigma;
        // the rest the specular image, the population of (vx, -vy) from
        // column x - vx at the mirror row), or bounce-back (retrace in y,
        // keep x)
        const int py = -1 - sy;
        if (DSW && d.wall == WALL_DS) {
          const double e = ds_arrival<vx>(d, U, cm, wq, theta);
          if (d.sigma == 1.0) return (S)e;
          constexpr int qr = reflect_y<L>(q);
          return (S)(d.sigma * e + (1.0 - d.sigma) * (double)fin[qr * qs + py * ys + sx]);
        }
        return fin[o * qs + py * ys + x] + (S)(wq * vx * ladd);
      }
    }
    if constexpr (vy < 0) {
      if (sy >= ny) {
        if (d.far == FAR_EQ) return S(0);
        const int py = 2 * ny - 1 - sy;  // stationary wall at y = ny - 1/2
        return fin[o * qs + py * ys + x];
      }
    }
    return fin[q * qs + sy * ys + sx];
  }
  // box in a rest-equilibrium far field
  if (sx < 0 || sx >= nx || sy < 0 || sy >= ny) return S(0);
  if (sx >= d.bx0 && sx < d.bx1 && sy >= d.by0 && sy < d.by1) {
    // per axis: mirror the source through the face plane when the arrival
    // lies outside the body's range on that axis, else keep the arrival
    int px = x, py = y;
    if (x < d.bx0) px = 2 * d.bx0 - 1 - sx;
    else if (x >= d.bx1) px = 2 * d.bx1 - 1 - sx;
    if (y < d.by0) py = 2 * d.by0 - 1 - sy;
    else if (y >= d.by1) py = 2 * d.by1 - 1 - sy;
    if (DSW && d.wall == WALL_DS && face >= 0) {
      // a face link of a diffuse box: the column's diffuse emission (a share
      // sigma; the rest the specular image -- the population of the velocity
      // mirrored in the face's normal at the source mirrored through the face
      // plane, with the moving-wall term on the faces normal to the motion)
      double e = ds_box_arrival(d.wcols[col], d.rho0, U, cm, wq, (double)vx, theta);
      if (d.sigma != 1.0) {
        double sp;
        if (face <= 1) {
          constexpr int qr = reflect_y<L>(q);
          sp = (double)fin[qr * qs + py * ys + sx];
        } else {
          constexpr int qr = reflect_x<L>(q);
          sp = (double)fin[qr * qs + sy * ys + px] + wq * vx * ladd;
        }
        e = d.sigma * e + (1.0 - d.sigma) * sp;
      }
      return (S)e;
    }
    return fin[o * qs + py * ys + px] + (S)(wq * vx * ladd);
  }
  return fin[q * qs + sy * ys + sx];
}

// Geometry of a solve for the boundary path, read once per cell (so that the
// per-population selects below work on registers).
struct EdgeGeom {
  int nx, ny, bx0, bx1, by0, by1;
  bool far_eq;
  int64_t qs, ys;
};

__device__ __forceinline__ EdgeGeom edge_geom(const SolveDesc& d) {
  return EdgeGeom{d.nx, d.ny, d.bx0, d.bx1, d.by0, d.by1, d.far == FAR_EQ, d.qs, d.ys};
}

// Boundary path of a box-geometry wavefront away from the body: only the
// domain edges (the rest-equilibrium far field) are in reach.
constexpr int kBoxOpen = 3;

// A zero of either storage precision, read by arrivals from the far field.
__device__ const double kZeroWord = 0.0;

// Moments (delta rho, jx, jy, Pxx, Pxy, Pyy) of the moving-wall terms of a
// cell's bounce-back arrivals.
template <typename S>
struct WallMom {
  S v[6];
};

// The pull of pull_edge with bounce-back walls only (no diffuse wall), for
// geometry G, without branches per lane: the source plane, row and column
// are selected and an arrival of zero (the far field) reads kZeroWord, so a
// wavefront issues its Q loads back to back.  The moving-wall term of an
// arrival, 2 w_i rho0 (v_i.U_w)/theta, is returned in `term` (-0 where there
// is none, so that adding it changes nothing).
template <class L, typename S, int G, int q>
__device__ __forceinline__ S pull_edge_bb(const EdgeGeom& g, const S* __restrict__ fin, int x,
                                          int y, int64_t idx, double ladd, double wq, S& term) {
  constexpr int vx = L::vx[q], vy = L::vy[q];
  constexpr int o = opposite<L>(q);
  const int sx = x - vx, sy = y - vy;
  if constexpr (G == kBoxOpen) {
    const bool zero = sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny;
    term = S(-0.0);
    const S* src = zero ? reinterpret_cast<const S*>(&kZeroWord)
                        : fin + (q * g.qs + idx - (vy * g.ys + vx));
    return *src;
  }
  int pl = q, px = sx, py = sy;
  bool zero = false, moving = false;
  if constexpr (G == GEOM_BOX) {
    // outside the domain: rest-equilibrium far field; inside the body: the
    // mirror cell of the link (per axis, through the face plane when the
    // arrival lies outside the body's range on that axis)
    zero = sx < 0 || sx >= g.nx || sy < 0 || sy >= g.ny;
    moving = sx >= g.bx0 && sx < g.bx1 && sy >= g.by0 && sy < g.by1;
    const int mx = x < g.bx0 ? 2 * g.bx0 - 1 - sx : (x >= g.bx1 ? 2 * g.bx1 - 1 - sx : x);
    const int my = y < g.by0 ? 2 * g.by0 - 1 - sy : (y >= g.by1 ? 2 * g.by1 - 1 - sy : y);
    pl = moving ? o : pl;
    px = moving ? mx : px;
    py = moving ? my : py;
  } else {
    px += px < 0 ? g.nx : 0;
    px -= px >= g.nx ? g.nx : 0;
    if constexpr (G == GEOM_PERIODIC) {
      py += py < 0 ? g.ny : 0;
      py -= py >= g.ny ? g.ny : 0;
    } else {
      if constexpr (vy > 0) {
        // moving wall at y = -1/2: retrace in y, keep x
        moving = sy < 0;
        pl = moving ? o : pl;
        px = moving ? x : px;
        py = moving ? -1 - sy : py;
      }
      if constexpr (vy < 0) {
        // stationary wall at y = ny - 1/2, or the rest-equilibrium far field
        const bool far = sy >= g.ny;
        zero = far && g.far_eq;
        pl = far ? o : pl;
        px = far ? x : px;
        py = far ? 2 * g.ny - 1 - sy : py;
      }
    }
  }
  term = moving ? (S)(wq * vx * ladd) : S(-0.0);
  const S* src =
      zero ? reinterpret_cast<const S*>(&kZeroWord) : fin + (pl * g.qs + py * g.ys + px);
  return *src;
}

// All Q pulls of a cell through pull_edge_bb for geometry G.  Plain BGK needs
// every arrival itself (population plus wall term); the regularized
// collision only their moments, so the wall terms go to `wall` instead.
template <class L, typename S, bool BGK, int G>
__device__ __forceinline__ void pull_cell_bb(S (&f)[L::Q], WallMom<S>& wall, const EdgeGeom& g,
                                             const S* __restrict__ fin, int x, int y, int64_t idx,
                                             double ladd, const KernelLattice& lat) {
  static_for<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int vx = L::vx[q], vy = L::vy[q];
    S term;
    f[q] = pull_edge_bb<L, S, G, q>(g, fin, x, y, idx, ladd, lat.w[L::orbit[q]], term);
    if constexpr (BGK) {
      f[q] += term;
    } else if constexpr (G == GEOM_BOX || (G == GEOM_PLATE && vy > 0)) {
      wall.v[0] += term;
      if constexpr (vx != 0) wall.v[1] += S(vx) * term;
      if constexpr (vy != 0) wall.v[2] += S(vy) * term;
      if constexpr (vx != 0) wall.v[3] += S(vx * vx) * term;
      if constexpr (vx * vy != 0) wall.v[4] += S(vx * vy) * term;
      if constexpr (vy != 0) wall.v[5] += S(vy * vy) * term;
    }
  });
}

// Deviation of the mass crossing the face column of fluid cell (x, y) of a
// diffuse box in this step: the populations of the column (the cells on the
// fluid side of the face in the cell's row or column, within R of it) whose
// straight destination lies in the body -- the bounce-back partners of the
// column's links.
template <class L, typename S>
__device__ __forceinline__ double box_cross_mass(const SolveDesc& d, const S* __restrict__ fin,
                                                 int face, int x, int y) {
  constexpr int R = L::R;
  const int64_t qs = d.qs, ys = d.ys;
  double cm = 0.0;
  static_for<0, L::Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int vx = L::vx[q], vy = L::vy[q];
    for (int k = 1; k <= R; ++k) {
      // the column's cell k away from the face, and where its population goes
      int cx = x, cy = y;
      bool into = false;
      if (face == 0) {
        cy = d.by0 - k;
        into = vy >= k && x + vx >= d.bx0 && x + vx < d.bx1;
      } else if (face == 1) {
        cy = d.by1 - 1 + k;
        into = -vy >= k && x + vx >= d.bx0 && x + vx < d.bx1;
      } else if (face == 2) {
        cx = d.bx0 - k;
        into = vx >= k && y + vy >= d.by0 && y + vy < d.by1;
      } else {
        cx = d.bx1 - 1 + k;
        into = -vx >= k && y + vy >= d.by0 && y + vy < d.by1;
      }
      if (into) cm += (double)fin[q * qs + cy * ys + cx];
    }
  });
  return cm;
}

// Update of one cell: pull, moments, collision, store.  OUTM stores the six H2 coefficients of the
// post-collision state (a0, bx, by, cxx, cxy, cyy) to the coefficient planes
// instead of the Q populations (regularized collision only; used for the first
// step after populations were loaded into a solver kept in coefficients).
template <class L, typename S, bool BGK, bool DSW, bool OUTM>
__device__ __forceinline__ void update_cell(const SolveDesc& d, const S* __restrict__ fin,
                                            S* __restrict__ fout, int64_t n, int c,
                                            const KernelLattice& lat) {
  constexpr int Q = L::Q, R = L::R;
  const int nx = d.nx, ny = d.ny;
  const int64_t qs = d.qs, ys = d.ys;
  const bool active = c < d.ncells;
  const int y = active ? c / nx : 0;
  const int x = active ? c - y * nx : 0;
  const bool is_box = d.geom == GEOM_BOX;
  const bool solid = is_box && x >= d.bx0 && x < d.bx1 && y >= d.by0 && y < d.by1;
  bool interior = x >= R && x < nx - R && y >= R && y < ny - R;
  if (is_box) interior = interior && !(x >= d.bx0 - R && x < d.bx1 + R && y >= d.by0 - R &&
                                       y < d.by1 + R);
  const bool fluid = active && !solid;
  const int64_t idx = y * ys + x;
  // With bounce-back walls a wavefront that has a cell near an edge or the
  // body pulls every cell through the boundary path (which also covers
  // interior cells): one pass of loads, no divergence.
  bool edge = fluid && !interior;
  if constexpr (!DSW) edge = __any(edge);

  S f[Q];
  WallMom<S> wall{{S(0), S(0), S(0), S(0), S(0), S(0)}};
  if (fluid && !edge) {
    static_for<0, Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      f[q] = fin[q * qs + idx - (L::vy[q] * ys + L::vx[q])];
    });
  } else if (fluid) {
    const double U = d.drive[n].u;
    const double ladd = d.ladd_scale * U;
    // diffuse wall: deviation of the mass crossing the wall in column x
    double cm = 0.0;
    int face = -1, col = 0;
    if (DSW && d.wall == WALL_DS && d.geom == GEOM_PLATE && y < R)
      static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        if constexpr (L::vy[q] < 0)
          for (int r = 0; r < -L::vy[q]; ++r) cm += (double)fin[q * qs + r * ys + x];
      });
    if (DSW && d.wall == WALL_DS && d.geom == GEOM_BOX) {
      face = box_face<R>(d, x, y);
      if (face >= 0) {
        col = box_column(d, face, x, y);
        cm = box_cross_mass<L, S>(d, fin, face, x, y);
      }
    }
    if constexpr (DSW) {
      static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        f[q] = pull_edge<L, S, DSW, q>(d, fin, x, y, ladd, lat.w[L::orbit[q]], U, cm, lat.theta,
                                       face, col);
      });
    } else {
      const EdgeGeom g = edge_geom(d);
      if (d.geom == GEOM_BOX) {
        if (__any(x >= g.bx0 - R && x < g.bx1 + R && y >= g.by0 - R && y < g.by1 + R))
          pull_cell_bb<L, S, BGK, GEOM_BOX>(f, wall, g, fin, x, y, idx, ladd, lat);
        else
          pull_cell_bb<L, S, BGK, kBoxOpen>(f, wall, g, fin, x, y, idx, ladd, lat);
      } else if (d.geom == GEOM_PERIODIC) {
        pull_cell_bb<L, S, BGK, GEOM_PERIODIC>(f, wall, g, fin, x, y, idx, ladd, lat);
      } else {
        pull_cell_bb<L, S, BGK, GEOM_PLATE>(f, wall, g, fin, x, y, idx, ladd, lat);
      }
    }
  } else {
    static_for<0, Q>([&](auto qc) { f[decltype(qc)::value] = S(0); });
  }

  // moments of the pulled deviations
  S drho = 0, jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0;
  static_for<0, Q>([&](auto qc) {
    constexpr int q = decltype(qc)::value;
    constexpr int vx = L::vx[q], vy = L::vy[q];
    const S v = f[q];
    drho += v;
    if constexpr (vx != 0) jx += S(vx) * v;
    if constexpr (vy != 0) jy += S(vy) * v;
    if constexpr (vx != 0) pxx += S(vx * vx) * v;
    if constexpr (vx * vy != 0) pxy += S(vx * vy) * v;
    if constexpr (vy != 0) pyy += S(vy * vy) * v;
  });
  if constexpr (!BGK && !DSW) {
    drho += wall.v[0];
    jx += wall.v[1];
    jy += wall.v[2];
    pxx += wall.v[3];
    pxy += wall.v[4];
    pyy += wall.v[5];
  }

  const S th = (S)lat.theta;
  const S inv_th = (S)(1.0 / lat.theta);
  const S h2 = (S)(0.5 / (lat.theta * lat.theta));
  const S om = (S)d.inv_tau;
  const S rho = (S)d.rho0 + drho;
  const S inv_rho = S(1) / rho;
  const S uxx = jx * jx * inv_rho, uxy = jx * jy * inv_rho, uyy = jy * jy * inv_rho;

  if (fluid && !(rho > S(0) && rho < S(INFINITY))) d.state->unstable = 1;

  if constexpr (!BGK) {
    const S axx = pxx - drho * th, ayy = pyy - drho * th, axy = pxy;
    const S bxx = axx - om * (axx - uxx);
    const S bxy = axy - om * (axy - uxy);
    const S byy = ayy - om * (ayy - uyy);
    const S a0 = drho - (bxx + byy) * (S(0.5) * inv_th);
    const S bx = jx * inv_th, by = jy * inv_th;
    const S cxx = bxx * h2, cxy = bxy * (S(2) * h2), cyy = byy * h2;
    if constexpr (OUTM) {
      if (fluid) {
        const int64_t g = y * d.mys + x;
        fout[g] = a0;
        fout[d.mks + g] = bx;
        fout[2 * d.mks + g] = by;
        fout[3 * d.mks + g] = cxx;
        fout[4 * d.mks + g] = cxy;
        fout[5 * d.mks + g] = cyy;
      }
    } else if (fluid) {
      static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int vx = L::vx[q], vy = L::vy[q];
        S p = a0;
        if constexpr (vx != 0) p += S(vx) * bx + S(vx * vx) * cxx;
        if constexpr (vy != 0) p += S(vy) * by + S(vy * vy) * cyy;
        if constexpr (vx * vy != 0) p += S(vx * vy) * cxy;
        // output is not re-read in this step: stream it past the caches
        __builtin_nontemporal_store((S)lat.w[L::orbit[q]] * p, &fout[q * qs + idx]);
      });
    }
  } else {
    // plain BGK: delta f^post = delta f + omega_r (delta f^eq - delta f)
    const S a0 = drho - (uxx + uyy) * (S(0.5) * inv_th);
    const S bx = jx * inv_th, by = jy * inv_th;
    const S cxx = uxx * h2, cxy = uxy * (S(2) * h2), cyy = uyy * h2;
    if (fluid) static_for<0, Q>([&](auto qc) {
      constexpr int q = decltype(qc)::value;
      constexpr int vx = L::vx[q], vy = L::vy[q];
      S p = a0;
      if constexpr (vx != 0) p += S(vx) * bx + S(vx * vx) * cxx;
      if constexpr (vy != 0) p += S(vy) * by + S(vy * vy) * cyy;
      if constexpr (vx * vy != 0) p += S(vx * vy) * cxy;
      const S feq = (S)lat.w[L::orbit[q]] * p;
      __builtin_nontemporal_store(f[q] + om * (feq - f[q]), &fout[q * qs + idx]);
    });
  }
}

// One workgroup of BS threads per tile of BS consecutive cells (row-major),
// one cell per thread.  The diffuse wall is a separate instantiation (DSW), so
// that the bounce-back kernel carries none of its code and registers.
template <class L, typename S, bool BGK, bool DSW, int BS, bool OUTM>
__global__ __launch_bounds__(BS) void step_kernel(const SolveDesc* __restrict__ descs,
                                                  const WorkItem* __restrict__ work,
                                                  KernelLattice lat) {
  // The host orders the work list so that workgroup b runs on XCD b % 8 with
  // whole lattice rows per XCD (see order_tiles); padding items are no-ops.
  const WorkItem wi = work[blockIdx.x];
  if (wi.tile < 0) return;
  const SolveDesc& d = descs[wi.solve];
  const int64_t n = d.state->step;
  const S* __restrict__ fin = static_cast<const S*>(d.buf[n & 1]);
  S* __restrict__ fout = static_cast<S*>(OUTM ? d.mbuf[(n & 1) ^ 1] : d.buf[(n & 1) ^ 1]);
  update_cell<L, S, BGK, DSW, OUTM>(d, fin, fout, n, wi.tile * BS + (int)threadIdx.x, lat);
}

// One workgroup per solve.  Wall force of step n by momentum exchange (Sec.
// 2 force F_f; eq. BB): every bounce-back link carries -v_i (f_opp(x_p) +
// f_i^adv(x)) = -v_i (2 f_opp(x_p) + 2 w_i rho0 (v_i.U_w)/theta) (+ the rest
// state), so F_n = F_static + K_ladd U_w(n) + sum over links of the reflected
// populations of step n's input state, read here from the step's input buffer
// (untouched by the step) and summed in a fixed order in FP64.  At a diffuse
// wall (eq. DS) f_i^adv is the wall's emission, which depends on the same
// input state only through the crossing mass of each column.  Then append
// F_n to the history ring, accumulate the lock-in sums when n lies in the
// window, and advance the step counter.
// mode 0: the step read populations; 1: coefficients; 2: per solve,
// coefficients if the solve keeps them (batches).
template <typename S>
__device__ void finalize_solve(const SolveDesc& d, int mode) {
  SolveState* st = d.state;
  const int64_t n = st->step;
  const bool coeffs = mode == 1 || (mode == 2 && d.mbuf[0] != nullptr);
  // the epilogue's loads (drive entry, lock-in sums), issued before the
  // force sums so that their latency overlaps them
  const bool in_window = n >= d.lockin_first && n < d.lockin_first + d.lockin_count;
  Drive dr{};
  double lk[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (threadIdx.x == 0) {
    dr = d.drive[n];
    if (in_window)
      for (int k = 0; k < 6; ++k) lk[k] = st->lockin[k];
  }
  double fx = 0.0, fy = 0.0, fm = 0.0;
  if (!coeffs && d.nwlinks > 0) {
    // box with diffuse or Maxwell faces: every link's arrival as the step
    // kernel formed it -- the column's diffuse emission from the column's
    // crossing mass (first pass), mixed with the specular image; corner links
    // bounce back -- and the momentum exchange -v_l (f_partner + f_arrival)
    const S* __restrict__ f = static_cast<const S*>(n & 1 ? d.buf[1] : d.buf[0]);
    __shared__ double cmass[kMaxWallCols];
    for (int c = threadIdx.x; c < d.nwcols; c += kBlock) {
      const WallCol col = d.wcols[c];
      double m = 0.0;
      for (int k = 0; k < col.count; ++k) m += (double)f[d.wlinks[col.first + k].off_partner];
      cmass[c] = m;
    }
    __syncthreads();
    const double U = d.drive[n].u;
    const double ladd = d.ladd_scale * U;
    for (int i = threadIdx.x; i < d.nwlinks; i += kBlock) {
      const WallLink l = d.wlinks[i];
      const double fp = (double)f[l.off_partner];
      double a;
      if (l.col < 0) {
        a = fp + l.w * l.vx * ladd;
      } else {
        a = ds_box_arrival(d.wcols[l.col], d.rho0, U, cmass[l.col], l.w, l.vx, d.theta);
        if (d.sigma != 1.0) {
          const double sp = (double)f[l.off_spec] + (l.normal ? l.w * l.vx * ladd : 0.0);
          a = d.sigma * a + (1.0 - d.sigma) * sp;
        }
      }
      fx -= l.vx * (fp + a);
      fy -= l.vy * (fp + a);
    }
  } else if (coeffs && d.nwlinks > 0) {
    // the same two passes on the H2 coefficients of the input state: a
    // population of velocity v at cell o is w_v (a0 + vx bx + vy by + vx^2 cxx
    // + vx vy cxy + vy^2 cyy)(o)
    const S* __restrict__ c = static_cast<const S*>(d.mbuf[n & 1]);
    const int64_t ks = d.mks;
    auto pop = [&](int64_t o, double w, double vx, double vy) {
      return w * ((double)c[o] + vx * (double)c[ks + o] + vy * (double)c[2 * ks + o] +
                  vx * vx * (double)c[3 * ks + o] + vx * vy * (double)c[4 * ks + o] +
                  vy * vy * (double)c[5 * ks + o]);
    };
    __shared__ double cmass[kMaxWallCols];
    for (int k = threadIdx.x; k < d.nwcols; k += kBlock) {
      const WallCol& col = d.wcols[k];
      double m = 0.0;
      for (int r = 0; r < 3; ++r)
        for (int j = 0; j < 6; ++j) m += col.mc[r][j] * (double)c[j * ks + col.cell[r]];
      cmass[k] = m;
    }
    __syncthreads();
    const double U = d.drive[n].u;
    const double ladd = d.ladd_scale * U;
    for (int i = threadIdx.x; i < d.nwlinks; i += kBlock) {
      const WallLink l = d.wlinks[i];
      const double fp = pop(l.cell_partner, l.w, -l.vx, -l.vy);
      double a;
      if (l.col < 0) {
        a = fp + l.w * l.vx * ladd;
      } else {
        a = ds_box_arrival(d.wcols[l.col], d.rho0, U, cmass[l.col], l.w, l.vx, d.theta);
        if (d.sigma != 1.0) {
          const double sp = l.normal ? pop(l.cell_spec, l.w, -l.vx, l.vy) + l.w * l.vx * ladd
                                     : pop(l.cell_spec, l.w, l.vx, -l.vy);
          a = d.sigma * a + (1.0 - d.sigma) * sp;
        }
      }
      fx -= l.vx * (fp + a);
      fy -= l.vy * (fp + a);
    }
  } else if (coeffs) {
    const S* __restrict__ c = static_cast<const S*>(d.mbuf[n & 1]);
    const int64_t ks = d.mks;
    for (int i = threadIdx.x; i < d.nfcells; i += kBlock) {
      const ForceCell& cell = d.fcells[i];
      const CellWeights& fc = d.cweights[cell.pat];
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double v = (double)c[k * ks + cell.off];
        fx += fc.wx[k] * v;
        fy += fc.wy[k] * v;
        fm += fc.wm[k] * v;
      }
    }
  } else {
    const S* __restrict__ f = static_cast<const S*>(n & 1 ? d.buf[1] : d.buf[0]);
#pragma unroll 4
    for (int i = threadIdx.x; i < d.nlinks; i += kBlock) {
      const ForceLink& link = d.links[i];
      const LinkWeights& l = d.lweights[link.pat];
      const double v = (double)f[link.off];
      fx += l.wx * v;
      fy += l.wy * v;
      fm += l.wm * v;
    }
  }
  __shared__ double red[3][kBlock / 64];
  fx = wave_sum(fx);
  fy = wave_sum(fy);
  fm = wave_sum(fm);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[0][wave] = fx;
    red[1][wave] = fy;
    red[2][wave] = fm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sx = 0.0, sy = 0.0, sm = 0.0;
#pragma unroll
    for (int k = 0; k < kBlock / 64; ++k) {
      sx += red[0][k];
      sy += red[1][k];
      sm += red[2][k];
    }
    fx = d.fstatic[0] + d.kladd[0] * dr.u + sx;
    fy = d.fstatic[1] + d.kladd[1] * dr.u + sy;
    if (d.wall == WALL_DS && d.geom == GEOM_PLATE) {
      // the diffuse emissions' share of -sum v_i f_i^adv over the links:
      // every column emits w_i rho_w E_i(U) along each link, rho_w from the
      // column's crossing mass (rest part nx rho0 A1, deviation sm)
      const double U = dr.u, uu = U * U;
      const double emit = d.ds[0] + uu * d.ds[1];
      const double nr = d.ds[5];
      fx -= d.sigma * (nr * d.ds[0] * U * d.ds[2] + sm * U * d.ds[2]) / emit;
      fy -= d.sigma *
            (nr * uu * (d.ds[0] * d.ds[4] - d.ds[1] * d.ds[3]) + sm * (d.ds[3] + uu * d.ds[4])) /
            emit;
    }
    const int64_t h = n % d.hist_cap;
    d.hist[2 * h] = fx;
    d.hist[2 * h + 1] = fy;
    if (in_window) {
      st->lockin[0] = lk[0] + fx * dr.s;
      st->lockin[1] = lk[1] + fx * dr.c;
      st->lockin[2] = lk[2] + fx;
      st->lockin[3] = lk[3] + fy * dr.s;
      st->lockin[4] = lk[4] + fy * dr.c;
      st->lockin[5] = lk[5] + fy;
    }
    st->step = n + 1;
  }
}

template <typename S>
__global__ __launch_bounds__(kBlock) void finalize_kernel(const SolveDesc* __restrict__ descs,
                                                          const int32_t* __restrict__ solves,
                                                          int mode) {
  finalize_solve<S>(descs[solves[blockIdx.x]], mode);
}

template <class L, typename S, bool BGK, bool DSW>
static hipError_t launch_step_t(int cpt, const SolveDesc* descs, const WorkItem* work, int nwork,
                                const KernelLattice& lat, hipStream_t stream,
                                const KernelEvents& ev) {
  switch (cpt) {
    case 1:
      launch_kernel(step_kernel<L, S, BGK, DSW, kBlock, false>, dim3(nwork), dim3(kBlock), stream,
                    ev, descs, work, lat);
      break;
    case 2:
      launch_kernel(step_kernel<L, S, BGK, DSW, 2 * kBlock, false>, dim3(nwork),
                    dim3(2 * kBlock), stream, ev, descs, work, lat);
      break;
    case 4:
      launch_kernel(step_kernel<L, S, BGK, DSW, 4 * kBlock, false>, dim3(nwork),
                    dim3(4 * kBlock), stream, ev, descs, work, lat);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t launch_step_l(bool bgk, bool ds, int cpt, bool outm, const SolveDesc* descs,
                                const WorkItem* work, int nwork, const KernelLattice& lat,
                                hipStream_t stream, const KernelEvents& ev) {
  if (outm) {
    // one step of a solver kept in coefficients: any wall
    if (bgk || cpt != 1) return hipErrorInvalidValue;
    launch_kernel(step_kernel<L, S, false, true, kBlock, true>, dim3(nwork), dim3(kBlock), stream,
                  ev, descs, work, lat);
    return hipGetLastError();
  }
  if (bgk)
    return ds ? launch_step_t<L, S, true, true>(cpt, descs, work, nwork, lat, stream, ev)
              : launch_step_t<L, S, true, false>(cpt, descs, work, nwork, lat, stream, ev);
  return ds ? launch_step_t<L, S, false, true>(cpt, descs, work, nwork, lat, stream, ev)
            : launch_step_t<L, S, false, false>(cpt, descs, work, nwork, lat, stream, ev);
}

hipError_t launch_step(int Q, bool f64, bool bgk, bool ds, int cpt, bool outm,
                       const SolveDesc* descs, const WorkItem* work, int nwork,
                       const KernelLattice& lat, hipStream_t stream, KernelEvents ev) {
  if (nwork <= 0) return hipSuccess;
  if (Q == 9)
    return f64 ? launch_step_l<D2Q9, double>(bgk, ds, cpt, outm, descs, work, nwork, lat, stream,
                                             ev)
               : launch_step_l<D2Q9, float>(bgk, ds, cpt, outm, descs, work, nwork, lat, stream,
                                            ev);
  return f64 ? launch_step_l<D2Q37, double>(bgk, ds, cpt, outm, descs, work, nwork, lat, stream,
                                            ev)
             : launch_step_l<D2Q37, float>(bgk, ds, cpt, outm, descs, work, nwork, lat, stream,
                                           ev);
}

hipError_t launch_finalize(bool f64, const SolveDesc* descs, const int32_t* solves, int nsolves,
                           int mode, hipStream_t stream) {
  if (nsolves <= 0) return hipSuccess;
  if (f64)
    hipLaunchKernelGGL(finalize_kernel<double>, dim3(nsolves), dim3(kBlock), 0, stream, descs,
                       solves, mode);
  else
    hipLaunchKernelGGL(finalize_kernel<float>, dim3(nsolves), dim3(kBlock), 0, stream, descs,
                       solves, mode);
  return hipGetLastError();
}

}  // namespace lbm
