// C ABI of the solver: validation, device memory layout, lifecycle, the
// per-step launch sequence, and host-side read-out (force history, lock-in
// fit, populations).  See include/lbm.h for the contract of each call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "internal.hpp"

using namespace lbm;

namespace lbm {

// Workgroups of a launch are dealt to the 8 XCDs in turn (workgroup b runs on
// XCD b % 8), and each XCD has its own L2.  Tiles of one lattice row share the
// cache lines at their ends (the pulls are shifted by up to 3 cells), so the
// rows ("super-rows" of `span` tiles, about one lattice row) are dealt to the
// XCDs in turn: workgroups 8k..8k+7 take tile j of 8 consecutive rows.  All
// XCDs then work on one compact band of rows at a time (good HBM page
// locality) while every row stays within one L2.  Positions without a tile
// are no-op items (tile -1), which also keeps the next solve aligned.
void order_tiles(std::vector<WorkItem>* out, int32_t solve, int32_t ntiles, int32_t span) {
  while (out->size() % 8) out->push_back(WorkItem{solve, -1});
  span = std::max<int32_t>(1, span);
  const int32_t nrows = (ntiles + span - 1) / span;
  for (int32_t g = 0; g < nrows; g += 8)
    for (int32_t k = 0; k < span; ++k)
      for (int32_t i = 0; i < 8; ++i) {
        const int32_t row = g + i, t = row * span + k;
        out->push_back(WorkItem{solve, row < nrows && t < ntiles ? t : -1});
      }
}

// Coefficient-kernel tiles (of a solve with this layout) that hold a cell
// with a wall link: the band of R cells around the body, the plate's wall rows
// (the same band the kernel tests per wavefront).
std::vector<char> coef_wall_tiles(const lbm_params* p, const Layout& lay, int R) {
  std::vector<char> wall((size_t)lay.mntiles, 0);
  int wx0 = 0, wx1 = p->nx, wy0 = 0, wy1 = 0;
  bool far_band = false;
  if (p->geometry == LBM_GEOM_BOX) {
    wx0 = p->box_x0 - R;
    wx1 = p->box_x0 + p->box_lx + R;
    wy0 = p->box_y0 - R;
    wy1 = p->box_y0 + p->box_ly + R;
  } else if (p->geometry == LBM_GEOM_PLATE) {
    wy1 = R;
    far_band = p->far == LBM_FAR_WALL;
  }
  const int th = coef_tile_rows(lay.coef_k);
  for (int32_t t = 0; t < lay.mntiles; ++t) {
    const int x0 = (t % lay.tiles_x) * kCoefTileW, y0 = (t / lay.tiles_x) * th;
    wall[t] = (x0 < wx1 && x0 + kCoefTileW > wx0 && y0 < wy1 && y0 + th > wy0) ||
              (far_band && y0 + th > p->ny - R);
  }
  return wall;
}

void order_coef_tiles(std::vector<WorkItem>* front, std::vector<WorkItem>* rest, int32_t solve,
                      const std::vector<char>& wall, int32_t ntiles, int32_t span, bool banded) {
  for (int32_t t = 0; t < ntiles; ++t)
    if (wall[t]) front->push_back(WorkItem{solve, t});
  const size_t from = rest->size();
  if (banded)
    order_tiles_banded(rest, solve, ntiles, span);
  else
    order_tiles(rest, solve, ntiles, span);
  for (size_t i = from; i < rest->size(); ++i) {
    WorkItem& w = (*rest)[i];
    if (w.tile >= 0 && wall[w.tile]) w.tile = -1;
  }
}

void join_front(std::vector<WorkItem>* front, const std::vector<WorkItem>& rest) {
  while (front->size() % 8) front->push_back(WorkItem{0, -1});
  front->insert(front->end(), rest.begin(), rest.end());
}

void order_tiles_banded(std::vector<WorkItem>* out, int32_t solve, int32_t ntiles,
                        int32_t span) {
  while (out->size() % 8) out->push_back(WorkItem{solve, -1});
  span = std::max<int32_t>(1, span);
  const int32_t nrows = (ntiles + span - 1) / span;
  const int32_t band = (nrows + 7) / 8, per = band * span;
  for (int32_t j = 0; j < per; ++j)
    for (int32_t x = 0; x < 8; ++x) {
      const int32_t row = x * band + j / span, t = row * span + j % span;
      out->push_back(WorkItem{solve, row < nrows && t < ntiles ? t : -1});
    }
}

// Work-list length order_tiles (and order_tiles_banded) produces for one
// solve starting aligned.
int64_t ordered_length(int64_t ntiles, int64_t span) {
  span = std::max<int64_t>(1, span);
  const int64_t nrows = (ntiles + span - 1) / span;
  return (nrows + 7) / 8 * 8 * span;
}

}  // namespace lbm

namespace {

template <class L>
void fill_lattice(HostLattice* h) {
  h->Q = L::Q;
  h->R = L::R;
  for (int i = 0; i < L::Q; ++i) {
    h->vx.push_back(L::vx[i]);
    h->vy.push_back(L::vy[i]);
    h->orbit.push_back(L::orbit[i]);
    h->opp.push_back(opposite<L>(i));
  }
}

bool host_lattice(int Q, HostLattice* h) {
  if (Q == 9) fill_lattice<D2Q9>(h);
  else if (Q == 37) fill_lattice<D2Q37>(h);
  else return false;
  return lattice_weights(Q, &h->lw);
}

// One coefficient plane must stay addressable with 32-bit byte offsets.
bool coefficient_plane_fits(const lbm_params* p) {
  const uint64_t es = p->storage == LBM_STORE_F64 ? 8 : 4;
  return (uint64_t)p->ny * align_up((uint64_t)p->nx, kCoefTileW) * es < ((uint64_t)1 << 31);
}

// Device state kept as the six H2 coefficients (else the Q populations).
bool uses_coefficients(const lbm_params* p) {
  if (p->representation == LBM_REPR_COEFFICIENTS ||
      p->representation == LBM_REPR_COEFFICIENTS_NOLOAD)
    return true;
  return p->representation == LBM_REPR_AUTO && p->collision == LBM_COLL_REGULARIZED &&
         p->nx >= kCoefTileW && coefficient_plane_fits(p);
}

int validate(const lbm_params* p, HostLattice* lat) {
  if (!p) return LBM_EINVAL;
  if (p->abi_version != LBM_ABI_VERSION) return LBM_EABI;
  if (!host_lattice((int)p->lattice, lat)) return LBM_EINVAL;
  if (p->storage != LBM_STORE_F64 && p->storage != LBM_STORE_F32_DEV) return LBM_EINVAL;
  if (p->collision != LBM_COLL_REGULARIZED && p->collision != LBM_COLL_BGK) return LBM_EINVAL;
  if (p->wall != LBM_WALL_BB && p->wall != LBM_WALL_DS && p->wall != LBM_WALL_MAXWELL)
    return LBM_EINVAL;
  if (p->wall != LBM_WALL_BB && p->geometry == LBM_GEOM_PERIODIC) return LBM_EINVAL;
  if (p->wall == LBM_WALL_MAXWELL && !(p->accommodation >= 0.0 && p->accommodation <= 1.0))
    return LBM_EINVAL;
  if (p->far != LBM_FAR_WALL && p->far != LBM_FAR_EQ) return LBM_EINVAL;
  if (p->representation > LBM_REPR_COEFFICIENTS_NOLOAD) return LBM_EINVAL;
  const bool coef_asked = p->representation == LBM_REPR_COEFFICIENTS ||
                          p->representation == LBM_REPR_COEFFICIENTS_NOLOAD;
  if (coef_asked && p->collision != LBM_COLL_REGULARIZED) return LBM_EINVAL;
  // a box with diffuse or Maxwell faces: at most kMaxWallCols face columns
  if (p->wall != LBM_WALL_BB && p->geometry == LBM_GEOM_BOX &&
      2 * ((int64_t)p->box_lx + p->box_ly) > kMaxWallCols)
    return LBM_EINVAL;
  const int R = lat->R;
  if (p->nx < std::max(3, R) || p->ny < std::max(3, R)) return LBM_EINVAL;
  if ((int64_t)p->nx * p->ny > (int64_t)1 << 30) return LBM_EINVAL;
  if (coef_asked && !coefficient_plane_fits(p)) return LBM_EINVAL;
  // tile: cells per thread of the population kernel, or tile variant of the
  // coefficient kernel
  if (uses_coefficients(p)) {
    if (p->tile > (uint32_t)kCoefKMax) return LBM_EINVAL;
  } else if (p->tile != 0 && p->tile != 1 && p->tile != 2 && p->tile != 4) {
    return LBM_EINVAL;
  }
  if (!(p->tau > 0.5)) return LBM_EINVAL;  // rejects NaN too; +inf allowed
  if (!std::isfinite(p->omega) || !std::isfinite(p->u0)) return LBM_EINVAL;
  if (!(p->rho0 > 0) || !std::isfinite(p->rho0)) return LBM_EINVAL;
  if (p->max_steps < 1 || p->max_steps > ((int64_t)1 << 32)) return LBM_EINVAL;
  if (p->lockin_first < 0 || p->lockin_count < 0 ||
      p->lockin_first + p->lockin_count > p->max_steps)
    return LBM_EINVAL;
  if (p->history_capacity < 0 || p->history_capacity > p->max_steps) return LBM_EINVAL;
  switch (p->geometry) {
    case LBM_GEOM_PLATE:
    case LBM_GEOM_PERIODIC:
      break;
    case LBM_GEOM_BOX:
      if (p->far != LBM_FAR_EQ) return LBM_EINVAL;
      if (p->box_lx < R || p->box_ly < R || p->box_x0 < R || p->box_y0 < R) return LBM_EINVAL;
      if ((int64_t)p->box_x0 + p->box_lx + R > p->nx ||
          (int64_t)p->box_y0 + p->box_ly + R > p->ny)
        return LBM_EINVAL;
      break;
    default:
      return LBM_EINVAL;
  }
  return LBM_OK;
}

bool in_body(const lbm_params* p, int x, int y) {
  return p->geometry == LBM_GEOM_BOX && x >= p->box_x0 && x < p->box_x0 + p->box_lx &&
         y >= p->box_y0 && y < p->box_y0 + p->box_ly;
}

// True if a population arriving at fluid cell (x, y) along q comes from the
// moving wall or body (a bounce-back link that carries force).
bool is_link(const lbm_params* p, const HostLattice& L, int x, int y, int q) {
  const int sx = x - L.vx[q], sy = y - L.vy[q];
  if (p->geometry == LBM_GEOM_PLATE) return sy < 0;
  if (p->geometry == LBM_GEOM_BOX) return in_body(p, sx, sy);
  return false;
}

// Mirror cell of the bounce-back link arriving at fluid cell (x, y) along q
// (half-way walls; the same rules as the kernels).
void mirror_of(const lbm_params* p, const HostLattice& L, int x, int y, int q, int* px, int* py) {
  const int sx = x - L.vx[q], sy = y - L.vy[q];
  if (p->geometry == LBM_GEOM_PLATE) {
    *px = x;
    *py = -1 - sy;
    return;
  }
  const int x0 = p->box_x0, x1 = p->box_x0 + p->box_lx;
  const int y0 = p->box_y0, y1 = p->box_y0 + p->box_ly;
  *px = x < x0 ? 2 * x0 - 1 - sx : (x >= x1 ? 2 * x1 - 1 - sx : x);
  *py = y < y0 ? 2 * y0 - 1 - sy : (y >= y1 ? 2 * y1 - 1 - sy : y);
}

// Momentum-exchange tables of the wall force.  Each bounce-back link (fluid
// arrival x along v_i, mirror cell x_p) contributes
//   -v_i (f_opp(x_p) + f_i^adv(x)) = -v_i (2 w_i rho0 + 2 df_opp(x_p) + 2 w_i rho0 (v_i.U_w)/theta)
// with df the stored deviation.  The rest part and the moving-wall part are
// geometry constants (fstatic, kladd times U_w), summed here in long double;
// the deviation part becomes the link list (population state) or, per mirror
// cell, two 6-vectors acting on the cell's H2 coefficients (coefficient state:
// df_opp(x_p) = w_i (a0 - vx bx - vy by + vx^2 cxx + vx vy cxy + vy^2 cyy)).
// At a diffuse wall (eq. DS) the arrival f_i^adv is the wall's emission: the
// tables then carry -v_i df_opp(x_p) and the crossing mass df_opp(x_p), and
// the emission's share follows from the lattice sums in `ds` (finalize).
struct ForceTables {
  std::vector<ForceLink> links;
  std::vector<ForceCell> cells;
  std::vector<LinkWeights> lweights;
  std::vector<CellWeights> cweights;
  double fstatic[2] = {0, 0}, kladd[2] = {0, 0};
  double ds[6] = {0, 0, 0, 0, 0, 0};
  // box with diffuse or Maxwell faces
  std::vector<WallCol> wcols;
  std::vector<WallLink> wlinks;
};

bool diffuse_box(const lbm_params* p) {
  return p->geometry == LBM_GEOM_BOX && p->wall != LBM_WALL_BB;
}

// Tables of a box with diffuse or Maxwell faces: its links face column by
// face column (faces below, above the body by arrival x, left, right of it
// by arrival y; in a column by arrival cell and direction), then the corner
// links; per column the lattice sums of its links (long double).  The force
// is -sum v_l (f_partner + f_arrival) over every link: the rest-state parts
// give fstatic, the rest is formed per link by the finalize.
void build_wall_tables(const lbm_params* p, const HostLattice& L, const Layout& lay,
                       ForceTables* t) {
  const int R = L.R;
  const int x0 = p->box_x0, x1 = p->box_x0 + p->box_lx;
  const int y0 = p->box_y0, y1 = p->box_y0 + p->box_ly;
  const long double th = L.lw.theta_ld;
  auto find = [&](int vx, int vy) {
    for (int j = 0; j < L.Q; ++j)
      if (L.vx[j] == vx && L.vy[j] == vy) return j;
    return -1;
  };
  auto face_of = [&](int x, int y) {
    const bool inx = x >= x0 && x < x1, iny = y >= y0 && y < y1;
    if (inx && !iny) return y < y0 ? 0 : 1;
    if (iny && !inx) return x < x0 ? 2 : 3;
    return -1;
  };
  long double sx = 0, sy = 0;
  // crossing-mass weights of the current column over its cells' coefficients
  long double mc[3][6];
  // the links of a fluid cell, in direction order
  auto add_cell = [&](int x, int y, int col) {
    for (int q = 0; q < L.Q; ++q) {
      const int vx = L.vx[q], vy = L.vy[q];
      const int sxs = x - vx, sys = y - vy;
      if (!in_body(p, sxs, sys)) continue;
      int px, py;
      mirror_of(p, L, x, y, q, &px, &py);
      const long double w = L.lw.w_orbit_ld[L.orbit[q]];
      WallLink l{};
      l.off_partner = L.opp[q] * lay.qs + py * lay.ys + px;
      l.cell_partner = (int64_t)py * lay.mpitch + px;
      l.col = col;
      l.w = (double)w;
      l.vx = vx;
      l.vy = vy;
      const int face = face_of(x, y);
      l.normal = face >= 2;
      if (face == 0 || face == 1) {
        l.off_spec = find(vx, -vy) * lay.qs + py * lay.ys + sxs;
        l.cell_spec = (int64_t)py * lay.mpitch + sxs;
      } else if (face >= 2) {
        l.off_spec = find(-vx, vy) * lay.qs + sys * lay.ys + px;
        l.cell_spec = (int64_t)sys * lay.mpitch + px;
      }
      if (col >= 0) {
        // the partner's distance from the face (it lies in the link's column)
        const int k = face == 0 ? y0 - py : face == 1 ? py - (y1 - 1) : face == 2 ? x0 - px
                                                                                  : px - (x1 - 1);
        const long double g[6] = {1, -(long double)vx, -(long double)vy,
                                  (long double)vx * vx, (long double)vx * vy,
                                  (long double)vy * vy};
        for (int j = 0; j < 6; ++j) mc[k - 1][j] += w * g[j];
      }
      sx -= 2.0L * w * p->rho0 * vx;
      sy -= 2.0L * w * p->rho0 * vy;
      t->wlinks.push_back(l);
    }
  };
  // columns: cells of a face column from the face outwards
  const int ncol = 2 * (p->box_lx + p->box_ly);
  t->wcols.assign((size_t)ncol, WallCol{});
  for (int c = 0; c < ncol; ++c) {
    int face, at;
    if (c < p->box_lx) { face = 0; at = x0 + c; }
    else if (c < 2 * p->box_lx) { face = 1; at = x0 + c - p->box_lx; }
    else if (c < 2 * p->box_lx + p->box_ly) { face = 2; at = y0 + c - 2 * p->box_lx; }
    else { face = 3; at = y0 + c - 2 * p->box_lx - p->box_ly; }
    WallCol& wc = t->wcols[(size_t)c];
    wc.first = (int32_t)t->wlinks.size();
    for (auto& row : mc)
      for (auto& v : row) v = 0;
    for (int k = 1; k <= R; ++k) {
      const int x = face <= 1 ? at : (face == 2 ? x0 - k : x1 - 1 + k);
      const int y = face >= 2 ? at : (face == 0 ? y0 - k : y1 - 1 + k);
      wc.cell[k - 1] = (int64_t)y * lay.mpitch + x;
      add_cell(x, y, c);
    }
    for (int k = 0; k < 3; ++k)
      for (int j = 0; j < 6; ++j) wc.mc[k][j] = (double)mc[k][j];
    wc.count = (int32_t)t->wlinks.size() - wc.first;
    long double mr = 0, z1 = 0, z2 = 0, l1 = 0;
    for (int i = wc.first; i < wc.first + wc.count; ++i) {
      const WallLink& l = t->wlinks[(size_t)i];
      const long double w = L.lw.w_orbit_ld[L.orbit[find((int)l.vx, (int)l.vy)]];
      const long double vx = l.vx;
      mr += w;
      z1 += w * vx / th;
      z2 += w * (vx * vx / (2 * th * th) - 1 / (2 * th));
      l1 += 2 * w * vx / th;
    }
    wc.Mr = (double)mr;
    wc.Z1 = (double)z1;
    wc.Z2 = (double)z2;
    wc.L1 = (double)l1;
  }
  // corner links: cells outside the body's range on both axes, within R
  for (int y = y0 - R; y < y1 + R; ++y)
    for (int x = x0 - R; x < x1 + R; ++x)
      if (!in_body(p, x, y) && face_of(x, y) < 0) add_cell(x, y, -1);
  t->fstatic[0] = (double)sx;
  t->fstatic[1] = (double)sy;
}

void build_force_tables(const lbm_params* p, const HostLattice& L, const Layout& lay,
                        ForceTables* t) {
  if (diffuse_box(p)) {
    build_wall_tables(p, L, lay, t);
    return;
  }
  long double sx = 0, sy = 0, kx = 0, ky = 0;
  // diffuse or Maxwell wall: a share sigma of every arrival is the diffuse
  // emission, the rest the specular image of a crossing population (the
  // same v_x): shear sees sigma of the reflected deviations, the normal
  // force 2 - sigma of them
  const bool diffuse = p->wall == LBM_WALL_DS || p->wall == LBM_WALL_MAXWELL;
  const long double sigma = p->wall == LBM_WALL_MAXWELL ? (long double)p->accommodation : 1.0L;
  const long double mwx = diffuse ? sigma : 2.0L, mwy = diffuse ? 2.0L - sigma : 2.0L;
  std::unordered_map<int64_t, size_t> index;  // mirror cell -> position in t->cells
  std::vector<CellWeights> cw;                 // the weights of t->cells
  auto cell_for = [&](int px, int py) -> CellWeights& {
    const int64_t key = (int64_t)py * p->nx + px;
    auto it = index.find(key);
    if (it != index.end()) return cw[it->second];
    ForceCell fc{};
    fc.off = (int64_t)py * lay.mpitch + px;
    index.emplace(key, t->cells.size());
    t->cells.push_back(fc);
    cw.push_back(CellWeights{});
    return cw.back();
  };
  // one pattern per distinct set of weights (compared bit for bit)
  std::unordered_map<std::string, int32_t> lpat, cpat;
  auto pattern = [](auto& pats, auto& table, const auto& wts) {
    const std::string key(reinterpret_cast<const char*>(&wts), sizeof(wts));
    auto it = pats.find(key);
    if (it != pats.end()) return it->second;
    const int32_t k = (int32_t)table.size();
    table.push_back(wts);
    pats.emplace(key, k);
    return k;
  };
  int x0 = 0, x1 = 0, y0 = 0, y1 = 0;
  if (p->geometry == LBM_GEOM_PLATE) {
    x0 = 0; x1 = p->nx; y0 = 0; y1 = std::min(L.R, p->ny);
  } else if (p->geometry == LBM_GEOM_BOX) {
    x0 = p->box_x0 - L.R; x1 = p->box_x0 + p->box_lx + L.R;
    y0 = p->box_y0 - L.R; y1 = p->box_y0 + p->box_ly + L.R;
  }
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) {
      if (in_body(p, x, y)) continue;
      for (int q = 0; q < L.Q; ++q) {
        if (!is_link(p, L, x, y, q)) continue;
        const long double w = L.lw.w_orbit_ld[L.orbit[q]];
        const int vx = L.vx[q], vy = L.vy[q];
        sx -= vx * 2.0L * w * p->rho0;
        sy -= vy * 2.0L * w * p->rho0;
        if (!diffuse) {
          kx -= vx * 2.0L * w * p->rho0 * vx / L.lw.theta_ld;
          ky -= vy * 2.0L * w * p->rho0 * vx / L.lw.theta_ld;
        }
        int px, py;
        mirror_of(p, L, x, y, q, &px, &py);
        const LinkWeights lwt{(double)(-mwx * vx), (double)(-mwy * vy), diffuse ? 1.0 : 0.0,
                              0.0};
        t->links.push_back(ForceLink{L.opp[q] * lay.qs + py * lay.ys + px,
                                     pattern(lpat, t->lweights, lwt), 0});
        if (lay.mom) {
          CellWeights& fc = cell_for(px, py);
          // basis of the opposite direction -v at the mirror cell
          const long double g[6] = {1, -(long double)vx, -(long double)vy,
                                    (long double)vx * vx, (long double)vx * vy,
                                    (long double)vy * vy};
          for (int k = 0; k < 6; ++k) {
            fc.wx[k] += (double)(-mwx * vx * w * g[k]);
            fc.wy[k] += (double)(-mwy * vy * w * g[k]);
            if (diffuse) fc.wm[k] += (double)(w * g[k]);
          }
        }
      }
    }
  for (size_t i = 0; i < t->cells.size(); ++i) t->cells[i].pat = pattern(cpat, t->cweights, cw[i]);
  t->fstatic[0] = (double)sx;
  t->fstatic[1] = (double)sy;
  t->kladd[0] = (double)kx;
  t->kladd[1] = (double)ky;
  if (diffuse) {
    // lattice sums over the directions the wall emits (v_y > 0)
    const long double th = L.lw.theta_ld;
    long double a1 = 0, a2 = 0, bx = 0, by0 = 0, by2 = 0;
    for (int q = 0; q < L.Q; ++q) {
      if (L.vy[q] <= 0) continue;
      const long double w = L.lw.w_orbit_ld[L.orbit[q]];
      const long double vx = L.vx[q], vy = L.vy[q];
      const long double e2 = vx * vx / (2 * th * th) - 1 / (2 * th);
      a1 += vy * w;
      a2 += vy * w * e2;
      bx += vy * vx * vx * w / th;
      by0 += vy * vy * w;
      by2 += vy * vy * w * e2;
    }
    t->ds[0] = (double)a1;
    t->ds[1] = (double)a2;
    t->ds[2] = (double)bx;
    t->ds[3] = (double)by0;
    t->ds[4] = (double)by2;
    t->ds[5] = (double)((long double)p->nx * p->rho0);
  }
}

void make_layout(const lbm_params* p, const HostLattice& L, Layout* lay) {
  const uint64_t es = p->storage == LBM_STORE_F64 ? 8 : 4;
  if (p->nx >= 64) {
    // row-interleaved: the Q rows of lattice row y are contiguous, so the Q
    // streams of a workgroup touch a few contiguous rows of Q*pitch elements
    lay->pitch = (int64_t)align_up(p->nx, 64);
    lay->qs = lay->pitch;
    lay->ys = (int64_t)L.Q * lay->pitch;
    lay->buf_elems = lay->ys * p->ny;
  } else {
    // narrow lattices: whole-lattice planes (a wavefront covers several rows
    // of one plane contiguously); planes start 256 elements past a
    // 256-element boundary apart to spread them over HBM channels
    lay->pitch = p->nx;
    lay->qs = (int64_t)align_up((uint64_t)p->ny * lay->pitch, 256) + 256;
    lay->ys = lay->pitch;
    lay->buf_elems = lay->qs * L.Q;
  }
  lay->mom = uses_coefficients(p);
  lay->loadable = !(lay->mom && p->representation == LBM_REPR_COEFFICIENTS_NOLOAD);
  if (lay->mom) {
    lay->coef_k = p->tile ? (int32_t)p->tile : kCoefKDefault;
    const int th = coef_tile_rows(lay->coef_k);
    lay->tiles_x = (p->nx + kCoefTileW - 1) / kCoefTileW;
    lay->mntiles = lay->tiles_x * ((p->ny + th - 1) / th);
    // element (k, y, x) of a buffer at k*mks + y*mpitch + x.  Row-interleaved
    // where the whole buffer stays addressable with 32-bit byte offsets: the
    // six coefficient rows of lattice row y side by side, so the staged rows
    // and the stores of a tile fall in one contiguous span (2 % faster on a
    // state streaming from HBM than six whole planes).  Larger lattices keep
    // six planes, each under 2 GiB, spaced 256 elements past a 256-element
    // boundary.
    const int64_t pitch = (int64_t)align_up(p->nx, 64);
    if ((uint64_t)p->ny * 6 * (uint64_t)pitch * es < ((uint64_t)1 << 31)) {
      lay->mpitch = 6 * pitch;
      lay->mks = pitch;
      lay->mbuf_bytes = ((uint64_t)align_up((uint64_t)p->ny * lay->mpitch, 256) + 256) * es;
    } else {
      lay->mpitch = pitch;
      lay->mks = (int64_t)align_up((uint64_t)p->ny * pitch, 256) + 256;
      lay->mbuf_bytes = 6 * (uint64_t)lay->mks * es;
    }
  }
  const int64_t ncells = (int64_t)p->nx * p->ny;
  // the coefficient solver's population kernel (first step after a load)
  // runs with one cell per thread
  lay->cpt = lay->mom ? 1 : (p->tile ? (int32_t)p->tile : 1);
  lay->cells_per_tile = kBlock * lay->cpt;
  lay->ntiles = (int32_t)((ncells + lay->cells_per_tile - 1) / lay->cells_per_tile);
  lay->hist_cap = p->history_capacity ? p->history_capacity : p->max_steps;
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o = align_up(o + std::max<uint64_t>(bytes, 1), kAlign);
    return at;
  };
  lay->off_desc = take(sizeof(SolveDesc));
  lay->off_state = take(sizeof(SolveState));
  // XCD-aware order pads each group of 8 rows to full length
  lay->nwork = (int32_t)ordered_length(lay->ntiles, (p->nx + lay->cells_per_tile - 1) /
                                                        lay->cells_per_tile);
  lay->off_work = take(sizeof(WorkItem) * (uint64_t)lay->nwork);
  if (lay->mom) {
    int64_t nwall = 0;
    for (char w : coef_wall_tiles(p, *lay, L.R)) nwall += w;
    lay->mnwork = (int32_t)((nwall + 7) / 8 * 8 + ordered_length(lay->mntiles, lay->tiles_x));
    lay->off_mwork = take(sizeof(WorkItem) * (uint64_t)lay->mnwork);
  }
  lay->off_solves = take(sizeof(int32_t));
  ForceTables ft;
  build_force_tables(p, L, *lay, &ft);
  lay->nlinks = (int32_t)ft.links.size();
  lay->nfcells = (int32_t)ft.cells.size();
  lay->off_links = take(sizeof(ForceLink) * ft.links.size());
  lay->off_fcells = take(sizeof(ForceCell) * ft.cells.size());
  lay->nlweights = (int32_t)ft.lweights.size();
  lay->ncweights = (int32_t)ft.cweights.size();
  lay->off_lweights = take(sizeof(LinkWeights) * ft.lweights.size());
  lay->off_cweights = take(sizeof(CellWeights) * ft.cweights.size());
  lay->nwcols = (int32_t)ft.wcols.size();
  lay->nwlinks = (int32_t)ft.wlinks.size();
  lay->off_wcols = take(sizeof(WallCol) * ft.wcols.size());
  lay->off_wlinks = take(sizeof(WallLink) * ft.wlinks.size());
  lay->off_drive = take(sizeof(Drive) * (uint64_t)p->max_steps);
  lay->off_hist = take(sizeof(double) * 2 * (uint64_t)lay->hist_cap);
  // a coefficient solver that cannot load populations has no population buffer
  lay->buf_bytes = lay->loadable ? (uint64_t)lay->buf_elems * es : 0;
  o = align_up(o, 4096);
  lay->off_buf[0] = lay->loadable ? take(lay->buf_bytes) : 0;
  if (lay->mom) {
    // one population buffer (a loaded state, read by the next step; none
    // without loads) and two coefficient buffers
    lay->off_buf[1] = lay->off_buf[0];
    o = align_up(o, 4096);
    lay->off_mbuf[0] = take(lay->mbuf_bytes);
    o = align_up(o, 4096);
    lay->off_mbuf[1] = take(lay->mbuf_bytes);
  } else {
    o = align_up(o, 4096);
    lay->off_buf[1] = take(lay->buf_bytes);
  }
  lay->total = o;
}


}  // namespace

namespace {

int init_solver(lbm_solver* s) {
  const lbm_params* p = &s->p;
  const Layout& lay = s->lay;
  char* b = s->base;
  ForceTables ft;
  build_force_tables(p, s->lat, lay, &ft);

  SolveDesc& d = s->desc;
  std::memset(&d, 0, sizeof(d));
  if (lay.loadable) {
    s->bufs[0] = d.buf[0] = b + lay.off_buf[0];
    s->bufs[1] = d.buf[1] = b + lay.off_buf[1];
  }
  d.drive = reinterpret_cast<const Drive*>(b + lay.off_drive);
  d.hist = reinterpret_cast<double*>(b + lay.off_hist);
  d.state = reinterpret_cast<SolveState*>(b + lay.off_state);
  d.links = reinterpret_cast<const ForceLink*>(b + lay.off_links);
  d.fcells = reinterpret_cast<const ForceCell*>(b + lay.off_fcells);
  d.lweights = reinterpret_cast<const LinkWeights*>(b + lay.off_lweights);
  d.cweights = reinterpret_cast<const CellWeights*>(b + lay.off_cweights);
  d.nlinks = lay.nlinks;
  if (lay.nwlinks > 0) {
    d.wcols = reinterpret_cast<const WallCol*>(b + lay.off_wcols);
    d.wlinks = reinterpret_cast<const WallLink*>(b + lay.off_wlinks);
    d.nwcols = lay.nwcols;
    d.nwlinks = lay.nwlinks;
  }
  d.theta = s->lat.lw.theta;
  d.nfcells = lay.nfcells;
  d.qs = lay.qs;
  d.ys = lay.ys;
  d.max_steps = p->max_steps;
  d.hist_cap = lay.hist_cap;
  d.lockin_first = p->lockin_first;
  d.lockin_count = p->lockin_count;
  d.nx = p->nx;
  d.ny = p->ny;
  d.ncells = p->nx * p->ny;
  d.geom = (int32_t)p->geometry;
  d.far = (int32_t)p->far;
  if (p->geometry == LBM_GEOM_BOX) {
    d.bx0 = p->box_x0;
    d.by0 = p->box_y0;
    d.bx1 = p->box_x0 + p->box_lx;
    d.by1 = p->box_y0 + p->box_ly;
  }
  d.inv_tau = std::isinf(p->tau) ? 0.0 : 1.0 / p->tau;
  d.rho0 = p->rho0;
  d.ladd_scale = 2.0 * p->rho0 / s->lat.lw.theta;
  d.fstatic[0] = ft.fstatic[0];
  d.fstatic[1] = ft.fstatic[1];
  d.kladd[0] = ft.kladd[0];
  d.kladd[1] = ft.kladd[1];
  d.wall = p->wall == LBM_WALL_BB ? WALL_BB : WALL_DS;
  d.sigma = p->wall == LBM_WALL_MAXWELL ? p->accommodation : 1.0;
  for (int k = 0; k < 6; ++k) d.ds[k] = ft.ds[k];
  if (lay.mom) {
    d.mbuf[0] = b + lay.off_mbuf[0];
    d.mbuf[1] = b + lay.off_mbuf[1];
    d.mks = lay.mks;
    d.mys = lay.mpitch;
    d.tiles_x = lay.tiles_x;
  }

  for (int k = 0; k < 8; ++k) s->klat.w[k] = s->lat.lw.w_orbit[k];
  s->klat.theta = s->lat.lw.theta;

  std::vector<WorkItem> work, mwork;
  order_tiles(&work, 0, lay.ntiles, (p->nx + lay.cells_per_tile - 1) / lay.cells_per_tile);
  if (lay.mom) {
    std::vector<WorkItem> rest;
    order_coef_tiles(&mwork, &rest, 0, coef_wall_tiles(p, lay, s->lat.R), lay.mntiles,
                     lay.tiles_x, 2 * lay.mbuf_bytes <= kCachedStateBytes);
    join_front(&mwork, rest);
    if ((int32_t)mwork.size() != lay.mnwork) return LBM_EINVAL;
  }
  std::vector<Drive> drive((size_t)p->max_steps);
  for (int64_t n = 0; n < p->max_steps; ++n) {
    const double arg = p->omega * ((double)n + 0.5);
    drive[n].u = p->u0 * std::sin(arg);
    drive[n].s = std::sin(arg);
    drive[n].c = std::cos(arg);
  }
  const int32_t solve0 = 0;
  s->d_desc = reinterpret_cast<SolveDesc*>(b + lay.off_desc);
  s->d_work = reinterpret_cast<WorkItem*>(b + lay.off_work);
  s->d_solves = reinterpret_cast<int32_t*>(b + lay.off_solves);
  s->d_mwork = lay.mom ? reinterpret_cast<WorkItem*>(b + lay.off_mwork) : nullptr;

  hipStream_t st = s->stream;
  int rc;
  if ((rc = hip_rc(hipMemcpyAsync(s->d_desc, &d, sizeof(d), hipMemcpyHostToDevice, st)))) return rc;
  if ((rc = hip_rc(hipMemcpyAsync(s->d_work, work.data(), sizeof(WorkItem) * work.size(),
                                  hipMemcpyHostToDevice, st))))
    return rc;
  if ((rc = hip_rc(hipMemcpyAsync(s->d_solves, &solve0, sizeof(solve0), hipMemcpyHostToDevice,
                                  st))))
    return rc;
  if (!ft.links.empty() &&
      (rc = hip_rc(hipMemcpyAsync(b + lay.off_links, ft.links.data(),
                                  sizeof(ForceLink) * ft.links.size(), hipMemcpyHostToDevice, st))))
    return rc;
  if (!ft.cells.empty() &&
      (rc = hip_rc(hipMemcpyAsync(b + lay.off_fcells, ft.cells.data(),
                                  sizeof(ForceCell) * ft.cells.size(), hipMemcpyHostToDevice, st))))
    return rc;
  if (!ft.lweights.empty() &&
      (rc = hip_rc(hipMemcpyAsync(b + lay.off_lweights, ft.lweights.data(),
                                  sizeof(LinkWeights) * ft.lweights.size(), hipMemcpyHostToDevice,
                                  st))))
    return rc;
  if (!ft.cweights.empty() &&
      (rc = hip_rc(hipMemcpyAsync(b + lay.off_cweights, ft.cweights.data(),
                                  sizeof(CellWeights) * ft.cweights.size(), hipMemcpyHostToDevice,
                                  st))))
    return rc;
  if (!ft.wcols.empty() &&
      (rc = hip_rc(hipMemcpyAsync(b + lay.off_wcols, ft.wcols.data(),
                                  sizeof(WallCol) * ft.wcols.size(), hipMemcpyHostToDevice, st))))
    return rc;
  if (!ft.wlinks.empty() &&
      (rc = hip_rc(hipMemcpyAsync(b + lay.off_wlinks, ft.wlinks.data(),
                                  sizeof(WallLink) * ft.wlinks.size(), hipMemcpyHostToDevice,
                                  st))))
    return rc;
  if ((rc = hip_rc(hipMemcpyAsync(b + lay.off_drive, drive.data(), sizeof(Drive) * drive.size(),
                                  hipMemcpyHostToDevice, st))))
    return rc;
  if (lay.mom) {
    if ((rc = hip_rc(hipMemcpyAsync(s->d_mwork, mwork.data(), sizeof(WorkItem) * mwork.size(),
                                    hipMemcpyHostToDevice, st))))
      return rc;

    if ((rc = hip_rc(hipMemsetAsync(b + lay.off_mbuf[0], 0, lay.mbuf_bytes, st)))) return rc;
    if ((rc = hip_rc(hipMemsetAsync(b + lay.off_mbuf[1], 0, lay.mbuf_bytes, st)))) return rc;
  }
  // rest state (zero deviations), zero counters, sums and history
  if ((rc = hip_rc(hipMemsetAsync(b + lay.off_state, 0, sizeof(SolveState), st)))) return rc;

  if ((rc = hip_rc(hipMemsetAsync(b + lay.off_hist, 0, sizeof(double) * 2 * lay.hist_cap, st))))
    return rc;
  if (lay.loadable && (rc = hip_rc(hipMemsetAsync(b + lay.off_buf[0], 0, lay.buf_bytes, st))))
    return rc;
  if (!lay.mom && (rc = hip_rc(hipMemsetAsync(b + lay.off_buf[1], 0, lay.buf_bytes, st))))
    return rc;
  return hip_rc(hipStreamSynchronize(st));
}

}  // namespace

int lbm::create_solver(const lbm_params* p, void* stream, void* dev_buf, uint64_t bytes,
                       bool graphs, lbm_solver** out) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_solver* s = new (std::nothrow) lbm_solver();
  if (!s) return LBM_ENOMEM;
  int rc = validate(p, &s->lat);
  if (rc) {
    delete s;
    return rc;
  }
  s->p = *p;
  make_layout(p, s->lat, &s->lay);
  s->stream = static_cast<hipStream_t>(stream);
  if (hipGetDevice(&s->device) != hipSuccess) {
    delete s;
    return LBM_EHIP;
  }
  if (dev_buf) {
    if (bytes < s->lay.total || (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) != 0) {
      delete s;
      return bytes < s->lay.total ? LBM_ENOMEM : LBM_EINVAL;
    }
    s->base = static_cast<char*>(dev_buf);
  } else {
    void* ptr = nullptr;
    if (hipMalloc(&ptr, s->lay.total) != hipSuccess) {
      (void)hipGetLastError();
      delete s;
      return LBM_ENOMEM;
    }
    s->base = static_cast<char*>(ptr);
    s->owned = true;
  }
  s->graphs_ok = graphs;
  rc = init_solver(s);
  if (rc) {
    if (s->owned) (void)hipFree(s->base);
    delete s;
    return rc;
  }
  *out = s;
  return LBM_OK;
}

// One step of a single solver: the population kernel, the population kernel
// writing coefficients (first step after populations were loaded into a
// coefficient solver), or the coefficient kernel; then the finalize.
namespace {

// Enqueue one step's launches (no host bookkeeping).
int launch_one_step(lbm_solver* s) {
  const bool f64 = s->p.storage == LBM_STORE_F64;
  const bool bgk = s->p.collision == LBM_COLL_BGK;
  const int Q = (int)s->p.lattice;
  const bool ds = s->p.wall != LBM_WALL_BB;
  int mode = 0;
  hipError_t e;
  if (!s->lay.mom) {
    e = launch_step(Q, f64, bgk, ds, s->lay.cpt, false, s->d_desc, s->d_work, s->lay.nwork,
                    s->klat, s->stream);
  } else if (s->pop_pending) {
    e = launch_step(Q, f64, false, ds, 1, true, s->d_desc, s->d_work, s->lay.nwork, s->klat,
                    s->stream);
    s->pop_pending = false;
  } else {
    e = launch_coef(Q, f64, s->lay.coef_k, ds, 2 * s->lay.mbuf_bytes > kCachedStateBytes,
                    s->d_desc, s->d_mwork, s->lay.mnwork, s->klat, s->stream);
    mode = 1;
  }
  if (e != hipSuccess) return LBM_EHIP;
  if (launch_finalize(f64, s->d_desc, s->d_solves, 1, mode, s->stream) != hipSuccess)
    return LBM_EHIP;
  return LBM_OK;
}

// Capture kGraphSteps steps of a solver whose state is in its steady
// representation (no pending population load).
bool capture_steps(lbm_solver* s) {
  if (s->stream == nullptr || s->pop_pending) return false;  // the null stream cannot be captured
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = true;
  for (int k = 0; k < kGraphSteps && ok; ++k) ok = launch_one_step(s) == LBM_OK;
  if (hipStreamEndCapture(s->stream, &g) != hipSuccess || !ok) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    return false;
  }
  hipGraphExec_t ex = nullptr;
  const bool inst = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  (void)hipGraphDestroy(g);
  if (!inst) {
    (void)hipGetLastError();
    return false;
  }
  s->graph = ex;
  return true;
}

}  // namespace

int step_one(lbm_solver* s) {
  const int rc = launch_one_step(s);
  if (rc) return rc;
  ++s->steps;
  return LBM_OK;
}

namespace {

int sync_and_check(lbm_solver* s) {
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  if (!s->sticky_unstable) {
    int32_t flag = 0;
    if (hipMemcpy(&flag, &s->desc.state->unstable, sizeof(flag), hipMemcpyDeviceToHost) !=
        hipSuccess)
      return LBM_EHIP;
    s->sticky_unstable = flag != 0;
  }
  return s->sticky_unstable ? LBM_EUNSTABLE : LBM_OK;
}

}  // namespace

extern "C" {

int lbm_params_init(lbm_params* p) {
  if (!p) return LBM_EINVAL;
  std::memset(p, 0, sizeof(*p));
  p->abi_version = LBM_ABI_VERSION;
  p->lattice = LBM_D2Q37;
  p->storage = LBM_STORE_F32_DEV;
  p->collision = LBM_COLL_REGULARIZED;
  p->wall = LBM_WALL_BB;
  p->accommodation = 1.0;
  p->geometry = LBM_GEOM_PLATE;
  p->far = LBM_FAR_WALL;
  p->rho0 = 1.0;
  return LBM_OK;
}

int lbm_lattice(int Q, int32_t* vx, int32_t* vy, double* w, double* theta) {
  HostLattice h;
  if (!host_lattice(Q, &h)) return LBM_EINVAL;
  for (int i = 0; i < Q; ++i) {
    if (vx) vx[i] = h.vx[i];
    if (vy) vy[i] = h.vy[i];
    if (w) w[i] = h.lw.w_orbit[h.orbit[i]];
  }
  if (theta) *theta = h.lw.theta;
  return LBM_OK;
}

int lbm_required_bytes(const lbm_params* p, uint64_t* bytes) {
  if (!bytes) return LBM_EINVAL;
  HostLattice lat;
  int rc = validate(p, &lat);
  if (rc) return rc;
  Layout lay;
  make_layout(p, lat, &lay);
  *bytes = lay.total;
  return LBM_OK;
}

int lbm_create(const lbm_params* p, void* hip_stream, lbm_solver** out) {
  return create_solver(p, hip_stream, nullptr, 0, true, out);
}

int lbm_create_in(const lbm_params* p, void* hip_stream, void* dev_buf, uint64_t bytes,
                  lbm_solver** out) {
  if (!dev_buf) return LBM_EINVAL;
  return create_solver(p, hip_stream, dev_buf, bytes, true, out);
}

int lbm_step(lbm_solver* s, int64_t nsteps) {
  if (!s || nsteps < 0) return LBM_EINVAL;
  if (s->steps + nsteps > s->p.max_steps) return LBM_ERANGE;
  int64_t k = 0;
  // a coefficient solver whose state was loaded as populations converts it
  // in its first step (another kernel than the steady one)
  if (s->pop_pending && k < nsteps) {
    int rc = step_one(s);
    if (rc) return rc;
    ++k;
  }
  // steady chunks replay one captured graph
  if (nsteps - k >= kGraphSteps && s->graphs_ok && !s->graph && !capture_steps(s))
    s->graphs_ok = false;
  for (; s->graph && k + kGraphSteps <= nsteps; k += kGraphSteps) {
    if (hipGraphLaunch(s->graph, s->stream) != hipSuccess) return LBM_EHIP;
    s->steps += kGraphSteps;
  }
  for (; k < nsteps; ++k) {
    int rc = step_one(s);
    if (rc) return rc;
  }
  return LBM_OK;
}

int lbm_synchronize(lbm_solver* s) {
  if (!s) return LBM_EINVAL;
  return sync_and_check(s);
}

int lbm_representation(const lbm_solver* s, int* repr) {
  if (!s || !repr) return LBM_EINVAL;
  *repr = s->lay.mom ? LBM_REPR_COEFFICIENTS : LBM_REPR_POPULATIONS;
  return LBM_OK;
}

int lbm_steps_done(const lbm_solver* s, int64_t* n) {
  if (!s || !n) return LBM_EINVAL;
  *n = s->steps;
  return LBM_OK;
}

int lbm_force_history(lbm_solver* s, int64_t first, int64_t count, double* fx, double* fy) {
  if (!s || first < 0 || count < 0) return LBM_EINVAL;
  const int64_t cap = s->lay.hist_cap;
  if (first + count > s->steps || first < std::max(s->hist_from, s->steps - std::min(s->steps, cap)))
    return LBM_ERANGE;
  int rc = sync_and_check(s);
  if (rc && rc != LBM_EUNSTABLE) return rc;
  std::vector<double> tmp((size_t)count * 2);
  int64_t done = 0;
  while (done < count) {
    const int64_t h = (first + done) % cap;
    const int64_t run = std::min(count - done, cap - h);
    if (hipMemcpy(tmp.data() + 2 * done, s->desc.hist + 2 * h, sizeof(double) * 2 * run,
                  hipMemcpyDeviceToHost) != hipSuccess)
      return LBM_EHIP;
    done += run;
  }
  for (int64_t i = 0; i < count; ++i) {
    if (fx) fx[i] = tmp[2 * i];
    if (fy) fy[i] = tmp[2 * i + 1];
  }
  return rc;
}

int lbm_lockin(lbm_solver* s, double sums[6], int64_t* nsamples) {
  if (!s || !sums) return LBM_EINVAL;
  int rc = sync_and_check(s);
  if (rc && rc != LBM_EUNSTABLE) return rc;
  SolveState st;
  if (hipMemcpy(&st, s->desc.state, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess)
    return LBM_EHIP;
  for (int k = 0; k < 6; ++k) sums[k] = st.lockin[k];
  if (nsamples)
    *nsamples = std::max<int64_t>(
        0, std::min(s->steps, s->p.lockin_first + s->p.lockin_count) - s->p.lockin_first);
  return rc;
}

int lbm_impedance(lbm_solver* s, double out[5]) {
  if (!s || !out) return LBM_EINVAL;
  double sums[6];
  int64_t ns = 0;
  int rc = lbm_lockin(s, sums, &ns);
  if (rc && rc != LBM_EUNSTABLE) return rc;
  if (ns < 3) return LBM_ERANGE;
  // normal equations of F ~ a sin + b cos + c with the drive table's basis
  long double G[3][4] = {{0}};
  for (int64_t n = s->p.lockin_first; n < s->p.lockin_first + ns; ++n) {
    const double arg = s->p.omega * ((double)n + 0.5);
    const long double b[3] = {std::sin(arg), std::cos(arg), 1.0L};
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) G[r][c] += b[r] * b[c];
  }
  G[0][3] = sums[0];
  G[1][3] = sums[1];
  G[2][3] = sums[2];
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (std::fabs(G[r][c]) > std::fabs(G[piv][c])) piv = r;
    if (G[piv][c] == 0) return LBM_ERANGE;
    for (int k = 0; k < 4; ++k) std::swap(G[c][k], G[piv][k]);
    for (int r = 0; r < 3; ++r) {
      if (r == c) continue;
      const long double m = G[r][c] / G[c][c];
      for (int k = c; k < 4; ++k) G[r][k] -= m * G[c][k];
    }
  }
  const long double a = G[0][3] / G[0][0], b = G[1][3] / G[1][1], c = G[2][3] / G[2][2];
  out[0] = (double)a;
  out[1] = (double)b;
  out[2] = (double)c;
  out[3] = (double)(-a / s->p.u0);
  out[4] = (double)(-b / s->p.u0);
  return rc;
}

namespace {

// Copy the current state out as FP64 [q][y][x] populations; with_rest adds
// w_i rho0.  A coefficient state is expanded to populations
// w_i (a0 + vx bx + vy by + vx^2 cxx + vx vy cxy + vy^2 cyy).
int copy_out(lbm_solver* s, double* host, uint64_t n, bool with_rest) {
  if (!s || !host) return LBM_EINVAL;
  const lbm_params& p = s->p;
  const HostLattice& L = s->lat;
  const int Q = L.Q;
  if (n != (uint64_t)Q * p.ny * p.nx) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  const bool f64 = p.storage == LBM_STORE_F64;
  const bool coeffs = s->lay.mom && !s->pop_pending;
  const uint64_t bytes = coeffs ? s->lay.mbuf_bytes : s->lay.buf_bytes;
  const void* src = coeffs ? s->desc.mbuf[s->steps & 1] : s->bufs[s->steps & 1];
  std::vector<char> stage(bytes);
  if (hipMemcpy(stage.data(), src, bytes, hipMemcpyDeviceToHost) != hipSuccess) return LBM_EHIP;
  auto at = [&](int64_t i) {
    return f64 ? reinterpret_cast<const double*>(stage.data())[i]
               : (double)reinterpret_cast<const float*>(stage.data())[i];
  };
  for (int q = 0; q < Q; ++q) {
    const double w = L.lw.w_orbit[L.orbit[q]];
    const double wr = with_rest ? w * p.rho0 : 0.0;
    const double vx = L.vx[q], vy = L.vy[q];
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        double dv;
        if (coeffs) {
          const int64_t g = y * s->lay.mpitch + x, ks = s->lay.mks;
          dv = w * (at(g) + vx * at(ks + g) + vy * at(2 * ks + g) + vx * vx * at(3 * ks + g) +
                    vx * vy * at(4 * ks + g) + vy * vy * at(5 * ks + g));
        } else {
          dv = at(q * s->lay.qs + y * s->lay.ys + x);
        }
        host[((size_t)q * p.ny + y) * p.nx + x] = in_body(&p, x, y) ? 0.0 : wr + dv;
      }
  }
  return LBM_OK;
}

// Copy FP64 [q][y][x] into the current population buffer; with_rest
// subtracts w_i rho0.  A coefficient solver reads it in its next step.
int copy_in(lbm_solver* s, const double* host, uint64_t n, bool with_rest) {
  if (!s || !host) return LBM_EINVAL;
  const lbm_params& p = s->p;
  const int Q = s->lat.Q;
  if (n != (uint64_t)Q * p.ny * p.nx) return LBM_EINVAL;
  if (!s->lay.loadable) return LBM_EINVAL;  // no population buffer to load into
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  const bool f64 = p.storage == LBM_STORE_F64;
  std::vector<char> stage(s->lay.buf_bytes, 0);
  for (int q = 0; q < Q; ++q) {
    const double wr = with_rest ? s->lat.lw.w_orbit[s->lat.orbit[q]] * p.rho0 : 0.0;
    for (int y = 0; y < p.ny; ++y)
      for (int x = 0; x < p.nx; ++x) {
        const int64_t dst = q * s->lay.qs + y * s->lay.ys + x;
        const double dv = in_body(&p, x, y) ? 0.0 : host[((size_t)q * p.ny + y) * p.nx + x] - wr;
        if (f64) reinterpret_cast<double*>(stage.data())[dst] = dv;
        else reinterpret_cast<float*>(stage.data())[dst] = (float)dv;
      }
  }
  if (hipMemcpy(s->bufs[s->steps & 1], stage.data(), s->lay.buf_bytes,
                hipMemcpyHostToDevice) != hipSuccess)
    return LBM_EHIP;
  if (s->lay.mom) s->pop_pending = true;
  return LBM_OK;
}

// Raw state blob: header, then the current buffer.
struct StateHeader {
  uint32_t magic, lattice, storage, coeffs;
  int32_t nx, ny;
  uint64_t bytes;
};
constexpr uint32_t kStateMagic = 0x4c424d32;  // "LBM2": row-interleaved coefficient buffers

uint64_t state_payload(const lbm_solver* s) {
  return (s->lay.mom && !s->pop_pending) ? s->lay.mbuf_bytes : s->lay.buf_bytes;
}

}  // namespace

int lbm_get_populations(lbm_solver* s, double* host, uint64_t n) {
  return copy_out(s, host, n, true);
}

int lbm_set_populations(lbm_solver* s, const double* host, uint64_t n) {
  return copy_in(s, host, n, true);
}

int lbm_get_deviations(lbm_solver* s, double* host, uint64_t n) {
  return copy_out(s, host, n, false);
}

int lbm_set_deviations(lbm_solver* s, const double* host, uint64_t n) {
  return copy_in(s, host, n, false);
}

int lbm_seek(lbm_solver* s, int64_t step, const double lockin_sums[6]) {
  if (!s || step < 0 || step >= s->p.max_steps) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  if ((step & 1) != (s->steps & 1)) {
    // the current state moves to the buffer that step n reads
    void* const* bufs = s->lay.mom && !s->pop_pending ? s->desc.mbuf : s->bufs;
    if (bufs[step & 1] != bufs[s->steps & 1] &&
        hipMemcpy(bufs[step & 1], bufs[s->steps & 1], state_payload(s),
                  hipMemcpyDeviceToDevice) != hipSuccess)
      return LBM_EHIP;
  }
  SolveState st{};
  st.step = step;
  for (int k = 0; k < 6; ++k) st.lockin[k] = lockin_sums ? lockin_sums[k] : 0.0;
  if (hipMemcpy(s->desc.state, &st, sizeof(st), hipMemcpyHostToDevice) != hipSuccess)
    return LBM_EHIP;
  s->steps = step;
  s->hist_from = step;
  s->sticky_unstable = false;
  return LBM_OK;
}

int lbm_state_size(const lbm_solver* s, uint64_t* bytes) {
  if (!s || !bytes) return LBM_EINVAL;
  *bytes = sizeof(StateHeader) + state_payload(s);
  return LBM_OK;
}

int lbm_get_state(lbm_solver* s, void* host, uint64_t bytes) {
  if (!s || !host) return LBM_EINVAL;
  const uint64_t payload = state_payload(s);
  if (bytes != sizeof(StateHeader) + payload) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  const bool coeffs = s->lay.mom && !s->pop_pending;
  StateHeader h{kStateMagic, s->p.lattice, s->p.storage, coeffs ? 1u : 0u, s->p.nx, s->p.ny,
                payload};
  std::memcpy(host, &h, sizeof(h));
  const void* src = coeffs ? s->desc.mbuf[s->steps & 1] : s->bufs[s->steps & 1];
  if (hipMemcpy(static_cast<char*>(host) + sizeof(h), src, payload, hipMemcpyDeviceToHost) !=
      hipSuccess)
    return LBM_EHIP;
  return LBM_OK;
}

int lbm_set_state(lbm_solver* s, const void* host, uint64_t bytes) {
  if (!s || !host || bytes < sizeof(StateHeader)) return LBM_EINVAL;
  StateHeader h;
  std::memcpy(&h, host, sizeof(h));
  if (h.magic != kStateMagic || h.lattice != s->p.lattice || h.storage != s->p.storage ||
      h.nx != s->p.nx || h.ny != s->p.ny || (h.coeffs && !s->lay.mom) ||
      (!h.coeffs && !s->lay.loadable))
    return LBM_EINVAL;
  const uint64_t payload = h.coeffs ? s->lay.mbuf_bytes : s->lay.buf_bytes;
  if (h.bytes != payload || bytes != sizeof(h) + payload) return LBM_EINVAL;
  if (hipStreamSynchronize(s->stream) != hipSuccess) return LBM_EHIP;
  void* dst = h.coeffs ? s->desc.mbuf[s->steps & 1] : s->bufs[s->steps & 1];
  if (hipMemcpy(dst, static_cast<const char*>(host) + sizeof(h), payload,
                hipMemcpyHostToDevice) != hipSuccess)
    return LBM_EHIP;
  if (s->lay.mom) s->pop_pending = !h.coeffs;
  return LBM_OK;
}

int lbm_destroy(lbm_solver* s) {
  if (!s) return LBM_OK;
  int rc = hipStreamSynchronize(s->stream) == hipSuccess ? LBM_OK : LBM_EHIP;
  if (s->graph) (void)hipGraphExecDestroy(s->graph);
  if (s->owned && hipFree(s->base) != hipSuccess) rc = LBM_EHIP;
  if (s->in_scratch) release_scratch(s->device);
  delete s;
  return rc;
}

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "out of memory or buffer too small";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ERANGE: return "out of range";
    case LBM_EUNSTABLE: return "unstable: non-positive or non-finite density";
    case LBM_EABI: return "ABI version mismatch";
    case LBM_ESCRATCH:
      return "static scratch buffer too small for these parameters, or in use by a live solver";
    default: return "unknown error";
  }
}

}  // extern "C"
