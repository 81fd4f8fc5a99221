// Regularized lattice-BGK step on H2-coefficient storage.
//
// The regularized collision (Sec. 5, eqs. regularization and fne) leaves
// every post-collision distribution in the span of the Hermite polynomials up
// to second order: with deviations from the rest state,
//   delta f_i(x) = w_i [ a0 + vx bx + vy by + vx^2 cxx + vx vy cxy + vy^2 cyy ](x).
// Six coefficients per cell describe the state exactly, so a step reads and
// writes 6 values per cell instead of Q and Q.
//
// A workgroup of four wavefronts updates a tile of 64 columns x 4 RB rows: it
// stages the coefficients of the tile and an R-cell halo in LDS, then the
// lane of column x in wavefront w computes the RB cells (x, w RB + k).  The
// pulled populations f_v(x) = delta f_v(x - v) (eq. advection) of those RB
// cells come from the union of their stencils; the lane reads each cell of
// the union from LDS once and adds its populations to every output cell that
// pulls from it.  For a source cell at column offset dx (so vx = -dx) the
// populations differ only through vy: f = g + vy^2 cyy + vy h with
// g = a0 + vx bx + vx^2 cxx and h = by + vx cxy.  Per output cell and source
// row the sums of w f, w vx f, w vx^2 f are gathered first and then scattered
// into the six moments (rho, j, Pi), which the collision turns into the six
// new coefficients.
//
// Walls (Sec. 4, eq. BB): cells inside the body and outside the domain are
// staged as zeros (the rest-equilibrium far field; the plate's wall
// half-spaces), so a population crossing the moving wall, the body or the
// stationary far wall arrives as zero; the lane of a cell within R of a wall
// then adds the bounce-back value f_opp(x_p) + 2 w_i rho0 (v_i.U_w)/theta
// (moving wall only), x_p the half-way mirror cell of the link (the rules of
// the population kernel), read from the step's input state; at a plate or a
// box face with the diffuse or the Maxwell wall it adds the diffuse emission
// (eq. DS) of the link's wall column, mixed with the specular image for the
// Maxwell wall.  The finalize kernel sums the momentum exchange from the same
// input state.
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "lattice.hpp"
#include "solver.hpp"
#include "walls.hpp"

namespace lbm {

// Constants of a launch in the storage precision: the orbit weights, their
// products with |vx| and vx^2 (the factors of the x-weighted sums; for
// |vx| = 1 the weight itself is used) and the theta factors of the
// coefficients.  Passed by value, so they sit in scalar registers.
template <typename S>
struct CoefConst {
  S w[8];
  S wx[8][4];   // w_o |vx|
  S wxx[8][4];  // w_o vx^2
  S theta;
  S inv_theta;        // 1 / theta
  S half_inv_theta;   // 1 / (2 theta)
  S inv_theta2;       // 1 / theta^2
  S half_inv_theta2;  // 1 / (2 theta^2)
};

template <typename S>
CoefConst<S> coef_const(const KernelLattice& lat) {
  CoefConst<S> c{};
  for (int o = 0; o < 8; ++o) {
    c.w[o] = (S)lat.w[o];
    for (int a = 0; a < 4; ++a) {
      c.wx[o][a] = (S)(lat.w[o] * a);
      c.wxx[o][a] = (S)(lat.w[o] * a * a);
    }
  }
  c.theta = (S)lat.theta;
  c.inv_theta = (S)(1.0 / lat.theta);
  c.half_inv_theta = (S)(0.5 / lat.theta);
  c.inv_theta2 = (S)(1.0 / (lat.theta * lat.theta));
  c.half_inv_theta2 = (S)(0.5 / (lat.theta * lat.theta));
  return c;
}

namespace {

// Index of velocity (vx, vy) in lattice L, or -1.
template <class L>
constexpr int find_q(int vx, int vy) {
  for (int q = 0; q < L::Q; ++q)
    if (L::vx[q] == vx && L::vy[q] == vy) return q;
  return -1;
}

template <typename S>
__device__ __forceinline__ S fmadd(S a, S b, S c) {
  if constexpr (sizeof(S) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

// Pointers into device global memory (loads and stores then address the
// global segment directly, with a scalar base and a 32-bit lane offset).
template <typename T>
using gptr = __attribute__((address_space(1))) T*;

template <typename T>
__device__ __forceinline__ gptr<T> as_global(T* p) {
  return (gptr<T>)p;
}

// A wave-uniform pointer held in scalar registers, so that every load or
// store through it is a scalar base plus a 32-bit per-lane byte offset.
template <typename T>
__device__ __forceinline__ gptr<T> scalar_ptr(gptr<T> p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (gptr<T>)(((uint64_t)hi << 32) | lo);
}

// Address of the element at byte offset `off` of plane `p`.
template <typename T>
__device__ __forceinline__ gptr<T> at(gptr<T> p, uint32_t off) {
  return (gptr<T>)((__attribute__((address_space(1))) char*)p + off);
}

// Two coefficients of a cell: (a0, bx), (by, cxx) or (cxy, cyy).
template <typename S>
using Pair = S __attribute__((ext_vector_type(2)));

template <typename T>
using lptr = __attribute__((address_space(3))) T*;

// The same LDS address, opaque to the compiler: reads relative to it use
// their small constant offsets directly instead of a new base register each.
template <typename T>
__device__ __forceinline__ lptr<const T> opaque(lptr<const T> p) {
  uint32_t a = (uint32_t)(uintptr_t)p;
  asm volatile("" : "+v"(a));
  return (lptr<const T>)(uintptr_t)a;
}

// Six running moment sums of one output row: delta rho, jx, jy, Pxx, Pxy, Pyy.
template <typename S>
struct Mom {
  S v[6];
};


// Empty instruction that takes the six sums as inputs and outputs and
// clobbers memory: the sums of one source row are complete here and the LDS
// reads of the next row are not hoisted above it, so the compiler keeps one
// source row in registers at a time.
template <typename S>
__device__ __forceinline__ void row_fence(Mom<S>& m) {
  asm volatile("" : "+v"(m.v[0]), "+v"(m.v[1]), "+v"(m.v[2]), "+v"(m.v[3]), "+v"(m.v[4]),
                    "+v"(m.v[5])::"memory");
}

// True if a source cell at column offset -vx and row offset iy (relative to
// the first of RB output rows) feeds any of those rows.
template <class L, int RB>
constexpr bool source_used(int vx, int iy) {
  for (int k = 0; k < RB; ++k) {
    const int vy = k - iy;
    if (vy >= -L::R && vy <= L::R && find_q<L>(vx, vy) >= 0) return true;
  }
  return false;
}

// Bounce-back contributions of the wall links of fluid cell (x, y): each link
// population arrived as zero from the stream; add f_opp(x_p) (+ the
// moving-wall term) and its moments.  Every cell a link reads (the mirror
// cell x_p, the diffuse wall's specular source and its crossing rows) lies
// within R - 1 cells of (x, y) along each axis, so inside the staged tile:
// the reads come from LDS (C, staged region starting at cell (ox, oy), rows
// of HW cells), not from global memory.
template <class L, typename S, bool DSW>
__device__ __forceinline__ Mom<S> add_links(Mom<S> m, const SolveDesc& d, const Pair<S>* C,
                                            int HW, int ox, int oy, int x, int y, S ladd,
                                            double U, const KernelLattice& lat,
                                            const CoefConst<S>& cc) {
  const lptr<const Pair<S>> T = (lptr<const Pair<S>>)C;
  // coefficient k (a0, bx, by, cxx, cxy, cyy) of the cell at (cx, cy)
  auto coef = [&](int cx, int cy, int k) __attribute__((always_inline)) -> S {
    const Pair<S> p = T[(3 * (cy - oy) + (k >> 1)) * HW + (cx - ox)];
    return (k & 1) ? p.y : p.x;
  };
  const bool is_box = d.geom == GEOM_BOX;
  // diffuse wall: deviation of the mass crossing the wall in column x, from
  // the coefficients of rows 0 .. R-1 (population q at row r crosses when
  // r < -v_qy)
  double cm = 0.0;
  // box with diffuse or Maxwell faces: the face and column of this arrival
  // cell; the column's crossing mass is linear in the coefficients of its R
  // cells (weights from the host), each within R - 1 cells of this one
  int face = -1, col = 0;
  if (DSW && d.wall == WALL_DS && is_box) {
    face = box_face<L::R>(d, x, y);
    if (face >= 0) {
      col = box_column(d, face, x, y);
      const WallCol& wc = d.wcols[col];
      static_for<0, L::R>([&](auto kc) __attribute__((always_inline)) {
        constexpr int k = decltype(kc)::value;  // the cell k + 1 cells from the face
        const int cx = face == 2 ? d.bx0 - 1 - k : (face == 3 ? d.bx1 + k : x);
        const int cy = face == 0 ? d.by0 - 1 - k : (face == 1 ? d.by1 + k : y);
#pragma unroll
        for (int j = 0; j < 6; ++j) cm += wc.mc[k][j] * (double)coef(cx, cy, j);
      });
    }
  }
  if (DSW && d.wall == WALL_DS && d.geom == GEOM_PLATE && y < L::R) {
    static_for<0, L::R>([&](auto rc) __attribute__((always_inline)) {
      constexpr int r = decltype(rc)::value;
      const double c0 = coef(x, r, 0), c1 = coef(x, r, 1), c2 = coef(x, r, 2),
                   c3 = coef(x, r, 3), c4 = coef(x, r, 4), c5 = coef(x, r, 5);
      static_for<0, L::Q>([&](auto qc) __attribute__((always_inline)) {
        constexpr int q = decltype(qc)::value;
        constexpr int vx = L::vx[q], vy = L::vy[q];
        if constexpr (vy < -r)
          cm += lat.w[L::orbit[q]] *
                (c0 + vx * c1 + vy * c2 + vx * vx * c3 + vx * vy * c4 + vy * vy * c5);
      });
    });
  }
  static_for<0, L::Q>([&](auto qc) __attribute__((always_inline)) {
    constexpr int q = decltype(qc)::value;
    constexpr int vx = L::vx[q], vy = L::vy[q];
    const int sx = x - vx, sy = y - vy;
    int px = -1, py = -1;
    bool moving = false, diffuse = false;
    if (is_box) {
      if (sx >= d.bx0 && sx < d.bx1 && sy >= d.by0 && sy < d.by1) {
        px = x < d.bx0 ? 2 * d.bx0 - 1 - sx : (x >= d.bx1 ? 2 * d.bx1 - 1 - sx : x);
        py = y < d.by0 ? 2 * d.by0 - 1 - sy : (y >= d.by1 ? 2 * d.by1 - 1 - sy : y);
        moving = true;
        diffuse = DSW && face >= 0;  // corner links keep bounce-back
      }
    } else if (d.geom == GEOM_PLATE) {
      if constexpr (vy > 0) {
        if (sy < 0) {
          px = x;
          py = -1 - sy;
          moving = true;
          diffuse = DSW && d.wall == WALL_DS;
        }
      }
      if constexpr (vy < 0) {
        if (sy >= d.ny && d.far == FAR_WALL) {
          px = x;
          py = 2 * d.ny - 1 - sy;
        }
      }
    }
    if (py >= 0) {
      constexpr int o = L::orbit[q];
      const S wq = cc.w[o];
      S f;
      if (DSW && diffuse) {
        const double wd = lat.w[L::orbit[q]];
        double e = is_box ? ds_box_arrival(d.wcols[col], d.rho0, U, cm, wd, double(vx), lat.theta)
                          : ds_arrival<vx>(d, U, cm, wd, lat.theta);
        if (d.sigma != 1.0) {
          double p;
          if (!is_box || face <= 1) {
            // specular share: the population of (vx, -vy) that crossed the
            // wall or face from column x - vx at the mirror row (the staged
            // halo holds the periodic image of a wrapped column)
            const int sxw = x - vx;
            p = coef(sxw, py, 0);
            if constexpr (vx != 0)
              p += double(vx) * coef(sxw, py, 1) + double(vx * vx) * coef(sxw, py, 3);
            if constexpr (vy != 0)
              p += double(-vy) * coef(sxw, py, 2) + double(vy * vy) * coef(sxw, py, 5);
            if constexpr (vx * vy != 0) p += double(-vx * vy) * coef(sxw, py, 4);
            p *= wd;
          } else {
            // a face normal to the motion: the population of (-vx, vy) that
            // crossed it from row y - vy at the mirror column, plus the
            // moving-wall term of the face moving along its normal
            const int syw = y - vy;
            p = coef(px, syw, 0);
            if constexpr (vx != 0)
              p += double(-vx) * coef(px, syw, 1) + double(vx * vx) * coef(px, syw, 3);
            if constexpr (vy != 0)
              p += double(vy) * coef(px, syw, 2) + double(vy * vy) * coef(px, syw, 5);
            if constexpr (vx * vy != 0) p += double(-vx * vy) * coef(px, syw, 4);
            p = wd * p + wd * double(vx) * d.ladd_scale * U;
          }
          e = d.sigma * e + (1.0 - d.sigma) * p;
        }
        f = (S)e;
      } else {
        // population of -v at the mirror cell
        S p = coef(px, py, 0);
        if constexpr (vx != 0) p += S(-vx) * coef(px, py, 1) + S(vx * vx) * coef(px, py, 3);
        if constexpr (vy != 0) p += S(-vy) * coef(px, py, 2) + S(vy * vy) * coef(px, py, 5);
        if constexpr (vx * vy != 0) p += S(vx * vy) * coef(px, py, 4);
        f = wq * p;
        if constexpr (vx != 0) {
          constexpr int a = vx < 0 ? -vx : vx;
          const S wa = a == 1 ? wq : cc.wx[o][a];
          if (moving) f = fmadd(vx < 0 ? -wa : wa, ladd, f);
        }
      }
      m.v[0] += f;
      if constexpr (vx != 0) m.v[1] += S(vx) * f;
      if constexpr (vy != 0) m.v[2] += S(vy) * f;
      if constexpr (vx != 0) m.v[3] += S(vx * vx) * f;
      if constexpr (vx * vy != 0) m.v[4] += S(vx * vy) * f;
      if constexpr (vy != 0) m.v[5] += S(vy * vy) * f;
    }
  });
  return m;
}


}  // namespace

// Tile shape of variant RB (RB cells per thread, four wavefronts).
template <class L, int RB>
struct CoefTile {
  static constexpr int R = L::R;
  static constexpr int NT = 64 * kCoefWaves;  // threads
  static constexpr int TH = kCoefWaves * RB;  // tile rows
  static constexpr int HW = kCoefTileW + 2 * R, HH = TH + 2 * R, NC = HW * HH;
  // staging: the 64 core cells of staged row r (columns R .. R + 63) are
  // loaded by wavefront r mod 4, one cell per lane; the 2R halo cells of
  // every staged row by the first NHALO threads
  static constexpr int NCR = (HH + kCoefWaves - 1) / kCoefWaves;  // core rows per wave
  static constexpr int NHALO = 2 * R * HH;
  static constexpr int NHIT = (NHALO + NT - 1) / NT;  // halo cells per thread
};

// A thread's share of a staged tile between its loads and its LDS writes.
template <class L, typename S, int RB>
struct StageRegs {
  S core[CoefTile<L, RB>::NCR][6];
  S halo[CoefTile<L, RB>::NHIT][6];
};

namespace {

// Raw buffer resource over `bytes` bytes at p (a wave-uniform address):
// loads at offsets past the end return zero.  Word 3 = 0x00020000 sets the
// 32-bit data format (bits 15-18 = 4) with no swizzle or index stride, the
// untyped-access setting of the gfx9 family.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t plane_rsrc(const void* p, uint32_t bytes) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)(((uint64_t)hi << 32) | lo), 0, (int)bytes,
                                           0x00020000);
}

template <typename S>
__device__ __forceinline__ S buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(S) == 4)
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
  else
    return __builtin_bit_cast(S, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}

// Store bypassing the caches' retention (the nontemporal policy bit): a
// separate instruction form from a plain store, which the compiler cannot
// merge with one.
template <typename S>
__device__ __forceinline__ void buf_store_nt(__amdgpu_buffer_rsrc_t r, uint32_t off, S v) {
  if constexpr (sizeof(S) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, 2);
  else
    __builtin_amdgcn_raw_buffer_store_b64(
        __builtin_bit_cast(__attribute__((__vector_size__(2 * sizeof(uint32_t)))) uint32_t, v),
        r, off, 0, 2);
}

// Extent of one coefficient plane's buffer resource: from its first element
// to the last element of its last row.  Element (k, y, x) sits at
// k*ks + y*ys + x: six whole planes (ks >= ny*ys) or, row-interleaved, the
// six rows of a lattice row side by side (ks = row pitch, ys = 6 ks); either
// way plane 5's resource ends inside the buffer.  The library keeps the
// extent below 2 GiB.
template <typename S>
__device__ __forceinline__ uint32_t plane_bytes(int ny, int64_t ys, int64_t ks) {
  return (uint32_t)(((int64_t)(ny - 1) * ys + (ks < ys ? ks : ys)) * (int64_t)sizeof(S));
}

// An offset past the end of every plane's resource (all below 2 GiB).
constexpr uint32_t kNoCell = 0x80000000u;

// Population that output row k pulls from the source cell at column offset
// dx and row offset iy (both relative to the lane's column and the wave's
// first output row), or -1.
template <class L>
constexpr int pull_q(int dx, int iy, int k) {
  const int vy = k - iy;
  if (vy < -L::R || vy > L::R) return -1;
  return find_q<L>(-dx, vy);
}

// First column offset of source row iy that feeds output row k (with
// vx != 0 if nz), or R + 1.
template <class L>
constexpr int first_dx(int iy, int k, bool nz) {
  for (int dx = -L::R; dx <= L::R; ++dx)
    if (pull_q<L>(dx, iy, k) >= 0 && (!nz || dx != 0)) return dx;
  return L::R + 1;
}

}  // namespace

// Read of memory that no thread writes during the launch, through the
// constant address space: a scalar load (no wait on vector memory) for a
// wave-uniform address.
template <typename T>
__device__ __forceinline__ T kread(const T* p) {
  return *(const __attribute__((address_space(4))) T*)p;
}

__device__ __forceinline__ WorkItem kread_item(const WorkItem* p) {
  return WorkItem{kread(&p->solve), kread(&p->tile)};
}

// Step index and state buffers of a solve for this launch.
template <typename S>
struct TileCtx {
  const S* min;  // input coefficients
  S* mout;       // output coefficients
  int64_t n;     // step index
};

template <typename S>
__device__ __forceinline__ TileCtx<S> tile_ctx(const SolveDesc& d) {
  const int64_t n = kread(&d.state->step);
  void* const b0 = kread(&d.mbuf[0]);
  void* const b1 = kread(&d.mbuf[1]);
  return {static_cast<const S*>(n & 1 ? b1 : b0), static_cast<S*>(n & 1 ? b0 : b1), n};
}

// Load a tile's staged region (the tile and its R-cell halo) into registers:
// body and outside cells as zeros, periodic images where the geometry wraps.
// Each core load of a wavefront covers 64 consecutive cells of one row of one
// coefficient, starting at a multiple of 64 cells: a tile's loads touch whole
// aligned segments, and only the 2R halo cells per row come in separately
// (a 70-cell row loaded lane by lane straddles rows at unaligned starts:
// 11 % slower on the memory side of a state streaming from HBM).
template <class L, typename S, int RB>
__device__ __forceinline__ void stage_load(const SolveDesc& d, const TileCtx<S>& t, int tile,
                                           StageRegs<L, S, RB>& g, int tid) {
  using T = CoefTile<L, RB>;
  constexpr int R = T::R, HH = T::HH;
  constexpr uint32_t es = sizeof(S);
  const S* min = t.min;
  const int nx = d.nx, ny = d.ny;
  const int64_t ks = d.mks;
  const int ys = (int)d.mys;
  const uint32_t bytes = plane_bytes<S>(ny, ys, ks);
  __amdgpu_buffer_rsrc_t rs[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) rs[k] = plane_rsrc(min + k * ks, bytes);
  const int x0 = (tile % d.tiles_x) * kCoefTileW;
  const int y0 = (tile / d.tiles_x) * T::TH;
  const int lane = tid & 63, wv = tid >> 6;
  const bool xper = d.geom != GEOM_BOX, yper = d.geom == GEOM_PERIODIC;
  const bool is_box = d.geom == GEOM_BOX;
  const int bx0 = d.bx0, bx1 = d.bx1, by0 = d.by0, by1 = d.by1;
  // byte offsets first, then the loads (one code path, so the wait before
  // each use covers exactly the loads it needs)
  uint32_t oc[T::NCR], oh[T::NHIT];
  // a staged region inside the lattice, clear of the body: every cell is
  // read as is
  const bool inside = x0 >= R && x0 + kCoefTileW + R <= nx && y0 >= R && y0 + T::TH + R <= ny &&
                      !(is_box && x0 - R < bx1 && x0 + kCoefTileW + R > bx0 && y0 - R < by1 &&
                        y0 + T::TH + R > by0);
  if (inside) {
    uint32_t o = (uint32_t)((y0 - R + wv) * ys + x0 + lane) * es;
    const uint32_t step = (uint32_t)(kCoefWaves * ys) * es;
#pragma unroll
    for (int m = 0; m < T::NCR; ++m) {
      // rows past the region (wave-uniform) read nothing and are not written
      oc[m] = wv + kCoefWaves * m < HH ? o : kNoCell;
      o += step;
    }
#pragma unroll
    for (int it = 0; it < T::NHIT; ++it) {
      const int i = tid + it * T::NT, j = i % (2 * R), hy = i / (2 * R);
      const int hx = j < R ? j : kCoefTileW + j;
      oh[it] = i < T::NHALO ? (uint32_t)((y0 - R + hy) * ys + x0 - R + hx) * es : kNoCell;
    }
  } else {
    // lattices narrower than the staged tile wrap more than once
    const bool narrow = nx < T::HW || (yper && ny < HH);
    auto offset = [&](int hx, int hy) -> uint32_t {
      int gx = x0 - R + hx, gy = y0 - R + hy;
      if (xper) {
        gx += gx < 0 ? nx : 0;
        gx -= gx >= nx ? nx : 0;
      }
      if (yper) {
        gy += gy < 0 ? ny : 0;
        gy -= gy >= ny ? ny : 0;
      }
      if (__builtin_expect(narrow, 0)) {
        if (xper) gx = (((x0 - R + hx) % nx) + nx) % nx;
        if (yper) gy = (((y0 - R + hy) % ny) + ny) % ny;
      }
      const bool solid = is_box && gx >= bx0 && gx < bx1 && gy >= by0 && gy < by1;
      const bool load = gx >= 0 && gx < nx && gy >= 0 && gy < ny && !solid;
      // cells without data read past the end of the plane: zeros
      return load ? (uint32_t)(gy * ys + gx) * es : kNoCell;
    };
#pragma unroll
    for (int m = 0; m < T::NCR; ++m) {
      const int hy = wv + kCoefWaves * m;
      oc[m] = hy < HH ? offset(R + lane, hy) : kNoCell;
    }
#pragma unroll
    for (int it = 0; it < T::NHIT; ++it) {
      const int i = tid + it * T::NT, j = i % (2 * R), hy = i / (2 * R);
      oh[it] = i < T::NHALO ? offset(j < R ? j : kCoefTileW + j, hy) : kNoCell;
    }
  }
#pragma unroll
  for (int m = 0; m < T::NCR; ++m)
#pragma unroll
    for (int k = 0; k < 6; ++k) g.core[m][k] = buf_load<S>(rs[k], oc[m]);
#pragma unroll
  for (int it = 0; it < T::NHIT; ++it)
#pragma unroll
    for (int k = 0; k < 6; ++k) g.halo[it][k] = buf_load<S>(rs[k], oh[it]);
}

// Moments, bounce-back corrections and collision of the RB cells of this
// thread, from the staged tile in LDS (staged row r holds the pairs
// (a0, bx), (by, cxx), (cxy, cyy) of its HW cells as three runs of HW): the
// new coefficients of the cells in the lattice and the fluid go to res.  U:
// the wall drive U_w of the step.
template <class L, typename S, int RB, bool DSW>
__device__ __forceinline__ void compute_tile(const SolveDesc& d, const TileCtx<S>& t, int tile,
                                             const Pair<S>* C, const KernelLattice& lat,
                                             const CoefConst<S>& cc, int tid,
                                             S (&res)[RB][6], uint32_t& valid, double U) {
  using T = CoefTile<L, RB>;
  constexpr int R = T::R, HW = T::HW;
  const int nx = d.nx, ny = d.ny;
  const int x0 = (tile % d.tiles_x) * kCoefTileW;
  const int y0 = (tile / d.tiles_x) * T::TH;
  const bool is_box = d.geom == GEOM_BOX;
  const int bx0 = d.bx0, bx1 = d.bx1, by0 = d.by0, by1 = d.by1;

  const int lane = tid & 63, wave = tid >> 6;
  const int x = x0 + lane, yb = y0 + wave * RB;

  Mom<S> acc[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k)
#pragma unroll
    for (int j = 0; j < 6; ++j) acc[k].v[j] = S(0);

  static_for<0, RB + 2 * R>([&](auto ic) __attribute__((always_inline)) {
    constexpr int iy = decltype(ic)::value - R;
    // staged row of source row iy, from the cell at column offset -R
    const lptr<const Pair<S>> row =
        opaque((lptr<const Pair<S>>)(C + (wave * RB + R + iy) * 3 * HW + lane));
    // per output row k (pulling along vy = k - iy): sums of w f, w vx f, w vx^2 f
    S t0[RB], t1[RB], t2[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) t0[k] = t1[k] = t2[k] = S(0);
    static_for<0, 2 * R + 1>([&](auto dxc) __attribute__((always_inline)) {
      constexpr int dx = decltype(dxc)::value - R;
      constexpr int vx = -dx;  // the source x - v sits at x + dx
      if constexpr (source_used<L, RB>(vx, iy)) {
        const Pair<S> p0 = row[dx + R], p1 = row[HW + dx + R], p2 = row[2 * HW + dx + R];
        // populations of the source cell along vx: f = g + vy^2 cyy + vy h
        S g = p0.x, h = p1.x;
        if constexpr (vx != 0) {
          g = fmadd(S(vx * vx), p1.y, fmadd(S(vx), p0.y, g));
          h = fmadd(S(vx), p2.x, h);
        }
        const S cyy = p2.y;
        static_for<0, RB>([&](auto kc) __attribute__((always_inline)) {
          constexpr int k = decltype(kc)::value;
          constexpr int vy = k - iy;
          constexpr int q = pull_q<L>(dx, iy, k);
          if constexpr (q >= 0) {
            constexpr int o = L::orbit[q];
            S f = g;
            if constexpr (vy != 0) f = fmadd(S(vy), h, fmadd(S(vy * vy), cyy, g));
            const S w = cc.w[o];
            if constexpr (dx == first_dx<L>(iy, k, false))
              t0[k] = w * f;
            else
              t0[k] = fmadd(w, f, t0[k]);
            if constexpr (vx != 0) {
              constexpr int a = vx < 0 ? -vx : vx;
              const S wa = a == 1 ? w : cc.wx[o][a];
              const S wb = a == 1 ? w : cc.wxx[o][a];
              const S wsx = vx < 0 ? -wa : wa;
              if constexpr (dx == first_dx<L>(iy, k, true)) {
                t1[k] = wsx * f;
                t2[k] = wb * f;
              } else {
                t1[k] = fmadd(wsx, f, t1[k]);
                t2[k] = fmadd(wb, f, t2[k]);
              }
            }
          }
        });
      }
    });
    static_for<0, RB>([&](auto kc) __attribute__((always_inline)) {
      constexpr int k = decltype(kc)::value;
      constexpr int vy = k - iy;
      if constexpr (vy >= -R && vy <= R) {
        Mom<S>& m = acc[k];
        if constexpr (iy == k - R) {
          // first source row of output row k
          m.v[0] = t0[k];
          m.v[1] = t1[k];
          m.v[3] = t2[k];
          m.v[2] = S(vy) * t0[k];
          m.v[4] = S(vy) * t1[k];
          m.v[5] = S(vy * vy) * t0[k];
        } else {
          m.v[0] += t0[k];
          m.v[1] += t1[k];
          m.v[3] += t2[k];
          if constexpr (vy != 0) {
            m.v[2] = fmadd(S(vy), t0[k], m.v[2]);
            m.v[4] = fmadd(S(vy), t1[k], m.v[4]);
            m.v[5] = fmadd(S(vy * vy), t0[k], m.v[5]);
          }
        }
      }
    });
#pragma unroll
    for (int k = 0; k < RB; ++k) row_fence(acc[k]);
  });

  // wall band of the tile (uniform): rows and columns whose cells may have a link
  int wx0 = 0, wx1 = nx, wy0 = 0, wy1 = 0;
  if (is_box) {
    wx0 = bx0 - R;
    wx1 = bx1 + R;
    wy0 = by0 - R;
    wy1 = by1 + R;
  } else if (d.geom == GEOM_PLATE) {
    wy1 = R;  // moving wall below row 0
  }
  const bool far_band = d.geom == GEOM_PLATE && d.far == FAR_WALL;
  const bool wave_has_wall = (x0 < wx1 && x0 + kCoefTileW > wx0 && yb < wy1 && yb + RB > wy0) ||
                             (far_band && yb + RB > ny - R);

  const S th = cc.theta;
  const S inv_th = cc.inv_theta;
  const S h2 = cc.half_inv_theta2;
  const S om = (S)d.inv_tau;
  const S rho0 = (S)d.rho0;
  // Every lane runs the collision of all its rows: cells outside the lattice
  // or inside the body see only staged zeros and finite sums, and their
  // results are dropped by the store (bit k of `valid`), so no lane leaves
  // the straight-line code.
  bool bad = false;
  // (a compile-time loop: unrolled whatever the size of the wall code)
  static_for<0, RB>([&](auto kc) __attribute__((always_inline)) {
    constexpr int k = decltype(kc)::value;
    Mom<S> m = acc[k];
    const int y = yb + k;
    const bool in = y < ny && x < nx && !(is_box && y >= by0 && y < by1 && x >= bx0 && x < bx1);
    valid |= in ? 1u << k : 0u;
    if (wave_has_wall) {
      const bool near =
          in && ((y >= wy0 && y < wy1 && x >= wx0 && x < wx1) || (far_band && y >= ny - R));
      if (near) {
        S ladd = (S)(d.ladd_scale * U);
        // computed per cell in the band: keeps its products out of the common path
        asm volatile("" : "+v"(ladd));
        m = add_links<L, S, DSW>(m, d, C, HW, x0 - R, y0 - R, x, y, ladd, U, lat, cc);
      }
    }
    const S drho = m.v[0], jx = m.v[1], jy = m.v[2];
    const S rho = rho0 + drho;
    S inv_rho;
    if constexpr (sizeof(S) == 4)
      inv_rho = __builtin_amdgcn_rcpf(rho);  // 1 ulp; the FP32 form's error is dominated by storage
    else
      inv_rho = S(1) / rho;
    bad |= in && !(rho > S(0) && rho < S(INFINITY));
    const S uxx = jx * jx * inv_rho, uxy = jx * jy * inv_rho, uyy = jy * jy * inv_rho;
    const S axx = m.v[3] - drho * th, ayy = m.v[5] - drho * th, axy = m.v[4];
    const S bxx = axx - om * (axx - uxx);
    const S bxy = axy - om * (axy - uxy);
    const S byy = ayy - om * (ayy - uyy);
    res[k][0] = drho - (bxx + byy) * cc.half_inv_theta;
    res[k][1] = jx * inv_th;
    res[k][2] = jy * inv_th;
    res[k][3] = bxx * h2;
    res[k][4] = bxy * cc.inv_theta2;
    res[k][5] = byy * h2;
  });
  if (bad) d.state->unstable = 1;
}

// Store the new coefficients of this thread's cells (those in the lattice
// and the fluid: bit k of `valid` for row k).
template <class L, typename S, int RB>
__device__ __forceinline__ void store_tile(const SolveDesc& d, const TileCtx<S>& t, int tile,
                                           int tid, const S (&res)[RB][6], uint32_t valid,
                                           bool streaming) {
  using T = CoefTile<L, RB>;
  const gptr<S> mout = as_global(t.mout);
  const int64_t ks = d.mks;
  const int ys = (int)d.mys;
  gptr<S> pout[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) pout[k] = scalar_ptr(mout + k * ks);
  // the same planes as buffer resources, for the nontemporal stores
  const uint32_t bytes = plane_bytes<S>(d.ny, ys, ks);
  __amdgpu_buffer_rsrc_t ro[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) ro[k] = plane_rsrc(t.mout + k * ks, bytes);
  const int x = (tile % d.tiles_x) * kCoefTileW + (tid & 63);
  const int yb = (tile / d.tiles_x) * T::TH + (tid >> 6) * RB;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    if (!(valid & (1u << k))) continue;
    const int y = yb + k;
    const uint32_t o = (uint32_t)(y * ys + x) * (uint32_t)sizeof(S);
    // a state that stays in the last-level cache between steps is stored
    // through it (the next step reads it back from there: 36.7 against
    // 43.3 us per beam-box launch); a state streaming from HBM bypasses it
    // (2.84 against 3.03 ms per launch of the 256-solve batch)
    if (streaming) {
#pragma unroll
      for (int j = 0; j < 6; ++j) buf_store_nt(ro[j], o, res[k][j]);
    } else {
#pragma unroll
      for (int j = 0; j < 6; ++j) *at(pout[j], o) = res[k][j];
    }
  }
}

// Write a loaded tile (stage_load) to LDS.
template <class L, typename S, int RB>
__device__ __forceinline__ void stage_store(Pair<S>* C, const StageRegs<L, S, RB>& g, int tid) {
  using T = CoefTile<L, RB>;
  constexpr int R = T::R, HW = T::HW;
  const int lane = tid & 63, wv = tid >> 6;
#pragma unroll
  for (int m = 0; m < T::NCR; ++m) {
    const int hy = wv + kCoefWaves * m;
    if (hy < T::HH)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        C[(hy * 3 + j) * HW + R + lane] = Pair<S>{g.core[m][2 * j], g.core[m][2 * j + 1]};
  }
#pragma unroll
  for (int it = 0; it < T::NHIT; ++it) {
    const int i = tid + it * T::NT, jj = i % (2 * R), hy = i / (2 * R);
    const int hx = jj < R ? jj : kCoefTileW + jj;
    if (i < T::NHALO)
#pragma unroll
      for (int j = 0; j < 3; ++j)
        C[(hy * 3 + j) * HW + hx] = Pair<S>{g.halo[it][2 * j], g.halo[it][2 * j + 1]};
  }
}

// DSW: with the diffuse-scattering wall (a separate instantiation, so that
// the bounce-back kernel carries none of its code).  One workgroup per work
// item.
template <class L, typename S, int RB, bool DSW>
__global__ __launch_bounds__(64 * kCoefWaves) void coef_kernel(const SolveDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ work,
                                                   KernelLattice lat, CoefConst<S> cc,
                                                   int streaming) {
  using T = CoefTile<L, RB>;
  // staged row r, pair j, column c at C[(3 r + j) HW + c]: the reads of a
  // pair are 64-bit (128-bit) loads at consecutive lanes
  __shared__ Pair<S> C[T::HH * 3 * T::HW];
  const WorkItem wi = kread_item(&work[blockIdx.x]);
  if (wi.tile < 0) return;
  const SolveDesc& d = descs[wi.solve];
  const TileCtx<S> ctx = tile_ctx<S>(d);
  // wall drive of the step (for the links): a new table entry every step, so
  // a cache miss; a vector load issued before the staging loads hides it
  // behind them (a scalar load would share its counter with the LDS reads)
  int nv = (int)ctx.n;
  asm volatile("" : "+v"(nv));
  const double U = as_global(d.drive)[nv].u;
  const int tid = (int)threadIdx.x;
  {
    // all loads of a thread are issued before the first LDS store, so the
    // block waits for one memory round trip, not one per staged cell
    StageRegs<L, S, RB> g;
    stage_load<L, S, RB>(d, ctx, wi.tile, g, tid);
    stage_store<L, S, RB>(C, g, tid);
  }
  __syncthreads();
  S res[RB][6];
  uint32_t valid = 0;
  compute_tile<L, S, RB, DSW>(d, ctx, wi.tile, C, lat, cc, tid, res, valid, U);
  store_tile<L, S, RB>(d, ctx, wi.tile, tid, res, valid, streaming != 0);
}

template <class L, typename S, int RB>
static hipError_t launch_rb(bool ds, bool streaming, const SolveDesc* descs, const WorkItem* work,
                            int nwork, const KernelLattice& lat, hipStream_t stream,
                            const KernelEvents& ev) {
  const CoefConst<S> cc = coef_const<S>(lat);
  const dim3 grid(nwork), block(64 * kCoefWaves);
  const int st = streaming ? 1 : 0;
  if (ds)
    launch_kernel(coef_kernel<L, S, RB, true>, grid, block, stream, ev, descs, work, lat, cc, st);
  else
    launch_kernel(coef_kernel<L, S, RB, false>, grid, block, stream, ev, descs, work, lat, cc, st);
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t launch_coef_t(int k, bool ds, bool streaming, const SolveDesc* descs,
                                const WorkItem* work, int nwork, const KernelLattice& lat,
                                hipStream_t stream, const KernelEvents& ev) {
  switch (k) {
    case 1:
      return launch_rb<L, S, 1>(ds, streaming, descs, work, nwork, lat, stream, ev);
    case 2:
      return launch_rb<L, S, 2>(ds, streaming, descs, work, nwork, lat, stream, ev);
    case 3:
      return launch_rb<L, S, 3>(ds, streaming, descs, work, nwork, lat, stream, ev);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_coef(int Q, bool f64, int k, bool ds, bool streaming, const SolveDesc* descs,
                       const WorkItem* work, int nwork, const KernelLattice& lat,
                       hipStream_t stream, KernelEvents ev) {
  if (nwork <= 0) return hipSuccess;
  if (Q == 9)
    return f64 ? launch_coef_t<D2Q9, double>(k, ds, streaming, descs, work, nwork, lat, stream,
                                             ev)
               : launch_coef_t<D2Q9, float>(k, ds, streaming, descs, work, nwork, lat, stream,
                                            ev);
  return f64 ? launch_coef_t<D2Q37, double>(k, ds, streaming, descs, work, nwork, lat, stream, ev)
             : launch_coef_t<D2Q37, float>(k, ds, streaming, descs, work, nwork, lat, stream, ev);
}

}  // namespace lbm
