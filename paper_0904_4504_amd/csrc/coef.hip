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
// the population kernel), read from the step's input state.  The finalize
// kernel sums the momentum exchange from the same input state.
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "lattice.hpp"
#include "solver.hpp"
#include "walls.hpp"

namespace lbm {

namespace {

// Index of velocity (vx, vy) in lattice L, or -1.
template <class L>
constexpr int find_q(int vx, int vy) {
  for (int q = 0; q < L::Q; ++q)
    if (L::vx[q] == vx && L::vy[q] == vy) return q;
  return -1;
}

constexpr int pmod(int a, int n) { return ((a % n) + n) % n; }

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
// moving-wall term) and its moments.
template <class L, typename S, bool DSW>
__device__ __forceinline__ Mom<S> add_links(Mom<S> m, const SolveDesc& d, gptr<const S> min,
                                                      int x, int y, S ladd, double U,
                                                      const KernelLattice& lat) {
  const int64_t ks = d.mks;
  const int ys = (int)d.mys;
  const bool is_box = d.geom == GEOM_BOX;
  // diffuse wall: deviation of the mass crossing the wall in column x, from
  // the coefficients of rows 0 .. R-1 (population q at row r crosses when
  // r < -v_qy)
  double cm = 0.0;
  if (DSW && d.wall == WALL_DS && d.geom == GEOM_PLATE && y < L::R) {
    static_for<0, L::R>([&](auto rc) __attribute__((always_inline)) {
      constexpr int r = decltype(rc)::value;
      const int g = r * ys + x;
      const double c0 = min[g], c1 = min[ks + g], c2 = min[2 * ks + g], c3 = min[3 * ks + g],
                   c4 = min[4 * ks + g], c5 = min[5 * ks + g];
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
      const S wq = (S)lat.w[L::orbit[q]];
      S f;
      if (DSW && diffuse) {
        double e = ds_arrival<vx>(d, U, cm, lat.w[L::orbit[q]], lat.theta);
        if (d.sigma != 1.0) {
          // specular share: the population of (vx, -vy) that crossed the
          // wall from column x - vx at the mirror row
          int sxw = x - vx;
          sxw += sxw < 0 ? d.nx : 0;
          sxw -= sxw >= d.nx ? d.nx : 0;
          const int g = py * ys + sxw;
          double p = min[g];
          if constexpr (vx != 0) p += double(vx) * min[ks + g] + double(vx * vx) * min[3 * ks + g];
          if constexpr (vy != 0)
            p += double(-vy) * min[2 * ks + g] + double(vy * vy) * min[5 * ks + g];
          if constexpr (vx * vy != 0) p += double(-vx * vy) * min[4 * ks + g];
          e = d.sigma * e + (1.0 - d.sigma) * lat.w[L::orbit[q]] * p;
        }
        f = (S)e;
      } else {
        const int g = py * ys + px;
        // population of -v at the mirror cell
        S p = min[g];
        if constexpr (vx != 0) p += S(-vx) * min[ks + g] + S(vx * vx) * min[3 * ks + g];
        if constexpr (vy != 0) p += S(-vy) * min[2 * ks + g] + S(vy * vy) * min[5 * ks + g];
        if constexpr (vx * vy != 0) p += S(vx * vy) * min[4 * ks + g];
        f = wq * p;
        if (moving) f += (wq * S(vx)) * ladd;
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
  static constexpr int TH = 4 * RB;  // tile rows
  static constexpr int HW = kCoefTileW + 2 * R, HH = TH + 2 * R, NC = HW * HH;
  static constexpr int NIT = (NC + 255) / 256;  // staged cells per thread
};

// Issue the loads of a tile's staged region (the tile and its R-cell halo)
// into registers: body and outside cells as zeros, periodic images where the
// geometry wraps.  No-op items stage nothing.
template <class L, typename S, int RB>
__device__ __forceinline__ void stage_load(const SolveDesc* __restrict__ descs, WorkItem wi,
                                           S (&c)[CoefTile<L, RB>::NIT][6]) {
  using T = CoefTile<L, RB>;
  constexpr int R = T::R, HW = T::HW, NC = T::NC;
#pragma unroll
  for (int it = 0; it < T::NIT; ++it)
#pragma unroll
    for (int k = 0; k < 6; ++k) c[it][k] = S(0);
  if (wi.tile < 0) return;
  const SolveDesc& d = descs[wi.solve];
  const int64_t n = d.state->step;
  const gptr<const S> min = as_global(static_cast<const S*>(d.mbuf[n & 1]));
  const int nx = d.nx, ny = d.ny;
  const int64_t ks = d.mks;
  const int ys = (int)d.mys;
  gptr<const S> pin[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) pin[k] = scalar_ptr(min + k * ks);
  const int x0 = (wi.tile % d.tiles_x) * kCoefTileW;
  const int y0 = (wi.tile / d.tiles_x) * T::TH;
  const bool xper = d.geom != GEOM_BOX, yper = d.geom == GEOM_PERIODIC;
  const bool is_box = d.geom == GEOM_BOX;
  const int bx0 = d.bx0, bx1 = d.bx1, by0 = d.by0, by1 = d.by1;
  // staged cell i = threadIdx.x + 256 it sits at (hx, hy) of the halo tile;
  // step (hx, hy) instead of dividing per cell
  constexpr int DX = 256 % HW, DY = 256 / HW;
  int hx = (int)threadIdx.x % HW, hy = (int)threadIdx.x / HW;
  // lattices narrower than the staged tile wrap more than once
  const bool narrow = nx < HW || (yper && ny < T::HH);
#pragma unroll
  for (int it = 0; it < T::NIT; ++it) {
    const int i = threadIdx.x + it * 256;
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
    const bool load = i < NC && gx >= 0 && gx < nx && gy >= 0 && gy < ny && !solid;
    // cells without data read cell (0, 0) and are zeroed below
    const int gxc = load ? gx : 0, gyc = load ? gy : 0;
    const uint32_t o = (uint32_t)(gyc * ys + gxc) * (uint32_t)sizeof(S);
#pragma unroll
    for (int k = 0; k < 6; ++k) c[it][k] = *at(pin[k], o);
#pragma unroll
    for (int k = 0; k < 6; ++k) c[it][k] = load ? c[it][k] : S(0);
    hx += DX;
    hy += DY;
    if (hx >= HW) {
      hx -= HW;
      ++hy;
    }
  }
}

// Moments, bounce-back corrections, collision and store of the RB cells of
// this thread, from the staged tile in LDS.
template <class L, typename S, int RB, bool DSW>
__device__ __forceinline__ void compute_tile(const SolveDesc& d, int tile,
                                             const S (&C)[6][CoefTile<L, RB>::NC],
                                             const KernelLattice& lat) {
  using T = CoefTile<L, RB>;
  constexpr int R = T::R, HW = T::HW;
  const int64_t n = d.state->step;
  const gptr<const S> min = as_global(static_cast<const S*>(d.mbuf[n & 1]));
  const gptr<S> mout = as_global(static_cast<S*>(d.mbuf[(n & 1) ^ 1]));
  const int nx = d.nx, ny = d.ny;
  const int64_t ks = d.mks;
  const int ys = (int)d.mys;
  gptr<S> pout[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) pout[k] = scalar_ptr(mout + k * ks);
  const int x0 = (tile % d.tiles_x) * kCoefTileW;
  const int y0 = (tile / d.tiles_x) * T::TH;
  const bool is_box = d.geom == GEOM_BOX;
  const int bx0 = d.bx0, bx1 = d.bx1, by0 = d.by0, by1 = d.by1;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int x = x0 + lane, yb = y0 + wave * RB;
  S wo[L::NORB];
#pragma unroll
  for (int k = 0; k < L::NORB; ++k) wo[k] = (S)lat.w[k];
  // staged cell of the lane's column + dx in the wave's source row iy
  // (iy = -R .. RB - 1 + R relative to the wave's first output row)
  const int cbase = (wave * RB + R) * HW + lane + R;

  Mom<S> acc[RB];
#pragma unroll
  for (int k = 0; k < RB; ++k)
#pragma unroll
    for (int j = 0; j < 6; ++j) acc[k].v[j] = S(0);

  static_for<0, RB + 2 * R>([&](auto ic) __attribute__((always_inline)) {
    constexpr int iy = decltype(ic)::value - R;
    // per output row k (pulling along vy = k - iy): sums of w f, w vx f, w vx^2 f
    S t0[RB], t1[RB], t2[RB];
#pragma unroll
    for (int k = 0; k < RB; ++k) t0[k] = t1[k] = t2[k] = S(0);
    static_for<0, 2 * R + 1>([&](auto dxc) __attribute__((always_inline)) {
      constexpr int dx = decltype(dxc)::value - R;
      constexpr int vx = -dx;  // the source x - v sits at x + dx
      if constexpr (source_used<L, RB>(vx, iy)) {
        const int ci = cbase + iy * HW + dx;
        // coefficients a0, bx, by, cxx, cxy, cyy of the source cell
        S g = C[0][ci];
        if constexpr (vx != 0) g += S(vx) * C[1][ci] + S(vx * vx) * C[3][ci];
        S h = C[2][ci];
        if constexpr (vx != 0) h += S(vx) * C[4][ci];
        const S cyy = C[5][ci];
        static_for<0, RB>([&](auto kc) __attribute__((always_inline)) {
          constexpr int k = decltype(kc)::value;
          constexpr int vy = k - iy;
          if constexpr (vy >= -R && vy <= R && find_q<L>(vx, vy) >= 0) {
            constexpr int q = find_q<L>(vx, vy);
            S f = g;
            if constexpr (vy != 0) f = (g + S(vy * vy) * cyy) + S(vy) * h;
            // integer factors vx, vx^2 become instruction constants; only
            // the NORB weights occupy registers
            const S u = wo[L::orbit[q]] * f;
            t0[k] += u;
            if constexpr (vx != 0) {
              t1[k] += S(vx) * u;
              t2[k] += S(vx * vx) * u;
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
        m.v[0] += t0[k];
        m.v[1] += t1[k];
        m.v[3] += t2[k];
        if constexpr (vy != 0) {
          m.v[2] += S(vy) * t0[k];
          m.v[4] += S(vy) * t1[k];
          m.v[5] += S(vy * vy) * t0[k];
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
  S ladd = S(0);
  if (wave_has_wall) ladd = (S)(d.ladd_scale * d.drive[n].u);

  const S th = (S)lat.theta;
  const S inv_th = (S)(1.0 / lat.theta);
  const S h2 = (S)(0.5 / (lat.theta * lat.theta));
  const S om = (S)d.inv_tau;
  const S rho0 = (S)d.rho0;
#pragma unroll
  for (int k = 0; k < RB; ++k) {
    Mom<S> m = acc[k];
    const int y = yb + k;
    if (y >= ny || x >= nx) continue;
    if (is_box && y >= by0 && y < by1 && x >= bx0 && x < bx1) continue;  // solid
    if (wave_has_wall) {
      const bool near = (y >= wy0 && y < wy1 && x >= wx0 && x < wx1) || (far_band && y >= ny - R);
      if (near) m = add_links<L, S, DSW>(m, d, min, x, y, ladd, d.drive[n].u, lat);
    }
    const S drho = m.v[0], jx = m.v[1], jy = m.v[2];
    const S rho = rho0 + drho;
    S inv_rho;
    if constexpr (sizeof(S) == 4)
      inv_rho = __builtin_amdgcn_rcpf(rho);  // 1 ulp; the FP32 form's error is dominated by storage
    else
      inv_rho = S(1) / rho;
    if (!(rho > S(0) && rho < S(INFINITY))) d.state->unstable = 1;
    const S uxx = jx * jx * inv_rho, uxy = jx * jy * inv_rho, uyy = jy * jy * inv_rho;
    const S axx = m.v[3] - drho * th, ayy = m.v[5] - drho * th, axy = m.v[4];
    const S bxx = axx - om * (axx - uxx);
    const S bxy = axy - om * (axy - uxy);
    const S byy = ayy - om * (ayy - uyy);
    const uint32_t o = (uint32_t)(y * ys + x) * (uint32_t)sizeof(S);
    // the output is not re-read in this step: stream it past the caches
    __builtin_nontemporal_store(drho - (bxx + byy) * (S(0.5) * inv_th), at(pout[0], o));
    __builtin_nontemporal_store(jx * inv_th, at(pout[1], o));
    __builtin_nontemporal_store(jy * inv_th, at(pout[2], o));
    __builtin_nontemporal_store(bxx * h2, at(pout[3], o));
    __builtin_nontemporal_store(bxy * (S(2) * h2), at(pout[4], o));
    __builtin_nontemporal_store(byy * h2, at(pout[5], o));
  }
}

// DSW: with the diffuse-scattering wall (a separate instantiation, so that
// the bounce-back kernel carries none of its code).
template <class L, typename S, int RB, bool DSW>
__global__ __launch_bounds__(256) void coef_kernel(const SolveDesc* __restrict__ descs,
                                                   const WorkItem* __restrict__ work,
                                                   KernelLattice lat) {
  using T = CoefTile<L, RB>;
  // one array per coefficient, so that every LDS read of a coefficient is a
  // 32-bit (64-bit) load at consecutive lanes
  __shared__ S C[6][T::NC];
  const WorkItem wi = work[blockIdx.x];
  if (wi.tile < 0) return;
  // all loads of a thread are issued before the first LDS store, so the
  // block waits for one memory round trip, not one per staged cell
  S c[T::NIT][6];
  stage_load<L, S, RB>(descs, wi, c);
#pragma unroll
  for (int it = 0; it < T::NIT; ++it) {
    const int i = threadIdx.x + it * 256;
    if (i < T::NC)
#pragma unroll
      for (int k = 0; k < 6; ++k) C[k][i] = c[it][k];
  }
  __syncthreads();
  compute_tile<L, S, RB, DSW>(descs[wi.solve], wi.tile, C, lat);
}

template <class L, typename S, int RB>
static hipError_t launch_rb(bool ds, const SolveDesc* descs, const WorkItem* work, int nwork,
                            const KernelLattice& lat, hipStream_t stream) {
  if (ds)
    hipLaunchKernelGGL((coef_kernel<L, S, RB, true>), dim3(nwork), dim3(256), 0, stream, descs,
                       work, lat);
  else
    hipLaunchKernelGGL((coef_kernel<L, S, RB, false>), dim3(nwork), dim3(256), 0, stream, descs,
                       work, lat);
  return hipGetLastError();
}

template <class L, typename S>
static hipError_t launch_coef_t(int k, bool ds, const SolveDesc* descs, const WorkItem* work,
                                int nwork, const KernelLattice& lat, hipStream_t stream) {
  switch (k) {
    case 1:
      return launch_rb<L, S, 1>(ds, descs, work, nwork, lat, stream);
    case 2:
      return launch_rb<L, S, 2>(ds, descs, work, nwork, lat, stream);
    case 3:
      return launch_rb<L, S, 3>(ds, descs, work, nwork, lat, stream);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_coef(int Q, bool f64, int k, bool ds, const SolveDesc* descs,
                       const WorkItem* work, int nwork, const KernelLattice& lat,
                       hipStream_t stream) {
  if (nwork <= 0) return hipSuccess;
  if (Q == 9)
    return f64 ? launch_coef_t<D2Q9, double>(k, ds, descs, work, nwork, lat, stream)
               : launch_coef_t<D2Q9, float>(k, ds, descs, work, nwork, lat, stream);
  return f64 ? launch_coef_t<D2Q37, double>(k, ds, descs, work, nwork, lat, stream)
             : launch_coef_t<D2Q37, float>(k, ds, descs, work, nwork, lat, stream);
}

}  // namespace lbm
