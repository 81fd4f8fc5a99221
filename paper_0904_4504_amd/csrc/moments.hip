// Regularized lattice-BGK step on H2-coefficient storage.
//
// The regularized collision (Sec. 5, eqs. regularization and fne) leaves
// every post-collision distribution in the span of the Hermite polynomials up
// to second order: with deviations from the rest state,
//   delta f_i(x) = w_i [ a0 + vx bx + vy by + vx^2 cxx + vx vy cxy + vy^2 cyy ](x).
// Six coefficients per cell therefore describe the state exactly, and a step
// needs 6 values read and 6 written per cell instead of Q and Q.  Each
// workgroup stages the coefficients of its 64 x 8 tile plus an R-cell halo in
// LDS, rebuilds the Q pulled populations f_i^adv(x) = f_i(x - v_i) (eq.
// advection) from the neighbours' coefficients, takes their moments, applies
// the collision and writes the cell's six new coefficients.
//
// Walls: cells within R of a bounce-back wall or of the body rebuild each
// crossing population from the mirror cell's coefficients in the opposite
// direction plus the moving-wall term 2 w_i rho0 (v_i.U_w)/theta (Sec. 4,
// eq. BB; the same half-way mirror rules as the population kernel); the
// finalize kernel sums the momentum exchange from the same input state.  Outside the domain the staged
// coefficients are periodic images (x for plates, x and y for periodic
// domains) or zero, i.e. the rest-equilibrium far field.
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "lattice.hpp"
#include "solver.hpp"

namespace lbm {

template <typename S>
struct Vec;
template <>
struct Vec<float> {
  using v4 = float4;
  using v2 = float2;
};
template <>
struct Vec<double> {
  using v4 = double4;
  using v2 = double2;
};

// Population of direction (vx, vy) (times 1/w) from the coefficients a = (a0,
// bx, by, cxx), b = (cxy, cyy); SIGN = -1 gives the opposite direction.
template <int vx, int vy, int SIGN, class V4, class V2, typename S>
__device__ __forceinline__ S poly(const V4& a, const V2& b) {
  S p = a.x;
  if constexpr (vx != 0) p += S(SIGN * vx) * a.y + S(vx * vx) * a.w;
  if constexpr (vy != 0) p += S(SIGN * vy) * a.z + S(vy * vy) * b.y;
  if constexpr (vx * vy != 0) p += S(vx * vy) * b.x;
  return p;
}

// EDGE = false: tiles in which no cell has a bounce-back link (the host
// classifies tiles); no wall code, no force.  EDGE = true: the other tiles.
template <class L, typename S, bool EDGE>
__global__ __launch_bounds__(kBlock) void moment_kernel(const SolveDesc* __restrict__ descs,
                                                        const WorkItem* __restrict__ work,
                                                        KernelLattice lat) {
  constexpr int Q = L::Q, R = L::R;
  constexpr int HW = kMomTileW + 2 * R, HH = kMomTileH + 2 * R, NC = HW * HH;
  constexpr int ROWS = kMomTileH / (kBlock / 64);  // rows per thread
  using V4 = typename Vec<S>::v4;
  using V2 = typename Vec<S>::v2;
  __shared__ V4 A[NC];
  __shared__ V2 B[NC];

  const WorkItem wi = work[blockIdx.x];
  if (wi.tile < 0) return;
  const SolveDesc& d = descs[wi.solve];
  const int64_t n = d.state->step;
  const S* __restrict__ min = static_cast<const S*>(d.mbuf[n & 1]);
  S* __restrict__ mout = static_cast<S*>(d.mbuf[(n & 1) ^ 1]);
  const int nx = d.nx, ny = d.ny;
  const int64_t ks = d.mks, ys = d.mys;
  const int x0 = (wi.tile % d.tiles_x) * kMomTileW;
  const int y0 = (wi.tile / d.tiles_x) * kMomTileH;
  const bool xper = d.geom != GEOM_BOX, yper = d.geom == GEOM_PERIODIC;

  // stage the tile and its halo
  for (int i = threadIdx.x; i < NC; i += kBlock) {
    const int hx = i % HW, hy = i / HW;
    int gx = x0 - R + hx, gy = y0 - R + hy;
    if (xper) {
      gx += gx < 0 ? nx : 0;
      gx -= gx >= nx ? nx : 0;
    }
    if (yper) {
      gy += gy < 0 ? ny : 0;
      gy -= gy >= ny ? ny : 0;
    }
    V4 a{S(0), S(0), S(0), S(0)};
    V2 b{S(0), S(0)};
    if (gx >= 0 && gx < nx && gy >= 0 && gy < ny) {
      const int64_t g = (int64_t)gy * ys + gx;
      a = V4{min[g], min[ks + g], min[2 * ks + g], min[3 * ks + g]};
      b = V2{min[4 * ks + g], min[5 * ks + g]};
    }
    A[i] = a;
    B[i] = b;
  }
  __syncthreads();

  const S th = (S)lat.theta;
  const S inv_th = (S)(1.0 / lat.theta);
  const S h2 = (S)(0.5 / (lat.theta * lat.theta));
  const S om = (S)d.inv_tau;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const bool is_box = d.geom == GEOM_BOX;

#pragma unroll
  for (int r = 0; r < ROWS; ++r) {
    const int ly = wave * ROWS + r;
    const int x = x0 + lane, y = y0 + ly;
    if (x >= nx || y >= ny) continue;
    const int ci = (ly + R) * HW + lane + R;
    bool edge = false;
    if constexpr (EDGE) {
      if (is_box && x >= d.bx0 && x < d.bx1 && y >= d.by0 && y < d.by1) continue;
      if (is_box)
        edge = x >= d.bx0 - R && x < d.bx1 + R && y >= d.by0 - R && y < d.by1 + R;
      else if (d.geom == GEOM_PLATE)
        edge = y < R || (d.far == FAR_WALL && y >= ny - R);
    }

    S drho = 0, jx = 0, jy = 0, pxx = 0, pxy = 0, pyy = 0;
    auto accumulate = [&](auto qc, S f) {
      constexpr int q = decltype(qc)::value;
      constexpr int vx = L::vx[q], vy = L::vy[q];
      drho += f;
      if constexpr (vx != 0) jx += S(vx) * f;
      if constexpr (vy != 0) jy += S(vy) * f;
      if constexpr (vx != 0) pxx += S(vx * vx) * f;
      if constexpr (vx * vy != 0) pxy += S(vx * vy) * f;
      if constexpr (vy != 0) pyy += S(vy * vy) * f;
    };
    if (!edge) {
      static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int vx = L::vx[q], vy = L::vy[q];
        constexpr int off = vy * HW + vx;
        const S f = (S)lat.w[L::orbit[q]] * poly<vx, vy, 1, V4, V2, S>(A[ci - off], B[ci - off]);
        accumulate(qc, f);
      });
    } else if constexpr (EDGE) {
      const double ladd = d.ladd_scale * d.drive[n].u;
      static_for<0, Q>([&](auto qc) {
        constexpr int q = decltype(qc)::value;
        constexpr int vx = L::vx[q], vy = L::vy[q];
        constexpr int off = vy * HW + vx;
        const double wq = lat.w[L::orbit[q]];
        const int sx = x - vx, sy = y - vy;
        // mirror cell of a bounce-back link (-1: not a link); `moving` adds
        // the wall term (the force is summed by the finalize kernel)
        int px = -1, py = -1;
        bool moving = false;
        if (is_box) {
          if (sx >= d.bx0 && sx < d.bx1 && sy >= d.by0 && sy < d.by1) {
            px = x < d.bx0 ? 2 * d.bx0 - 1 - sx : (x >= d.bx1 ? 2 * d.bx1 - 1 - sx : x);
            py = y < d.by0 ? 2 * d.by0 - 1 - sy : (y >= d.by1 ? 2 * d.by1 - 1 - sy : y);
            moving = true;
          }
        } else {
          if constexpr (vy > 0) {
            if (sy < 0) {
              px = x;
              py = -1 - sy;
              moving = true;
            }
          }
          if constexpr (vy < 0) {
            if (sy >= ny && d.far == FAR_WALL) {
              px = x;
              py = 2 * ny - 1 - sy;
            }
          }
        }
        S f;
        if (py >= 0) {
          const int cm = (py - y0 + R) * HW + (px - x0 + R);
          const S fr = (S)wq * poly<vx, vy, -1, V4, V2, S>(A[cm], B[cm]);
          f = moving ? fr + (S)(wq * vx * ladd) : fr;
        } else {
          f = (S)wq * poly<vx, vy, 1, V4, V2, S>(A[ci - off], B[ci - off]);
        }
        accumulate(qc, f);
      });
    }

    const S rho = (S)d.rho0 + drho;
    const S inv_rho = S(1) / rho;
    if (!(rho > S(0) && rho < S(INFINITY))) d.state->unstable = 1;
    const S uxx = jx * jx * inv_rho, uxy = jx * jy * inv_rho, uyy = jy * jy * inv_rho;
    const S axx = pxx - drho * th, ayy = pyy - drho * th, axy = pxy;
    const S bxx = axx - om * (axx - uxx);
    const S bxy = axy - om * (axy - uxy);
    const S byy = ayy - om * (ayy - uyy);
    const int64_t g = (int64_t)y * ys + x;
    // the output is not re-read in this step: stream it past the caches
    __builtin_nontemporal_store(drho - (bxx + byy) * (S(0.5) * inv_th), &mout[g]);
    __builtin_nontemporal_store(jx * inv_th, &mout[ks + g]);
    __builtin_nontemporal_store(jy * inv_th, &mout[2 * ks + g]);
    __builtin_nontemporal_store(bxx * h2, &mout[3 * ks + g]);
    __builtin_nontemporal_store(bxy * (S(2) * h2), &mout[4 * ks + g]);
    __builtin_nontemporal_store(byy * h2, &mout[5 * ks + g]);
  }

}

template <class L, typename S>
static hipError_t launch_moment_t(bool edge, const SolveDesc* descs, const WorkItem* work,
                                  int nwork, const KernelLattice& lat, hipStream_t stream) {
  if (edge)
    hipLaunchKernelGGL((moment_kernel<L, S, true>), dim3(nwork), dim3(kBlock), 0, stream, descs,
                       work, lat);
  else
    hipLaunchKernelGGL((moment_kernel<L, S, false>), dim3(nwork), dim3(kBlock), 0, stream, descs,
                       work, lat);
  return hipGetLastError();
}

hipError_t launch_moment(int Q, bool f64, bool edge, const SolveDesc* descs, const WorkItem* work,
                         int nwork, const KernelLattice& lat, hipStream_t stream) {
  if (nwork <= 0) return hipSuccess;
  if (Q == 9)
    return f64 ? launch_moment_t<D2Q9, double>(edge, descs, work, nwork, lat, stream)
               : launch_moment_t<D2Q9, float>(edge, descs, work, nwork, lat, stream);
  return f64 ? launch_moment_t<D2Q37, double>(edge, descs, work, nwork, lat, stream)
             : launch_moment_t<D2Q37, float>(edge, descs, work, nwork, lat, stream);
}

}  // namespace lbm
