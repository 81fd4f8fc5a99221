// Discrete velocity sets of the solver (compile-time abscissae) and the
// host-side derivation of their quadrature weights.
//
// D2Q37: the Gauss-Hermite velocity set of the paper's appendix table
// ("Model Parameters D2Q37"): orbits (0,0), (1,0), (1,1), (2,0), (2,2),
// (3,0), (1,2), (1,3) in lattice units (lattice speed c = 1, so
// theta = 1/c^2).  D2Q9: the textbook degree-5 rule (not in the paper).
//
// Canonical order (used for every population exchanged through the C ABI):
// orbits in table order; inside an orbit, members by polar angle in [0, 2pi).
#pragma once

namespace lbm {

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int R = 1;        // longest link along one axis
  static constexpr int NORB = 3;
  static constexpr int vx[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
  static constexpr int vy[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
  static constexpr int orbit[Q] = {0, 1, 1, 1, 1, 2, 2, 2, 2};
};

struct D2Q37 {
  static constexpr int Q = 37;
  static constexpr int R = 3;
  static constexpr int NORB = 8;
  static constexpr int vx[Q] = {0,                                        // (0,0)
                                1, 0, -1, 0,                              // (1,0)
                                1, -1, -1, 1,                             // (1,1)
                                2, 0, -2, 0,                              // (2,0)
                                2, -2, -2, 2,                             // (2,2)
                                3, 0, -3, 0,                              // (3,0)
                                2, 1, -1, -2, -2, -1, 1, 2,               // (1,2)
                                3, 1, -1, -3, -3, -1, 1, 3};              // (1,3)
  static constexpr int vy[Q] = {0,
                                0, 1, 0, -1,
                                1, 1, -1, -1,
                                0, 2, 0, -2,
                                2, 2, -2, -2,
                                0, 3, 0, -3,
                                1, 2, 2, 1, -1, -2, -2, -1,
                                1, 3, 3, 1, -1, -3, -3, -1};
  static constexpr int orbit[Q] = {0, 1, 1, 1, 1, 2, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5,
                                   5, 5, 6, 6, 6, 6, 6, 6, 6, 6, 7, 7, 7, 7, 7, 7, 7, 7};
};

// Index of the opposite velocity (v_opp = -v), evaluated at compile time.
template <class L>
constexpr int opposite(int i) {
  for (int j = 0; j < L::Q; ++j)
    if (L::vx[j] == -L::vx[i] && L::vy[j] == -L::vy[i]) return j;
  return -1;
}

// Index of the specular image (vx, -vy), evaluated at compile time.
template <class L>
constexpr int reflect_y(int i) {
  for (int j = 0; j < L::Q; ++j)
    if (L::vx[j] == L::vx[i] && L::vy[j] == -L::vy[i]) return j;
  return -1;
}

// Index of the specular image in x, (-vx, vy), evaluated at compile time.
template <class L>
constexpr int reflect_x(int i) {
  for (int j = 0; j < L::Q; ++j)
    if (L::vx[j] == -L::vx[i] && L::vy[j] == L::vy[i]) return j;
  return -1;
}

// Quadrature weights per orbit and theta, derived on the host.
struct LatticeWeights {
  int Q;
  int norb;
  double w_orbit[8];
  double theta;
  long double w_orbit_ld[8];
  long double theta_ld;
};

// Fills `out` for Q = 9 or 37; returns false for any other Q or if the
// moment system cannot be solved.
bool lattice_weights(int Q, LatticeWeights* out);

}  // namespace lbm
