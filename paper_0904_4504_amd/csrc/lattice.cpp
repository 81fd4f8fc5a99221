// Host-side derivation of the quadrature weights of the velocity sets.
//
// The paper prints the D2Q37 weights to about 15-16 significant digits
// (appendix table) together with the lattice speed c = 1.19697977039307
// sqrt(theta).  Those digits are too few for an FP64 path that must agree
// with a long-double reference to 1e-12, so the weights are re-derived from
// what defines them: a square-symmetric rule of algebraic degree 9 reproduces
// the Gaussian moments sum_i w_i vx^p vy^q = (p-1)!!(q-1)!! theta^((p+q)/2)
// for every even p, q with p + q <= 8 (Sec. 5: a rule of degree d integrates
// the moments exactly).  Nine conditions, eight orbit weights and theta.
//
// Method (long double): for a trial theta the eight conditions other than
// the pure degree-8 one (p, q) = (8, 0) are linear in the orbit weights and
// are solved by Gaussian elimination (condition number about 2e4); theta is
// the root of the remaining condition, found by the secant method from
// theta = 1/c^2.  (The eight conditions without the mixed (4, 4) one are
// singular, so that one cannot be the left-out condition.)
#include "lattice.hpp"

#include <cmath>

namespace lbm {
namespace {

long double dfact(int n) {
  long double r = 1;
  for (; n > 1; n -= 2) r *= n;
  return r;
}

long double ipow(int v, int p) {
  long double r = 1;
  for (int k = 0; k < p; ++k) r *= v;
  return r;
}

// Orbit moment sums  M[k](p, q) = sum over the members of orbit k of vx^p vy^q.
template <class L>
long double orbit_moment(int k, int p, int q) {
  long double s = 0;
  for (int i = 0; i < L::Q; ++i)
    if (L::orbit[i] == k) s += ipow(L::vx[i], p) * ipow(L::vy[i], q);
  return s;
}

// The first eight enter the linear solve; the last one fixes theta.
constexpr int kPowers[9][2] = {{0, 0}, {2, 0}, {4, 0}, {2, 2}, {6, 0},
                               {4, 2}, {6, 2}, {4, 4}, {8, 0}};

// Solve the 8 linear conditions (all but the last power) for the orbit
// weights at a given theta; returns the residual of the last condition.
bool weights_at(long double theta, long double w[8], long double* resid) {
  long double A[8][9];
  for (int r = 0; r < 8; ++r) {
    const int p = kPowers[r][0], q = kPowers[r][1];
    for (int k = 0; k < 8; ++k) A[r][k] = orbit_moment<D2Q37>(k, p, q);
    A[r][8] = dfact(p - 1) * dfact(q - 1) * std::pow(theta, (long double)((p + q) / 2));
  }
  for (int c = 0; c < 8; ++c) {
    int piv = c;
    for (int r = c + 1; r < 8; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    if (A[piv][c] == 0) return false;
    if (piv != c)
      for (int k = 0; k < 9; ++k) {
        long double t = A[c][k];
        A[c][k] = A[piv][k];
        A[piv][k] = t;
      }
    for (int r = c + 1; r < 8; ++r) {
      long double m = A[r][c] / A[c][c];
      for (int k = c; k < 9; ++k) A[r][k] -= m * A[c][k];
    }
  }
  for (int r = 7; r >= 0; --r) {
    long double s = A[r][8];
    for (int k = r + 1; k < 8; ++k) s -= A[r][k] * w[k];
    w[r] = s / A[r][r];
  }
  long double m = 0;
  for (int k = 0; k < 8; ++k) m += w[k] * orbit_moment<D2Q37>(k, 8, 0);
  *resid = m - dfact(7) * std::pow(theta, 4.0L);
  return true;
}

bool solve_d2q37(long double w[8], long double* theta_out) {
  const long double c = 1.19697977039307L;  // appendix table footnote
  long double t0 = 1.0L / (c * c), t1 = t0 * (1.0L + 1e-9L);
  long double r0, r1;
  if (!weights_at(t0, w, &r0) || !weights_at(t1, w, &r1)) return false;
  for (int it = 0; it < 60 && r1 != r0; ++it) {
    long double t2 = t1 - r1 * (t1 - t0) / (r1 - r0);
    t0 = t1;
    r0 = r1;
    t1 = t2;
    if (!weights_at(t1, w, &r1)) return false;
    if (std::fabs(t1 - t0) <= 1e-19L * t1) break;
  }
  *theta_out = t1;
  return weights_at(t1, w, &r1);
}

}  // namespace

bool lattice_weights(int Q, LatticeWeights* out) {
  if (Q == 9) {
    out->Q = 9;
    out->norb = D2Q9::NORB;
    const long double w[3] = {4.0L / 9.0L, 1.0L / 9.0L, 1.0L / 36.0L};
    for (int k = 0; k < 8; ++k) out->w_orbit_ld[k] = k < 3 ? w[k] : 0.0L;
    out->theta_ld = 1.0L / 3.0L;
  } else if (Q == 37) {
    out->Q = 37;
    out->norb = D2Q37::NORB;
    if (!solve_d2q37(out->w_orbit_ld, &out->theta_ld)) return false;
  } else {
    return false;
  }
  for (int k = 0; k < 8; ++k) out->w_orbit[k] = (double)out->w_orbit_ld[k];
  out->theta = (double)out->theta_ld;
  return true;
}

}  // namespace lbm
