/*
 * CPU oracle for the oscillating-body lattice-BGK problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg load this library.  It shares no code, header, table or
 * helper with the HIP library; the lattice constants come from its own
 * generator (gen_constants.py -> lattice_constants.h).
 *
 * Plain and slow on purpose: one loop over cells and directions per step,
 * full populations f (not deviations), every formula written as the paper
 * states it.  Compiled twice, with ORACLE_REAL = double and with
 * ORACLE_REAL = long double, so the oracle's own rounding floor can be
 * measured.  OpenMP only splits the row loop; the force is summed over rows
 * afterwards in a fixed order, so results do not depend on the thread count.
 *
 * Method (Sec. 5, eqs. LBGK, feq_h2, MME_lbgk, advection, regularization,
 * fne; Sec. 4 eq. BB; Sec. 6 moving-wall drive):
 *   advection   f_i^adv(x) = f_i(x - v_i)                       (eq. advection)
 *   moments     rho = sum f, rho u = sum f v                      (eq. MME_lbgk)
 *   equilibrium f_i^eq = w_i rho [1 + v.u/th + (v.u)^2/2th^2 - u^2/2th]  (eq. feq_h2)
 *   non-eq.     fne_i = w_i/(2 th^2)(v_a v_b - th d_ab) sum_j (f_j^adv - f_j^eq) v_ja v_jb
 *   collision   f_i(x + v_i, t + 1) = f_i^eq + (1 - 1/tau) fne_i  (eq. regularization)
 * Readings where the paper is silent (each is listed in the design notes):
 *   - tau is the relaxation time of the discrete update (viscosity
 *     nu = theta (tau - 1/2)); tau = +inf is allowed (pure streaming in BGK mode).
 *   - One step = pull advection then collision; the initial array is the
 *     post-collision state at t = 0.  Step n uses the wall velocity
 *     U_w = u0 sin(omega (n + 1/2)) and its force is stamped at t = n + 1/2.
 *   - Bounce-back (eq. BB, linearised): a population arriving at x whose
 *     source lies in the wall takes the opposite population from the mirror
 *     point x_p plus 2 w_i rho0 (v_i . U_w)/theta.  The wall is half-way
 *     between nodes.  Plate: wall at y = -1/2, x_p = (x, v_iy - 1 - y).
 *     Box: per axis, if the arrival coordinate lies outside the body's range
 *     the source coordinate is mirrored through that face plane, otherwise
 *     the arrival coordinate is kept (corners: both axes mirrored).
 *   - Force on the body (momentum exchange) F = -sum_links v_i (f_opp(x_p) + f_i^adv(x)).
 *   - Far field: stationary half-way bounce-back at y = ny - 1/2 (plate), or
 *     rest-equilibrium ghost populations w_i rho0 outside the domain.
 *   - Diffuse scattering (eq. DS) at the plate: a population arriving from the
 *     wall in column x is the H2 equilibrium at the wall velocity and the wall
 *     density rho_w(x); rho_w(x) balances the mass of the populations of
 *     column x that cross the wall in this step (zero normal mass flux, eq.
 *     kinetic_bc), the crossing links counted as in bounce-back.
 *   - Maxwell wall of accommodation sigma (Sec. 3, sigma_v): the arrival is
 *     sigma times the diffuse one plus (1 - sigma) times the specular image:
 *     the population of (vx, -vy) that crossed the wall from column x - vx
 *     at the mirror row (reflected in y only; its tangential velocity, and
 *     so the wall's tangential motion, does not enter).
 *   - Diffuse and Maxwell walls on the box: a link belongs to the face on
 *     whose axis its arrival cell lies outside the body's range (a corner
 *     link, outside on both axes, keeps bounce-back).  A face is cut into
 *     columns, one per arrival coordinate along it.  The diffuse wall emits
 *     into every link of a column the H2 equilibrium at the wall velocity
 *     times the column's wall density, which returns to the fluid the mass
 *     bounce-back would return through those links (the crossing mass, plus
 *     on the faces normal to the motion the mass the moving face displaces;
 *     on a plate this is the zero-normal-flux rule above).  The specular
 *     image is the population that left the source point reflected through
 *     the face plane, with the velocity's normal component reversed; on the
 *     faces normal to the motion it carries the moving-wall term.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "lattice_constants.h"

#ifndef ORACLE_REAL
#define ORACLE_REAL double
#endif
typedef ORACLE_REAL real;

#define ORC_MAXQ 37

enum { ORC_GEOM_PLATE = 0, ORC_GEOM_BOX = 1, ORC_GEOM_PERIODIC = 2 };
enum { ORC_FAR_WALL = 0, ORC_FAR_EQ = 1 };
enum { ORC_COLL_REGULARIZED = 0, ORC_COLL_BGK = 1 };
enum { ORC_WALL_BB = 0, ORC_WALL_DS = 1, ORC_WALL_MAXWELL = 2 };

typedef struct {
  int Q;          /* 9 or 37 */
  int geometry;   /* ORC_GEOM_* */
  int far;        /* ORC_FAR_* (plate only; the box always uses ORC_FAR_EQ) */
  int collision;  /* ORC_COLL_* */
  int nx, ny;     /* fluid domain; plate and periodic: x periodic */
  int box_x0, box_y0, box_lx, box_ly; /* box: solid cells [x0,x0+lx) x [y0,y0+ly) */
  double tau;     /* lattice relaxation time, > 1/2, may be +inf */
  double omega;   /* drive angular frequency, rad per step */
  double u0;      /* drive amplitude: U_w(t) = u0 sin(omega t) along x */
  double rho0;    /* rest density */
  int nthreads;   /* OpenMP threads, 0 = runtime default */
  int wall;       /* ORC_WALL_*: model of the moving wall or body (plate or box) */
  double sigma;   /* MAXWELL: tangential momentum accommodation, 0 (specular) .. 1 (DS) */
} oracle_params;

typedef struct {
  int Q;
  int vx[ORC_MAXQ], vy[ORC_MAXQ], opp[ORC_MAXQ];
  int refl[ORC_MAXQ];  /* index of (vx, -vy): the specular image in y */
  int reflx[ORC_MAXQ]; /* index of (-vx, vy): the specular image in x */
  real w[ORC_MAXQ];
  real theta;
} lattice;

static int load_lattice(int Q, lattice* L) {
  const int(*v)[2];
  const long double* w;
  long double th;
  if (Q == 9) {
    v = ORC_Q9_V; w = ORC_Q9_W; th = ORC_Q9_THETA;
  } else if (Q == 37) {
    v = ORC_Q37_V; w = ORC_Q37_W; th = ORC_Q37_THETA;
  } else {
    return -1;
  }
  L->Q = Q;
  L->theta = (real)th;
  for (int i = 0; i < Q; ++i) {
    L->vx[i] = v[i][0];
    L->vy[i] = v[i][1];
    L->w[i] = (real)w[i];
  }
  for (int i = 0; i < Q; ++i) {
    L->opp[i] = -1;
    for (int j = 0; j < Q; ++j)
      if (v[j][0] == -v[i][0] && v[j][1] == -v[i][1]) L->opp[i] = j;
    if (L->opp[i] < 0) return -1;
    L->refl[i] = -1;
    L->reflx[i] = -1;
    for (int j = 0; j < Q; ++j) {
      if (v[j][0] == v[i][0] && v[j][1] == -v[i][1]) L->refl[i] = j;
      if (v[j][0] == -v[i][0] && v[j][1] == v[i][1]) L->reflx[i] = j;
    }
    if (L->refl[i] < 0 || L->reflx[i] < 0) return -1;
  }
  return 0;
}

static int vmax_of(const lattice* L) {
  int m = 0;
  for (int i = 0; i < L->Q; ++i) {
    if (abs(L->vx[i]) > m) m = abs(L->vx[i]);
    if (abs(L->vy[i]) > m) m = abs(L->vy[i]);
  }
  return m;
}

static int wrap(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

static int in_body(const oracle_params* p, int x, int y) {
  return p->geometry == ORC_GEOM_BOX && x >= p->box_x0 && x < p->box_x0 + p->box_lx &&
         y >= p->box_y0 && y < p->box_y0 + p->box_ly;
}

static int check_params(const oracle_params* p, const lattice* L) {
  const int m = vmax_of(L);
  if (p->nx < 1 || p->ny < 1) return -1;
  if (!(p->tau > 0.5)) return -1;
  if (p->geometry == ORC_GEOM_BOX) {
    if (p->box_lx < m || p->box_ly < m) return -1;
    if (p->box_x0 < m || p->box_y0 < m) return -1;
    if (p->box_x0 + p->box_lx + m > p->nx || p->box_y0 + p->box_ly + m > p->ny) return -1;
  } else if (p->geometry == ORC_GEOM_PLATE) {
    if (p->ny < m) return -1;
  } else if (p->geometry != ORC_GEOM_PERIODIC) {
    return -1;
  }
  const int walled = p->geometry == ORC_GEOM_PLATE || p->geometry == ORC_GEOM_BOX;
  if (p->wall == ORC_WALL_DS) return walled ? 0 : -1;
  if (p->wall == ORC_WALL_MAXWELL) return walled && p->sigma >= 0 && p->sigma <= 1 ? 0 : -1;
  return p->wall == ORC_WALL_BB ? 0 : -1;
}

/* Cell-major storage of the oracle's own: f[(y*nx + x)*Q + i]. */
#define F_AT(f, x, y, i) ((f)[((size_t)(y) * p->nx + (x)) * L->Q + (i)])
#define G_AT(f, x, y, i) ((f)[((size_t)(y) * p->nx + (x)) * L.Q + (i)])

/* Advection of one population into fluid cell (x, y) along direction i
 * (eq. advection with the boundary rules above).  Adds the momentum-exchange
 * contribution of a moving-wall link to (*fx, *fy). */
/* H2 equilibrium factor of direction i at velocity (U, 0), eq. feq_h2 / (w_i rho). */
static real eq_factor(const lattice* L, int i, real U) {
  const real vu = L->vx[i] * U, th = L->theta;
  return 1 + vu / th + vu * vu / (2 * th * th) - U * U / (2 * th);
}

/* Diffuse-scattering wall density of every plate column: mass of the
 * populations crossing the wall at y = -1/2 over the mass the wall emits per
 * unit density, rho_w(x) = sum_cross f / sum_{v_y>0} v_y w eq_factor. */
static void wall_density(const oracle_params* p, const lattice* L, const real* f, real U,
                         real* rho_w) {
  real emit = 0;
  for (int i = 0; i < L->Q; ++i)
    if (L->vy[i] > 0) emit += L->vy[i] * L->w[i] * eq_factor(L, i, U);
  for (int x = 0; x < p->nx; ++x) {
    real m = 0;
    for (int i = 0; i < L->Q; ++i)
      for (int r = 0; r < -L->vy[i]; ++r) m += F_AT(f, x, r, i);
    rho_w[x] = m / emit;
  }
}

/* Face of a box link by its arrival cell (x, y): 0 below the body, 1 above,
 * 2 left of it, 3 right of it; -1 for a corner link.  Column of the link on
 * its face: faces 0, 1 by x, faces 2, 3 by y, numbered face after face. */
static int box_face(const oracle_params* p, int x, int y) {
  const int x0 = p->box_x0, x1 = p->box_x0 + p->box_lx;
  const int y0 = p->box_y0, y1 = p->box_y0 + p->box_ly;
  const int inx = x >= x0 && x < x1, iny = y >= y0 && y < y1;
  if (inx && !iny) return y < y0 ? 0 : 1;
  if (iny && !inx) return x < x0 ? 2 : 3;
  return -1;
}

static int box_column(const oracle_params* p, int face, int x, int y) {
  const int lx = p->box_lx, ly = p->box_ly;
  switch (face) {
    case 0: return x - p->box_x0;
    case 1: return lx + x - p->box_x0;
    case 2: return 2 * lx + y - p->box_y0;
    default: return 2 * lx + ly + y - p->box_y0;
  }
}

/* Bounce-back mirror cell of the box link arriving at (x, y) from source
 * (sx, sy) in the body: per axis, through the face plane when the arrival
 * lies outside the body's range on that axis, else the arrival coordinate. */
static void box_mirror(const oracle_params* p, int x, int y, int sx, int sy, int* px, int* py) {
  const int x0 = p->box_x0, x1 = p->box_x0 + p->box_lx;
  const int y0 = p->box_y0, y1 = p->box_y0 + p->box_ly;
  *px = x < x0 ? 2 * x0 - 1 - sx : (x >= x1 ? 2 * x1 - 1 - sx : x);
  *py = y < y0 ? 2 * y0 - 1 - sy : (y >= y1 ? 2 * y1 - 1 - sy : y);
}

/* Wall density of every face column of the box: the mass bounce-back would
 * deliver through the column's links (each reflected population plus its
 * moving-wall term) over the mass the wall emits per unit density through
 * them, sum over the links of w_i times the equilibrium factor. */
static void box_wall_density(const oracle_params* p, const lattice* L, const real* f, real U,
                             real* rho_w) {
  const int m = vmax_of(L);
  const int ncol = 2 * (p->box_lx + p->box_ly);
  real* num = (real*)calloc((size_t)ncol, sizeof(real));
  real* den = (real*)calloc((size_t)ncol, sizeof(real));
  for (int y = p->box_y0 - m; y < p->box_y0 + p->box_ly + m; ++y)
    for (int x = p->box_x0 - m; x < p->box_x0 + p->box_lx + m; ++x) {
      if (in_body(p, x, y)) continue;
      const int face = box_face(p, x, y);
      if (face < 0) continue;
      const int c = box_column(p, face, x, y);
      for (int i = 0; i < L->Q; ++i) {
        const int sx = x - L->vx[i], sy = y - L->vy[i];
        if (!in_body(p, sx, sy)) continue;
        int px, py;
        box_mirror(p, x, y, sx, sy, &px, &py);
        num[c] += F_AT(f, px, py, L->opp[i]) + 2 * L->w[i] * (real)p->rho0 * (L->vx[i] * U) / L->theta;
        den[c] += L->w[i] * eq_factor(L, i, U);
      }
    }
  for (int c = 0; c < ncol; ++c) rho_w[c] = den[c] != 0 ? num[c] / den[c] : 0;
  free(num);
  free(den);
}

static real advect_one(const oracle_params* p, const lattice* L, const real* f, int x, int y,
                       int i, real U, const real* rho_w, real* fx, real* fy) {
  const int vx = L->vx[i], vy = L->vy[i];
  int sx = x - vx, sy = y - vy;
  const real rest = L->w[i] * (real)p->rho0;
  if (p->geometry == ORC_GEOM_PERIODIC) {
    return F_AT(f, wrap(sx, p->nx), wrap(sy, p->ny), i);
  }
  if (p->geometry == ORC_GEOM_PLATE) {
    sx = wrap(sx, p->nx);
    if (sy < 0) {
      /* crossed the moving wall at y = -1/2: retrace in y, keep x */
      int py = -1 - sy;
      real fr = F_AT(f, x, py, L->opp[i]);
      real fa;
      if (!rho_w) {
        fa = fr + 2 * L->w[i] * (real)p->rho0 * (vx * U) / L->theta;
      } else {
        fa = L->w[i] * rho_w[x] * eq_factor(L, i, U);
        if (p->wall == ORC_WALL_MAXWELL) {
          /* specular part: the population of (vx, -vy) that left column
             x - vx at the mirror row and is reflected in y only */
          const real sp = F_AT(f, sx, py, L->refl[i]);
          fa = (real)p->sigma * fa + (1 - (real)p->sigma) * sp;
        }
      }
      *fx -= vx * (fr + fa);
      *fy -= vy * (fr + fa);
      return fa;
    }
    if (sy >= p->ny) {
      if (p->far == ORC_FAR_EQ) return rest;
      /* stationary half-way wall at y = ny - 1/2 */
      int py = 2 * p->ny - 1 - sy;
      return F_AT(f, x, py, L->opp[i]);
    }
    return F_AT(f, sx, sy, i);
  }
  /* box inside a rest-equilibrium far field */
  if (sx < 0 || sx >= p->nx || sy < 0 || sy >= p->ny) return rest;
  if (in_body(p, sx, sy)) {
    int px, py;
    box_mirror(p, x, y, sx, sy, &px, &py);
    const real fr = F_AT(f, px, py, L->opp[i]);
    const real ladd = 2 * L->w[i] * (real)p->rho0 * (vx * U) / L->theta;
    const int face = box_face(p, x, y);
    real fa;
    if (!rho_w || face < 0) {
      fa = fr + ladd; /* bounce-back wall, or a corner link */
    } else {
      fa = L->w[i] * rho_w[box_column(p, face, x, y)] * eq_factor(L, i, U);
      if (p->wall == ORC_WALL_MAXWELL) {
        /* specular part: the population that left the source point
           reflected through the face plane, normal velocity reversed; the
           faces normal to the motion add the moving-wall term */
        real sp;
        if (face <= 1)
          sp = F_AT(f, sx, py, L->refl[i]);
        else
          sp = F_AT(f, px, sy, L->reflx[i]) + ladd;
        fa = (real)p->sigma * fa + (1 - (real)p->sigma) * sp;
      }
    }
    *fx -= vx * (fr + fa);
    *fy -= vy * (fr + fa);
    return fa;
  }
  return F_AT(f, sx, sy, i);
}

/* Equilibrium, eq. feq_h2. */
static void equilibrium(const lattice* L, real rho, real ux, real uy, real* feq) {
  const real th = L->theta;
  for (int i = 0; i < L->Q; ++i) {
    real vu = L->vx[i] * ux + L->vy[i] * uy;
    real uu = ux * ux + uy * uy;
    feq[i] = L->w[i] * rho * (1 + vu / th + vu * vu / (2 * th * th) - uu / (2 * th));
  }
}

/* One collision of the populations of a cell (eqs. MME_lbgk, feq_h2,
 * regularization and fne, or plain BGK). */
static void collide(const lattice* L, int collision, real inv_tau, const real* fa, real* fout) {
  const int Q = L->Q;
  const real th = L->theta;
  real rho = 0, jx = 0, jy = 0;
  for (int i = 0; i < Q; ++i) {
    rho += fa[i];
    jx += fa[i] * L->vx[i];
    jy += fa[i] * L->vy[i];
  }
  real ux = jx / rho, uy = jy / rho;
  real feq[ORC_MAXQ];
  equilibrium(L, rho, ux, uy, feq);
  const real keep = 1 - inv_tau;
  if (collision == ORC_COLL_BGK) {
    for (int i = 0; i < Q; ++i) fout[i] = feq[i] + keep * (fa[i] - feq[i]);
    return;
  }
  real axx = 0, axy = 0, ayy = 0;
  for (int j = 0; j < Q; ++j) {
    real d = fa[j] - feq[j];
    axx += d * L->vx[j] * L->vx[j];
    axy += d * L->vx[j] * L->vy[j];
    ayy += d * L->vy[j] * L->vy[j];
  }
  for (int i = 0; i < Q; ++i) {
    real hxx = L->vx[i] * L->vx[i] - th;
    real hxy = (real)(L->vx[i] * L->vy[i]);
    real hyy = L->vy[i] * L->vy[i] - th;
    /* the sum over alpha, beta counts the off-diagonal pair twice */
    real fne = L->w[i] / (2 * th * th) * (hxx * axx + 2 * hxy * axy + hyy * ayy);
    fout[i] = feq[i] + keep * fne;
  }
}

static real inv_tau_of(double tau) { return isinf(tau) ? (real)0 : 1 / (real)tau; }

/* ---------------------------------------------------------------- exports */

/* Lattice tables in canonical order.  Returns 0 or -1 for an unknown Q. */
int oracle_lattice(int Q, int* vx, int* vy, double* w, double* theta) {
  lattice L;
  if (load_lattice(Q, &L)) return -1;
  for (int i = 0; i < Q; ++i) {
    vx[i] = L.vx[i];
    vy[i] = L.vy[i];
    w[i] = (double)L.w[i];
  }
  *theta = (double)L.theta;
  return 0;
}

/* Equilibrium populations for (rho, ux, uy). */
int oracle_equilibrium(int Q, double rho, double ux, double uy, double* feq) {
  lattice L;
  real out[ORC_MAXQ];
  if (load_lattice(Q, &L)) return -1;
  equilibrium(&L, rho, ux, uy, out);
  for (int i = 0; i < Q; ++i) feq[i] = (double)out[i];
  return 0;
}

/* Collision of one cell: fin -> fout (both length Q, canonical order). */
int oracle_collide(int Q, int collision, double tau, const double* fin, double* fout) {
  lattice L;
  real a[ORC_MAXQ] = {0}, b[ORC_MAXQ] = {0};
  if (load_lattice(Q, &L)) return -1;
  for (int i = 0; i < Q; ++i) a[i] = fin[i];
  collide(&L, collision, inv_tau_of(tau), a, b);
  for (int i = 0; i < Q; ++i) fout[i] = (double)b[i];
  return 0;
}

/* Columns of the diffuse / Maxwell wall: the plate's nx, the box's perimeter. */
static int wall_columns(const oracle_params* p) {
  return p->geometry == ORC_GEOM_BOX ? 2 * (p->box_lx + p->box_ly) : p->nx;
}

static real* import_f(const oracle_params* p, const lattice* L, const double* f0) {
  size_t n = (size_t)p->nx * p->ny * L->Q;
  real* f = (real*)malloc(n * sizeof(real));
  if (!f) return NULL;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x)
      for (int i = 0; i < L->Q; ++i) {
        real v;
        if (in_body(p, x, y)) v = 0;
        else if (f0) v = f0[((size_t)i * p->ny + y) * p->nx + x];
        else v = L->w[i] * (real)p->rho0;
        F_AT(f, x, y, i) = v;
      }
  return f;
}

static void export_f(const oracle_params* p, const lattice* L, const real* f, double* out) {
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x)
      for (int i = 0; i < L->Q; ++i)
        out[((size_t)i * p->ny + y) * p->nx + x] = in_body(p, x, y) ? 0.0 : (double)F_AT(f, x, y, i);
}

/* Advection only (no collision) with wall velocity U: f (layout [q][y][x])
 * -> fadv (same layout).  Solid cells of fadv are 0.  fx, fy receive the
 * momentum-exchange force of the moving wall / body. */
int oracle_advect(const oracle_params* p, const double* f_in, double U, double* f_adv, double* fx,
                  double* fy) {
  lattice L;
  if (load_lattice(p->Q, &L) || check_params(p, &L)) return -1;
  real* f = import_f(p, &L, f_in);
  if (!f) return -2;
  real* rho_w = NULL;
  if (p->wall == ORC_WALL_DS || p->wall == ORC_WALL_MAXWELL) {
    rho_w = (real*)malloc(sizeof(real) * (size_t)wall_columns(p));
    if (!rho_w) { free(f); return -2; }
    if (p->geometry == ORC_GEOM_BOX) box_wall_density(p, &L, f, (real)U, rho_w);
    else wall_density(p, &L, f, (real)U, rho_w);
  }
  real Fx = 0, Fy = 0;
  for (int y = 0; y < p->ny; ++y)
    for (int x = 0; x < p->nx; ++x)
      for (int i = 0; i < L.Q; ++i) {
        size_t o = ((size_t)i * p->ny + y) * p->nx + x;
        if (in_body(p, x, y)) {
          f_adv[o] = 0;
          continue;
        }
        f_adv[o] = (double)advect_one(p, &L, f, x, y, i, (real)U, rho_w, &Fx, &Fy);
      }
  *fx = (double)Fx;
  *fy = (double)Fy;
  free(f);
  free(rho_w);
  return 0;
}

/* Run nsteps steps from f0 (layout [q][y][x]; NULL = rest state w_i rho0).
 * fx[n], fy[n] receive the force on the moving wall / body at t = n + 1/2
 * (either may be NULL).  f_final (may be NULL) receives the final state. */
int oracle_run(const oracle_params* p, const double* f0, long nsteps, double* fx, double* fy,
               double* f_final) {
  lattice L;
  if (load_lattice(p->Q, &L) || check_params(p, &L)) return -1;
  real* f = import_f(p, &L, f0);
  real* g = import_f(p, &L, NULL);
  real* rowfx = (real*)calloc((size_t)p->ny, sizeof(real));
  real* rowfy = (real*)calloc((size_t)p->ny, sizeof(real));
  const int diffuse = p->wall == ORC_WALL_DS || p->wall == ORC_WALL_MAXWELL;
  real* rho_w = diffuse ? (real*)calloc((size_t)wall_columns(p), sizeof(real)) : NULL;
  if (!f || !g || !rowfx || !rowfy || (diffuse && !rho_w)) {
    free(f); free(g); free(rowfx); free(rowfy); free(rho_w);
    return -2;
  }
  const real inv_tau = inv_tau_of(p->tau);
#ifdef _OPENMP
  if (p->nthreads > 0) omp_set_num_threads(p->nthreads);
#endif
  for (long n = 0; n < nsteps; ++n) {
    const real U = (real)(p->u0 * sin(p->omega * ((double)n + 0.5)));
    if (rho_w) {
      if (p->geometry == ORC_GEOM_BOX) box_wall_density(p, &L, f, U, rho_w);
      else wall_density(p, &L, f, U, rho_w);
    }
#pragma omp parallel for schedule(static)
    for (int y = 0; y < p->ny; ++y) {
      real Fx = 0, Fy = 0;
      for (int x = 0; x < p->nx; ++x) {
        if (in_body(p, x, y)) continue;
        real fa[ORC_MAXQ], fo[ORC_MAXQ];
        for (int i = 0; i < L.Q; ++i) fa[i] = advect_one(p, &L, f, x, y, i, U, rho_w, &Fx, &Fy);
        collide(&L, p->collision, inv_tau, fa, fo);
        for (int i = 0; i < L.Q; ++i) G_AT(g, x, y, i) = fo[i];
      }
      rowfx[y] = Fx;
      rowfy[y] = Fy;
    }
    real Fx = 0, Fy = 0;
    for (int y = 0; y < p->ny; ++y) {
      Fx += rowfx[y];
      Fy += rowfy[y];
    }
    if (fx) fx[n] = (double)Fx;
    if (fy) fy[n] = (double)Fy;
    real* t = f;
    f = g;
    g = t;
  }
  if (f_final) export_f(p, &L, f, f_final);
  free(f); free(g); free(rowfx); free(rowfy); free(rho_w);
  return 0;
}

/* Lock-in projection (Sec. 2 force decomposition F_f = -m(gamma x_t + beta x_tt)):
 * least-squares fit of F_n ~ a sin(omega t_n) + b cos(omega t_n) + c over
 * n in [first, first + count), t_n = n + 1/2, by the 3x3 normal equations in
 * long double.  With u = u0 sin(omega t) and F = -(R u + (X/omega) du/dt):
 * R = -a/u0 and X = -b/u0.  out = {a, b, c, R, X}. */
int oracle_lockin_fit(const double* F, long first, long count, double omega, double u0,
                      double* out) {
  long double G[3][4] = {{0}};
  for (long n = first; n < first + count; ++n) {
    long double t = (long double)n + 0.5L;
    long double b[3] = {sinl(omega * t), cosl(omega * t), 1.0L};
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) G[r][c] += b[r] * b[c];
      G[r][3] += b[r] * (long double)F[n];
    }
  }
  /* Gaussian elimination with partial pivoting */
  for (int c = 0; c < 3; ++c) {
    int piv = c;
    for (int r = c + 1; r < 3; ++r)
      if (fabsl(G[r][c]) > fabsl(G[piv][c])) piv = r;
    if (G[piv][c] == 0) return -1;
    for (int k = 0; k < 4; ++k) {
      long double t = G[c][k];
      G[c][k] = G[piv][k];
      G[piv][k] = t;
    }
    for (int r = 0; r < 3; ++r) {
      if (r == c) continue;
      long double m = G[r][c] / G[c][c];
      for (int k = c; k < 4; ++k) G[r][k] -= m * G[c][k];
    }
  }
  long double a = G[0][3] / G[0][0], b = G[1][3] / G[1][1], c = G[2][3] / G[2][2];
  out[0] = (double)a;
  out[1] = (double)b;
  out[2] = (double)c;
  out[3] = (double)(-a / u0);
  out[4] = (double)(-b / u0);
  return 0;
}
