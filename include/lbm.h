/*
 * lbm.h -- C ABI of the MI355X lattice-BGK solver for an oscillating body in
 * a BGK gas (Colosqui, Karabacak, Ekinci & Yakhot, "Lattice Boltzmann
 * simulation of high-frequency flows: electromechanical resonators in
 * gaseous media", 2009).
 *
 * The problem (Sec. 2 and Sec. 6): a rigid body with static geometry whose
 * wall moves with U_w(t) = u0 sin(omega t) along x, in a gas of relaxation
 * time tau.  The output is the fluid force F_f(t) on the body and its split
 * into a dissipative and an inertial part, F = -(R u + (X/omega) du/dt),
 * i.e. the complex impedance Z = R + iX as a function of tau*omega.
 *
 * The method (Sec. 5): lattice BGK on a Gauss-Hermite velocity set (D2Q9 or
 * the paper's D2Q37, appendix table), second-order Hermite equilibrium (eq.
 * feq_h2), advection f_i^adv(x) = f_i(x - v_i) (eq. advection), regularized
 * collision f_i = f_i^eq + (1 - 1/tau) fne_i (eqs. regularization, fne);
 * walls by bounce-back (Sec. 4, eq. BB) with the moving-wall term.
 *
 * Conventions
 *  - Lattice units: cell spacing 1, time step 1, integer velocities, theta =
 *    sound speed squared (1/3 for D2Q9, 0.69795332201968309 for D2Q37).
 *  - tau is the relaxation time of the discrete update; the gas viscosity is
 *    nu = theta (tau - 1/2) and the gas relaxation time tau_g = tau - 1/2,
 *    so a workload point tau_g*omega maps to tau = tau_g*omega/omega + 1/2.
 *  - One step = pull advection + collision.  Step n (t = n -> n+1) uses
 *    U_w(n + 1/2) and its force F_n is stamped at t_n = n + 1/2.
 *  - Populations exchanged through this ABI are FP64 full populations f
 *    (not deviations), layout [q][y][x] (x fastest), q in the canonical
 *    velocity order given by lbm_lattice().  Cells inside the body read as 0
 *    and are ignored on input.
 *  - Every call returns 0 (LBM_OK) or a negative LBM_E* code; nothing aborts
 *    on bad input and no C++ exception crosses the ABI.
 *  - A solver is used from one host thread at a time.  Different solvers on
 *    different streams are independent.  Results are deterministic: the
 *    force reduction has a fixed order, so equal parameters and populations
 *    give bit-identical forces.
 */
#ifndef LBM_H
#define LBM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2

typedef struct lbm_solver lbm_solver; /* opaque; owned by the library */

enum {
  LBM_OK = 0,
  LBM_EINVAL = -1,    /* invalid argument or parameter combination */
  LBM_ENOMEM = -2,    /* device or host allocation failed, or caller buffer too small */
  LBM_EHIP = -3,      /* a HIP runtime call failed (no device, launch failure, ...) */
  LBM_ERANGE = -4,    /* step beyond max_steps, or history request outside the ring */
  LBM_EUNSTABLE = -5, /* a cell reached rho <= 0 or a non-finite value */
  LBM_EABI = -6,      /* params.abi_version != LBM_ABI_VERSION */
  LBM_ESCRATCH = -7   /* lbm_create_static: the parameters need more than
                         LBM_STATIC_SCRATCH_BYTES, or a live solver holds the array */
};

enum { LBM_D2Q9 = 9, LBM_D2Q37 = 37 };

/* Population storage on the device.  Both store deviations f - w_i rho0.
 * F32_DEV collides in FP32; the wall force and the lock-in sums stay FP64. */
enum { LBM_STORE_F64 = 0, LBM_STORE_F32_DEV = 1 };

/* Collision: regularized (eqs. regularization, fne) or plain BGK
 * f_i = f_i^eq + (1 - 1/tau)(f_i^adv - f_i^eq) (eq. LBGK, for checks). */
enum { LBM_COLL_REGULARIZED = 0, LBM_COLL_BGK = 1 };

/* Wall model of the moving plate or body: bounce-back (eq. BB), or diffuse
 * scattering (eq. DS): a population arriving from the moving wall in column
 * x is the H2 equilibrium (eq. feq_h2) at the wall velocity with the wall
 * density rho_w(x) that balances the mass of the populations of column x
 * crossing the wall in that step (zero normal mass flux, eq. kinetic_bc; the
 * crossing populations are those bounce-back would reflect into column x).
 * Maxwell wall: a fraction `accommodation` (sigma_v of Sec. 3, 0..1) of
 * every arrival is the diffuse one and the rest the specular image -- the
 * population of (vx, -vy) that crossed the wall from column x - vx at the
 * mirror row, reflected in y only; 1 is the diffuse wall, 0 specular
 * reflection (no shear).  On a box each link belongs to the face on whose
 * axis its arrival cell lies outside the body (links outside it on both axes,
 * at the corners, keep bounce-back); a face is cut into columns, one per
 * arrival coordinate along it; a diffuse column returns the mass bounce-back
 * would return through its links (on the faces normal to the motion this
 * includes the mass the moving face displaces); the specular image is the
 * population that left the source point mirrored through the face plane with
 * its normal velocity reversed, plus the moving-wall term on the faces normal
 * to the motion.  A box with diffuse or Maxwell faces has at most 1024 face
 * columns (2 (box_lx + box_ly)).  The stationary far wall of a plate stays
 * bounce-back. */
enum { LBM_WALL_BB = 0, LBM_WALL_DS = 1, LBM_WALL_MAXWELL = 2 };

/* Geometry.
 *  PLATE:    x periodic (nx cells); the moving wall lies half-way below row
 *            0 (y = -1/2); the far side is selected by `far`.
 *  BOX:      solid rectangle [box_x0, box_x0+box_lx) x [box_y0, box_y0+box_ly)
 *            moving along x inside an nx x ny domain with a rest-equilibrium
 *            far field on all four sides (far must be LBM_FAR_EQ).
 *  PERIODIC: no body, periodic in x and y (no force; for checks). */
enum { LBM_GEOM_PLATE = 0, LBM_GEOM_BOX = 1, LBM_GEOM_PERIODIC = 2 };

/* Far side of a plate: stationary half-way bounce-back at y = ny - 1/2, or
 * rest-equilibrium ghost populations w_i rho0. */
enum { LBM_FAR_WALL = 0, LBM_FAR_EQ = 1 };

/* Device representation of the state.  The regularized collision (eqs.
 * regularization, fne) leaves every post-collision distribution in the span
 * of the Hermite polynomials up to second order, so six coefficients per
 * cell describe it exactly; a step then moves 6 values per cell in and out of
 * HBM instead of Q.  After populations are loaded (lbm_set_populations /
 * lbm_set_deviations) the next step reads them directly, so an arbitrary
 * initial state is honoured exactly; that needs a population buffer (Q values
 * per cell) beside the coefficients.  COEFFICIENTS_NOLOAD keeps the
 * coefficients without it (48 instead of 196 bytes per cell in FP32): the run
 * starts from rest, lbm_set_populations / lbm_set_deviations and a
 * population blob in lbm_set_state return LBM_EINVAL, everything else works
 * as with COEFFICIENTS (lbm_representation reports LBM_REPR_COEFFICIENTS). */
enum { LBM_REPR_AUTO = 0, LBM_REPR_POPULATIONS = 1, LBM_REPR_COEFFICIENTS = 2,
       LBM_REPR_COEFFICIENTS_NOLOAD = 3 };

typedef struct lbm_params {
  uint32_t abi_version;  /* LBM_ABI_VERSION */
  uint32_t lattice;      /* LBM_D2Q9 or LBM_D2Q37 */
  uint32_t storage;      /* LBM_STORE_* */
  uint32_t collision;    /* LBM_COLL_* */
  uint32_t wall;         /* LBM_WALL_BB, LBM_WALL_DS or LBM_WALL_MAXWELL (plate or box) */
  uint32_t geometry;     /* LBM_GEOM_* */
  uint32_t far;          /* LBM_FAR_* */
  uint32_t tile;         /* kernel tile.  Populations: 0 (= 1), 1, 2 or 4; one workgroup of
                            256*tile threads updates 256*tile consecutive cells, one per
                            thread.  Coefficients: 0 (= 3), 1, 2 or 3 = K; one workgroup
                            of 256 threads updates a tile of 64 columns x 4K rows, K
                            cells per thread.  Batch members kept in the same
                            representation must agree. */
  uint32_t representation; /* device state: 0 = automatic, 1 = the Q populations, 2 = the six
                            H2 coefficients of the regularized post-collision state
                            (regularized collision only; automatic picks 2 when nx >= 64
                            and one coefficient plane, ny x nx rounded up to 64, stays
                            under 2 GiB), 3 = as 2 without population loads */
  int32_t nx, ny;        /* domain in cells; nx >= 3 and ny >= 3 */
  int32_t box_x0, box_y0, box_lx, box_ly; /* BOX only; sides and margins >= longest link */
  double tau;            /* relaxation time of the update, > 1/2; +inf allowed (BGK: free streaming) */
  double omega;          /* drive angular frequency, radians per step */
  double u0;             /* drive amplitude, lattice units (Mach u0/sqrt(theta)) */
  double rho0;           /* rest density, > 0 */
  int64_t max_steps;     /* length of the run: the drive table covers steps [0, max_steps) */
  int64_t lockin_first;  /* lock-in window [first, first + count) in steps */
  int64_t lockin_count;
  int64_t history_capacity; /* force samples kept on the device (ring); 0 = max_steps */
  double accommodation;  /* LBM_WALL_MAXWELL: fraction of diffuse re-emission, 0..1 */
} lbm_params;

/* Fill *p with defaults: ABI version, D2Q37, F32_DEV, regularized, BB, plate
 * with a stationary far wall, rho0 = 1, accommodation 1; sizes, tau, drive
 * and steps zero. */
int lbm_params_init(lbm_params* p);

/* Velocity set in canonical order (orbits of the appendix table, members by
 * polar angle) and its weights, derived from the Gauss-Hermite moment
 * conditions (Sec. 5, appendix).  vx, vy, w: caller arrays of length Q.
 * Host only; needs no GPU. */
int lbm_lattice(int Q, int32_t* vx, int32_t* vy, double* w, double* theta);

/* Device bytes lbm_create_in needs for these parameters (validates them).
 * Host only; needs no GPU. */
int lbm_required_bytes(const lbm_params* p, uint64_t* bytes);

/* Create a solver on the current HIP device, enqueueing its initialisation
 * (rest state, counters) on `hip_stream` (a hipStream_t; NULL = the null
 * stream).  The library allocates and owns its device memory.  The stream
 * stays the caller's and must outlive the solver. */
int lbm_create(const lbm_params* p, void* hip_stream, lbm_solver** out);

/* As lbm_create, but in caller-owned device memory `dev_buf` of `bytes`
 * bytes (>= lbm_required_bytes, 256-byte aligned), e.g. a torch tensor; the
 * caller keeps it alive until lbm_destroy. */
int lbm_create_in(const lbm_params* p, void* hip_stream, void* dev_buf, uint64_t bytes,
                  lbm_solver** out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): as
 * lbm_create_in, but the solver's device memory is the library's own static
 * scratch array of LBM_STATIC_SCRATCH_BYTES on the current device (one array
 * per device, held until the process ends).  No device memory is allocated
 * or freed by this call, by lbm_step on the solver or by its lbm_destroy;
 * host-side bookkeeping uses the C++ heap.  The solver steps without HIP
 * graphs (instantiating one may allocate).  Everything the solver reads is
 * initialised by this call (rest state, counters, tables), so whatever an
 * earlier solver left in the array does not matter.  One such solver per
 * device at a time: while it lives (until lbm_destroy), another
 * lbm_create_static on that device returns LBM_ESCRATCH, as do parameters
 * whose lbm_required_bytes exceeds LBM_STATIC_SCRATCH_BYTES.  Launches of two
 * processes' static solvers on one device do not share the array (each
 * process has its own copy); work enqueued on the array by a destroyed solver
 * has completed (lbm_destroy waits). */
#define LBM_STATIC_SCRATCH_BYTES ((uint64_t)64 << 20)
int lbm_create_static(const lbm_params* p, void* hip_stream, lbm_solver** out);

/* Enqueue nsteps steps on the solver's stream and return without waiting.
 * Calls of 32 steps or more replay a HIP graph of 32 steps that the first
 * such call captures on the stream.  On the null stream, or if that first
 * call finds the stream already being captured by the caller, the solver
 * launches step by step from then on (into the caller's capture, if any).
 * Results are the same either way.
 * LBM_ERANGE if the run would pass max_steps (nothing is enqueued). */
int lbm_step(lbm_solver* s, int64_t nsteps);

/* Wait for the enqueued work.  LBM_EUNSTABLE if any step so far produced a
 * cell with rho <= 0 or a non-finite value (the solver stays usable for
 * lbm_get_populations and lbm_destroy). */
int lbm_synchronize(lbm_solver* s);

/* Representation the solver keeps on the device (LBM_REPR_POPULATIONS or
 * LBM_REPR_COEFFICIENTS). */
int lbm_representation(const lbm_solver* s, int* repr);

/* Steps enqueued so far (host-side count; no wait). */
int lbm_steps_done(const lbm_solver* s, int64_t* n);

/* Force of the gas on the moving wall or body at step n, the F_f of Sec. 2
 * computed by momentum exchange across the wall links (Sec. 6; eq. BB, and
 * eq. DS for the diffuse wall), FP64, stamped at t_n = n + 1/2.
 * Copy F_x[n], F_y[n] for n in [first, first + count) into caller arrays
 * (either may be NULL).  Waits for the stream.  LBM_ERANGE unless the
 * samples were computed and are still in the ring.  On an unstable solver
 * the arrays are filled and LBM_EUNSTABLE is returned (also by lbm_lockin
 * and lbm_impedance). */
int lbm_force_history(lbm_solver* s, int64_t first, int64_t count, double* fx, double* fy);

/* Lock-in sums of the force against the drive's phase (Sec. 2: the part of
 * F_f in phase with the velocity gives the damping, the part in phase with
 * the acceleration the added mass), over the part of the window computed so
 * far (waits):
 * sums = {sum F_x sin(omega t_n), sum F_x cos(omega t_n), sum F_x,
 *         the same three for F_y};  *nsamples = steps summed. */
int lbm_lockin(lbm_solver* s, double sums[6], int64_t* nsamples);

/* Impedance of the oscillating wall or body, the complex Z = R + iX of
 * eq. nems_W_tw, from the decomposition F_f = -m(gamma x_t + beta x_tt) of
 * Sec. 2 (R the damping, X / omega the added mass).
 * Least-squares fit F_x[n] ~ a sin(omega t_n) + b cos(omega t_n) + c over
 * the computed part of the window (3x3 normal equations, long double), and
 * the impedance of the drive u = u0 sin(omega t): R = -a/u0, X = -b/u0.
 * out = {a, b, c, R, X}.  Waits.  LBM_ERANGE if fewer than 3 samples. */
int lbm_impedance(lbm_solver* s, double out[5]);

/* Copy the current populations to/from host memory (n = Q*ny*nx doubles,
 * layout above).  Both wait for the stream and work on an unstable solver
 * too (they do not report LBM_EUNSTABLE).  Adding and removing the rest
 * state w_i rho0 rounds at its magnitude, so a get/set round trip is exact
 * only to that rounding; use the deviation calls below for checkpoints. */
int lbm_get_populations(lbm_solver* s, double* host, uint64_t n);
int lbm_set_populations(lbm_solver* s, const double* host, uint64_t n);

/* The same for the deviations f - w_i rho0 (FP64 on the host for both
 * storages).  With the population representation a round trip is bit-exact;
 * with coefficients, reading rebuilds the populations from them. */
int lbm_get_deviations(lbm_solver* s, double* host, uint64_t n);
int lbm_set_deviations(lbm_solver* s, const double* host, uint64_t n);

/* Raw device state (representation header + the current buffer), for
 * bit-exact checkpoints in either representation.  lbm_state_size gives the
 * byte count; lbm_set_state accepts only a blob taken from a solver with the
 * same parameters by a build with the same buffer layout (the header carries
 * a layout tag; any other blob gives LBM_EINVAL).  Both wait for the
 * stream. */
int lbm_state_size(const lbm_solver* s, uint64_t* bytes);
int lbm_get_state(lbm_solver* s, void* host, uint64_t bytes);
int lbm_set_state(lbm_solver* s, const void* host, uint64_t bytes);

/* Move the solver to step n (0 <= n < max_steps) with the given lock-in
 * sums (NULL = zeros).  The current state becomes that of step n; force
 * history before n is no longer available.  Together with lbm_get_state +
 * lbm_lockin at step n of one solver and lbm_set_state on another, this
 * resumes a run from a checkpoint bit-exactly.  Waits for the stream. */
int lbm_seek(lbm_solver* s, int64_t step, const double lockin_sums[6]);

/* Wait for the stream, then free the solver.  NULL is a no-op. */
int lbm_destroy(lbm_solver* s);

/* ------------------------------------------------------------------ batches
 * A batch advances many solvers -- uneven lattices with the same lattice,
 * storage and collision, created on the batch's stream -- with one fused
 * stream-collide launch per step over the tiles of every member of a kind
 * and one launch that reduces each member's wall force.  Each member runs the
 * kernel it runs when stepped alone, so its results are bit-identical alone
 * and in any mix.  Members may join and leave between steps
 * (continuous batching); a member stops when it reaches its max_steps.
 * Member read-out (force history, impedance, populations) goes through the
 * lbm_solver calls above.  The batch never owns or frees its members. */
typedef struct lbm_batch lbm_batch;

/* Empty batch on `hip_stream` (must be the members' stream).  Steps of at
 * least 32 are replayed from a captured HIP graph unless the stream is the
 * null stream (which cannot be captured). */
int lbm_batch_create(void* hip_stream, lbm_batch** out);

/* Add / remove a member (between steps).  LBM_EINVAL if the solver's stream,
 * lattice, storage or collision differs from the batch, if two members kept
 * in the same representation differ in `tile`, or on a double add / a remove of a
 * non-member.  A member joins at its own current step.  The kinds of member
 * -- kept as populations or as coefficients, with a bounce-back or a diffuse
 * (or Maxwell) moving wall -- are advanced by one launch each per step. */
int lbm_batch_add(lbm_batch* b, lbm_solver* s);
int lbm_batch_remove(lbm_batch* b, lbm_solver* s);

/* Number of members and of members that still have steps to run. */
int lbm_batch_size(const lbm_batch* b, int* members, int* active);

/* Enqueue up to nsteps steps of every member that has steps left; members
 * that reach max_steps stop there.  Returns without waiting. */
int lbm_batch_step(lbm_batch* b, int64_t nsteps);

/* Wait for the batch's stream; LBM_EUNSTABLE if any member is unstable. */
int lbm_batch_synchronize(lbm_batch* b);

/* Steps per captured graph (0 = launch every step directly). */
int lbm_batch_set_graphs(lbm_batch* b, int steps_per_graph);

/* Measurement: with timing enabled, every fused step-kernel launch is
 * bracketed by HIP events on the batch's stream (graphs are not used);
 * lbm_batch_kernel_time waits and returns the summed kernel time in ms and
 * the number of launches since timing was (re)enabled. */
int lbm_batch_timing(lbm_batch* b, int enable);
int lbm_batch_kernel_time(lbm_batch* b, double* ms, int64_t* launches);

/* Wait for the stream and free the batch (not its members).  NULL: no-op. */
int lbm_batch_destroy(lbm_batch* b);

/* Static message for an LBM_* code. */
const char* lbm_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
