"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (FP64 storage: 1e-12 relative on forces and impedance, T1 of the
design; FP32 deviation storage: 1e-4 relative on |Z| and 1e-4 rad on the
phase, and a per-step bound derived from FP32 rounding for short runs).
The oracle is run live on small cases; the full-size workloads compare with
stored oracle results in tests/golden (written by make_golden.py).
"""
import cmath
import json
import math
import os

import numpy as np
import pytest

import lbm_inputs as W
import oracle as O

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0904_4504_amd as P
    return P


def _oracle_params(s, threads=0):
    return O.OracleParams(
        Q=s.Q, nx=s.nx, ny=s.ny, tau=s.tau, omega=s.omega, u0=s.u0, rho0=s.rho0,
        geometry={W.PLATE: O.GEOM_PLATE, W.BOX: O.GEOM_BOX, W.PERIODIC: O.GEOM_PERIODIC}[s.geometry],
        far=O.FAR_WALL if s.far == W.FAR_WALL else O.FAR_EQ,
        collision=O.COLL_REGULARIZED if s.collision == "regularized" else O.COLL_BGK,
        box_x0=s.box[0], box_y0=s.box[1], box_lx=s.box[2], box_ly=s.box[3], nthreads=threads,
        wall={"bb": O.WALL_BB, "ds": O.WALL_DS, "maxwell": O.WALL_MAXWELL}[s.wall],
        sigma=s.accommodation)


def _gpu(P, s, f0=None, state=False, memory="torch", history_capacity=0, repr_=0, tile=0):
    p = P.params_from_solve(s, history_capacity, representation=repr_, tile=tile)
    with P.Solver(p, memory=memory) as sv:
        if f0 is not None:
            sv.set_populations(f0)
        sv.step(s.nsteps)
        sv.synchronize()
        cap = history_capacity or s.nsteps
        fx, fy = sv.force_history(s.nsteps - cap, cap)
        z = sv.impedance() if s.window_count >= 3 else None
        f = sv.get_populations() if state else None
    return fx, fy, z, f


def _f0(s, w, seed, amp):
    """Rest state plus a seeded perturbation (relative amplitude amp)."""
    f = w[:, None, None] * s.rho0 * (1 + W.random_state(s.Q, s.ny, s.nx, seed, amp))
    if s.geometry == W.BOX:
        x0, y0, lx, ly = s.box
        f[:, y0:y0 + ly, x0:x0 + lx] = 0.0
    return f


SMALL = {
    # name: (Q, geometry, far, collision, nx, ny, box, tau)
    "q9_plate_wall_narrow": (9, W.PLATE, W.FAR_WALL, "regularized", 5, 300, (0, 0, 0, 0), 0.8),
    "q9_plate_eq_wide": (9, W.PLATE, W.FAR_EQ, "regularized", 70, 41, (0, 0, 0, 0), 0.6),
    "q9_box": (9, W.BOX, W.FAR_EQ, "regularized", 70, 45, (20, 15, 12, 9), 0.9),
    "q9_periodic_bgk": (9, W.PERIODIC, W.FAR_EQ, "bgk", 33, 29, (0, 0, 0, 0), 0.7),
    "q37_plate_wall_narrow": (37, W.PLATE, W.FAR_WALL, "regularized", 4, 333, (0, 0, 0, 0), 2.0),
    "q37_plate_eq_wide": (37, W.PLATE, W.FAR_EQ, "regularized", 67, 40, (0, 0, 0, 0), 0.7),
    "q37_box": (37, W.BOX, W.FAR_EQ, "regularized", 71, 47, (21, 15, 13, 10), 1.3),
    "q37_box_bgk": (37, W.BOX, W.FAR_EQ, "bgk", 64, 40, (20, 14, 6, 5), 0.8),
    "q37_periodic": (37, W.PERIODIC, W.FAR_EQ, "regularized", 31, 37, (0, 0, 0, 0), 5.0),
    "q37_plate_large_tau": (37, W.PLATE, W.FAR_WALL, "regularized", 4, 260, (0, 0, 0, 0), 16298.0),
    # periodic lattices shorter than a staged coefficient tile (18 rows for
    # D2Q37, 14 for D2Q9): the staging wraps rows more than once
    "q37_periodic_short": (37, W.PERIODIC, W.FAR_EQ, "regularized", 66, 11, (0, 0, 0, 0), 1.0),
    "q9_periodic_short": (9, W.PERIODIC, W.FAR_EQ, "regularized", 64, 5, (0, 0, 0, 0), 0.8),
}


def _small_solve(name, storage, nsteps=40, wall="bb", sigma=1.0):
    Q, geom, far, coll, nx, ny, box, tau = SMALL[name]
    om = 2 * math.pi / 32
    return W.Solve(Q=Q, geometry=geom, far=far, nx=nx, ny=ny, tau=tau, omega=om, u0=1e-3,
                   box=box, nsteps=nsteps, window_first=8, window_count=nsteps - 8,
                   storage=storage, collision=coll, name=name, wall=wall, accommodation=sigma)


def _small_parity(P, name, storage, repr_, tile=0, wall="bb", sigma=1.0):
    s = _small_solve(name, storage, wall=wall, sigma=sigma)
    print(f"case {name} {storage} repr {repr_} tile {tile} wall {wall} {sigma} {s.nx}x{s.ny}",
          flush=True)
    v, w, th = P.lattice(s.Q)
    f0 = _f0(s, w, seed=sum(map(ord, name)) % 1000, amp=1e-3)
    fx, fy, z, f = _gpu(P, s, f0, state=True, repr_=repr_, tile=tile)
    ox, oy, of = O.run(_oracle_params(s), s.nsteps, f0=f0, want_state=True, variant="ld")
    wo = O.lattice(s.Q, "ld")[1]
    dev_o = of - wo[:, None, None] * s.rho0
    dev_g = f - w[:, None, None] * s.rho0
    if s.geometry == W.BOX:
        x0, y0, lx, ly = s.box
        dev_o[:, y0:y0 + ly, x0:x0 + lx] = 0
        dev_g[:, y0:y0 + ly, x0:x0 + lx] = 0
    scale = np.max(np.abs(dev_o))
    tol_pop, tol_f = (1e-12, 1e-12) if storage == "f64" else (2e-5, 2e-5)
    # populations cross the ABI as full f in FP64: one rounding of each side
    # at the magnitude of w_i rho0 is the floor of this comparison
    floor = 2 * np.spacing(np.max(w) * s.rho0)
    assert np.max(np.abs(dev_g - dev_o)) <= tol_pop * scale + floor
    if s.geometry != W.PERIODIC:
        fscale = max(np.max(np.abs(ox)), np.max(np.abs(oy)))
        assert np.max(np.abs(fx - ox)) <= tol_f * fscale
        assert np.max(np.abs(fy - oy)) <= tol_f * fscale
        if np.max(np.abs(ox)) <= 1e-12 * fscale:
            # no shear at all (specular wall): no impedance to compare
            assert np.max(np.abs(fx)) <= 1e-12 * fscale
            return
        zo = O.lockin_fit(ox, s.window_first, s.window_count, s.omega, s.u0)
        assert abs(z["Z"] - zo["Z"]) <= (1e-11 if storage == "f64" else 1e-4) * abs(zo["Z"])


@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", list(SMALL))
def test_small_parity(P, name, storage, repr_):
    """Populations after 40 steps and every per-step force, element by element,
    for both device representations (the first step reads the loaded
    populations, later steps the H2 coefficients)."""
    if repr_ == 2 and SMALL[name][3] != "regularized":
        pytest.skip("coefficients hold only the regularized (H2) state")
    _small_parity(P, name, storage, repr_)


@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", ["q9_plate_wall_narrow", "q9_plate_eq_wide",
                                  "q37_plate_wall_narrow", "q37_plate_eq_wide",
                                  "q37_plate_large_tau"])
def test_small_parity_diffuse_wall(P, name, storage, repr_):
    """The diffuse-scattering moving wall (eq. DS) against the oracle:
    populations after 40 steps, every per-step force and the impedance."""
    _small_parity(P, name, storage, repr_, wall="ds")


@pytest.mark.parametrize("sigma", [0.0, 0.6])
@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", ["q9_plate_wall_narrow", "q37_plate_wall_narrow",
                                  "q37_plate_eq_wide"])
def test_small_parity_maxwell_wall(P, name, storage, repr_, sigma):
    """The Maxwell wall (accommodation sigma: specular at 0) against the
    oracle: populations after 40 steps, every per-step force, the impedance."""
    _small_parity(P, name, storage, repr_, wall="maxwell", sigma=sigma)


@pytest.mark.parametrize("wall,sigma", [("ds", 1.0), ("maxwell", 0.0), ("maxwell", 0.6)])
@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", ["q9_box", "q37_box", "q37_box_bgk"])
def test_small_parity_box_walls(P, name, storage, repr_, wall, sigma):
    """Diffuse, specular and mixed faces on the box (faces cut into columns,
    corner links bounce back) in both device representations against the
    oracle: populations after 40 steps, every per-step force, the impedance."""
    if repr_ == 2 and SMALL[name][3] != "regularized":
        pytest.skip("coefficients hold only the regularized (H2) state")
    _small_parity(P, name, storage, repr_, wall=wall, sigma=sigma)


@pytest.mark.parametrize("wall,sigma", [("ds", 1.0), ("maxwell", 0.0), ("maxwell", 0.6)])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("Q", [9, 37])
def test_box_walls_free_molecular(P, Q, storage, wall, sigma):
    """Free streaming past the convex box from rest: every population that
    reaches it is at rest, so each step's force is the closed form the link
    enumeration gives (the free-molecular limit, eq. free-molecular, for these
    faces; the oracle is pinned to the same enumeration)."""
    from tests.test_oracle_pins import _free_molecular_box_force
    v, w, th = P.lattice(Q)
    box, om, n = (12, 14, 10, 7), 2 * math.pi / 50, 60
    s = W.Solve(Q=Q, geometry=W.BOX, far=W.FAR_EQ, nx=40, ny=40, tau=float("inf"), omega=om,
                u0=1e-3, box=box, nsteps=n, window_first=10, window_count=n - 10,
                storage=storage, collision="bgk", wall=wall, accommodation=sigma)
    fx, fy, z, _ = _gpu(P, s)
    U = 1e-3 * np.sin(om * (np.arange(n) + 0.5))
    expect = np.array([_free_molecular_box_force(v, w, th, box, u, sigma, wall)[0] for u in U])
    tol = 1e-13 if storage == "f64" else 2e-7
    # the sums cancel O(1) rest-state terms: compare at that scale
    scale = max(np.max(np.abs(expect)), 1.0) if storage == "f64" else np.max(np.abs(expect))
    assert np.max(np.abs(fx - expect)) <= tol * scale
    assert np.max(np.abs(fy)) <= tol * scale


@pytest.mark.parametrize("tile", [1, 3])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", ["q9_box", "q37_box", "q37_plate_eq_wide", "q37_periodic",
                                  "q37_plate_wall_narrow", "q37_periodic_short",
                                  "q9_periodic_short"])
def test_small_parity_coef_tiles(P, name, storage, tile):
    """The coefficient kernel with its other tiles (1 and 3 cells per thread,
    tiles of 4 and 12 rows) against the oracle."""
    _small_parity(P, name, storage, 2, tile)


@pytest.mark.parametrize("wall,sigma", [("ds", 1.0), ("maxwell", 0.4)])
@pytest.mark.parametrize("tile", [1, 2])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
@pytest.mark.parametrize("name", ["q9_box", "q37_box", "q37_plate_eq_wide"])
def test_small_parity_coef_tiles_walls(P, name, storage, tile, wall, sigma):
    """The diffuse and Maxwell walls (plate and box faces) in the coefficient
    kernel's other tile shapes (1 and 2 cells per thread: every wall cell then
    sits at another place of its tile and of the staged halo) against the
    oracle."""
    _small_parity(P, name, storage, 2, tile, wall=wall, sigma=sigma)


@pytest.mark.parametrize("wall", ["bb", "ds", "maxwell"])
@pytest.mark.parametrize("Q", [9, 37])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_first_step_and_free_molecular_limit(P, Q, storage, wall):
    """Closed forms: with free streaming (BGK, tau = inf) and an open far
    field every population reaching the wall is at rest (eq. free-molecular).
    Bounce-back: F_n = -2 rho0 C_s nx U_w at every step.  Diffuse wall: the
    wall emits w_i rho_w E_i(U_w) with rho_w = rho0 A1 / (A1 + U_w^2 A2), so
    F_n = -rho0 C_s nx U_w A1 / (A1 + U_w^2 A2) -- half of bounce-back to
    O(U_w^2) (BB = 2 x DS).  Maxwell wall of accommodation sigma: sigma times
    the diffuse force (its specular share exerts no shear).
    C_s = sum_{v_y<0} w |v_y| v_x^2 / theta, A1 = sum_{v_y>0} v_y w,
    A2 = sum_{v_y>0} v_y w (v_x^2/2theta^2 - 1/2theta)."""
    v, w, th = P.lattice(Q)
    C_s = sum(w[i] * abs(v[i, 1]) * v[i, 0] ** 2 / th for i in range(Q) if v[i, 1] < 0)
    A1 = sum(w[i] * v[i, 1] for i in range(Q) if v[i, 1] > 0)
    A2 = sum(w[i] * v[i, 1] * (v[i, 0] ** 2 / (2 * th * th) - 1 / (2 * th))
             for i in range(Q) if v[i, 1] > 0)
    om = 2 * math.pi / 64
    sigma = 0.3 if wall == "maxwell" else 1.0
    s = W.Solve(Q=Q, geometry=W.PLATE, far=W.FAR_EQ, nx=300, ny=40, tau=float("inf"),
                omega=om, u0=1e-3, nsteps=256, window_first=64, window_count=192,
                storage=storage, collision="bgk", wall=wall, accommodation=sigma)
    fx, fy, z, _ = _gpu(P, s)
    U = 1e-3 * np.sin(om * (np.arange(256) + 0.5))
    if wall == "bb":
        expect = -2 * C_s * s.nx * U
    else:
        expect = -sigma * C_s * s.nx * U * A1 / (A1 + U * U * A2)
    tol = 1e-13 if storage == "f64" else 2e-7
    assert np.max(np.abs(fx - expect)) <= tol * np.max(np.abs(expect))
    R = (2 if wall == "bb" else sigma) * C_s
    assert z["R"] / s.nx == pytest.approx(R, rel=10 * tol if wall == "bb" else 1e-6)
    assert abs(z["X"] / s.nx) <= 10 * tol


def _golden(name):
    path = os.path.join(GOLDEN, name + ".json")
    if not os.path.exists(path):
        pytest.skip(f"no stored oracle result {name}")
    with open(path) as fh:
        return json.load(fh)


def _cmp_samples(fx, g, tol, key="fx"):
    steps = np.array(g["samples"]["step"])
    ref = np.array(g["samples"][key])
    scale = g["max_abs_fx"]
    err = np.max(np.abs(fx[steps] - ref)) / scale
    assert err <= tol, err
    return err


@pytest.mark.parametrize("repr_", [0, 2], ids=["auto", "coefficients"])
def test_stokes_plate_full_fp64(P, repr_):
    """D2Q9 FP64, 4 x 256, 160 850 steps with seeded noise: every sampled force
    and the impedance within 1e-12 of the long-double oracle, in the
    representation the library picks (populations, for so narrow a lattice)
    and in the H2 coefficients (the coefficient kernel's staging then wraps
    each 4-cell row some 16 times)."""
    g = _golden("stokes_plate")["ld"]
    s = W.stokes_plate()
    v, w, th = P.lattice(9)
    f0 = w[:, None, None] * s.rho0 + W.initial_noise(s)
    fx, fy, z, _ = _gpu(P, s, f0, repr_=repr_)
    _cmp_samples(fx, g, 1e-12)
    assert z["R"] == pytest.approx(g["fit"]["R"], rel=1e-12)
    assert z["X"] == pytest.approx(g["fit"]["X"], rel=1e-12)
    Zs = (1 + 1j) * math.sqrt(0.1 * s.omega / 2)
    assert abs(abs(z["Z"] / s.nx) / abs(Zs) - 1) < 1e-2


@pytest.mark.parametrize("repr_", [0, 2], ids=["auto", "coefficients"])
@pytest.mark.parametrize("tw", W.PLATE_SWEEP_TAU_OMEGA)
def test_plate_sweep_full(P, tw, repr_):
    """D2Q37, 4 x 2048, 30 periods: FP32-deviation storage within 1e-4 on |Z|
    and 1e-4 rad on the phase of the FP64 oracle; FP64 storage within 1e-12;
    in the representation the library picks and in the H2 coefficients."""
    g = _golden(f"plate_sweep_tw{tw:g}")
    Zo = complex(g["fit"]["R"], g["fit"]["X"])
    for storage in ("f32dev", "f64"):
        s = W.plate_sweep(tw, storage=storage)
        fx, fy, z, _ = _gpu(P, s, repr_=repr_)
        print(f"tw={tw} {storage} repr {repr_} Z={z['Z']} oracle={Zo}", flush=True)
        if storage == "f64":
            assert abs(z["Z"] - Zo) <= 1e-12 * abs(Zo)
            _cmp_samples(fx, g, 1e-11)
        else:
            assert abs(abs(z["Z"]) / abs(Zo) - 1) <= 1e-4
            assert abs(cmath.phase(z["Z"]) - cmath.phase(Zo)) <= 1e-4


@pytest.mark.parametrize("repr_", [0, 1], ids=["auto", "populations"])
@pytest.mark.parametrize("tw", W.BEAM_TAU_OMEGA)
def test_beam_box_full(P, tw, repr_):
    """D2Q37 FP32 deviation storage, 1024^2 with a 32 x 16 body, 20 480 steps:
    impedance within 1e-4 (|Z|) and 1e-4 rad of the FP64 oracle; the body is
    y-symmetric so the lift stays at rounding level.  In the representation
    the library picks (the H2 coefficients) and as populations."""
    g = _golden(f"beam_box_tw{tw:g}")
    Zo = complex(g["fit"]["R"], g["fit"]["X"])
    s = W.beam_box(tw)
    fx, fy, z, _ = _gpu(P, s, repr_=repr_)
    print(f"tw={tw} repr {repr_} Z={z['Z']} oracle={Zo}", flush=True)
    assert abs(abs(z["Z"]) / abs(Zo) - 1) <= 1e-4
    assert abs(cmath.phase(z["Z"]) - cmath.phase(Zo)) <= 1e-4
    _cmp_samples(fx, g, 1e-3)
    assert np.max(np.abs(fy)) <= 1e-5 * np.max(np.abs(fx))


def _solve_from_golden(g, storage="f32dev"):
    """The workload a stored oracle run was made for, in the given storage."""
    d = dict(g["solve"])
    d["box"] = tuple(d["box"])
    d["storage"] = storage
    return W.Solve(**d)


def _batch_full(P, names, representation=0):
    """Run the stored workloads `names` (FP32 deviation storage, from rest,
    the representation the library picks unless one is given) as one batch;
    return the (golden, solve, force history, impedance) of each."""
    import torch
    gs = [_golden(n) for n in names]
    solves = [_solve_from_golden(g) for g in gs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        svs = [P.Solver(P.params_from_solve(s, loads=False, representation=representation),
                        stream=stream) for s in solves]
        b = P.Batch(stream)
        try:
            for sv, s in zip(svs, solves):
                print(f"case {s.name} {s.nx}x{s.ny} box {s.box} tau*omega {s.tau_omega:.4g} "
                      f"steps {s.nsteps} repr {sv.representation}", flush=True)
                b.add(sv)
            b.step(max(s.nsteps for s in solves))
            b.synchronize()
            out = []
            for g, s, sv in zip(gs, solves, svs):
                fx, _ = sv.force_history(0, s.nsteps)
                out.append((g, s, fx, sv.impedance(), sv.representation))
        finally:
            b.close()
            for sv in svs:
                sv.close()
    return out


def _assert_t2(z, g, name):
    """T2: |Z| within 1e-4 relative and the phase within 1e-4 rad of the
    stored FP64 oracle run."""
    Zo = complex(g["fit"]["R"], g["fit"]["X"])
    dz = abs(abs(z["Z"]) / abs(Zo) - 1)
    dp = abs(cmath.phase(z["Z"]) - cmath.phase(Zo))
    print(f"{name}: Z={z['Z']:.10g} oracle={Zo:.10g} |Z| {dz:.2e} phase {dp:.2e}", flush=True)
    assert dz <= 1e-4 and dp <= 1e-4, (name, dz, dp)


WIDE_PLATES = [f"wide_plate_{far}_tw{tw:g}" for far in ("wall", "eq") for tw in (0.01, 100.0)]
WALL_PLATES = [f"wide_plate_eq_{w}_tw{tw:g}" for w in ("ds", "maxwell0.6") for tw in (0.01, 100.0)]


def test_wide_plates_full_in_batch(P):
    """64 x 2048 plates (kept as H2 coefficients, the coefficient kernel's
    plate path) at tau*omega = 0.01 and 100 with the stationary far wall and
    with the rest-equilibrium far field, 20 480 steps each, advanced as one
    batch in FP32: impedance within T2 of the stored FP64 oracle runs, and
    every stored force sample within 1e-3 of the force scale."""
    for g, s, fx, z, repr_ in _batch_full(P, WIDE_PLATES):
        assert repr_ == P.lbm.REPR_COEFFICIENTS
        _assert_t2(z, g, s.name)
        _cmp_samples(fx, g, 1e-3)


@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
def test_wall_plates_full_in_batch(P, repr_):
    """The 64 x 2048 plate with the diffuse wall and with the Maxwell wall of
    accommodation 0.6 (rest-equilibrium far field) at tau*omega = 0.01 and
    100, 20 480 steps, advanced as one batch in FP32 in either device
    representation: impedance within T2 of the stored FP64 oracle runs and
    every stored force sample within 1e-3 of the force scale."""
    for g, s, fx, z, got in _batch_full(P, WALL_PLATES, representation=repr_):
        assert got == repr_
        _assert_t2(z, g, s.name)
        _cmp_samples(fx, g, 1e-3)


WALL_BOXES = [f"wall_box_{w}_tw{tw}" for tw in ("0.01", "1", "100") for w in ("ds", "maxwell0")]


@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
def test_wall_boxes_full_in_batch(P, repr_):
    """The 32 x 16 body in a 256^2 domain with diffuse and with specular
    faces, tau*omega = 0.01, 1 and 100, 20 480 steps, advanced as one batch in
    FP32 in either device representation: impedance within T2 of the stored
    FP64 oracle runs and every stored force sample within 1e-3 of the force
    scale."""
    for g, s, fx, z, got in _batch_full(P, WALL_BOXES, representation=repr_):
        assert got == repr_
        _assert_t2(z, g, s.name)
        _cmp_samples(fx, g, 1e-3)


def test_sweep_matches_oracle_on_reduced_points(P):
    """The damping sweep (plates AR = 0, rectangles AR = 1, 10, 26; bounce-back
    and diffuse walls) run by `run_sweep` as one batch on reduced points
    (period 64, 2 + 2 periods, plates 4 x 96, rectangles 8 x 8, 4 x 40, 3 x 78
    in 128^2) at tau*omega 0.01 and 1: every impedance within T2 of the
    oracle, and the nondimensional damping is R / (rho0 sqrt(theta/2) P)."""
    from paper_0904_4504_amd import sweep as S
    pts = S.sweep_solves(tau_omegas=(0.01, 1.0), period=64, transient_periods=2,
                         window_periods=2, plate_ny=96, box_n=128,
                         box_lx={1: 8, 10: 4, 26: 3})
    recs = S.run_sweep(pts)
    v, w, th = P.lattice(37)
    for (s, ar, wall, perim), r in zip(pts, recs):
        fx, _, _ = O.run(_oracle_params(s), s.nsteps)
        zo = O.lockin_fit(fx, s.window_first, s.window_count, s.omega, s.u0)
        _assert_t2({"Z": complex(r["R"], r["X"])}, {"fit": zo}, s.name)
        assert r["gamma_bar"] == pytest.approx(r["R"] / (s.rho0 * math.sqrt(th / 2) * perim),
                                               rel=1e-15)


def _subsample_names():
    small, large, drawn = W.batch_parity_subsample()
    return [f"batch_{i}" for i in [small] + drawn + [large]]


def test_batch_subsample_full(P):
    """The seeded 4-solve subsample of the 256-solve batch (its smallest and
    largest solve and two drawn by PCG64(40)), from rest, as one batch in FP32
    with the representation the library picks: every solve for its full
    20 480 steps except the largest (2026 x 2026), stored for 4096 steps;
    impedance within T2 of the stored FP64 oracle runs."""
    names = [n for n in _subsample_names()
             if os.path.exists(os.path.join(GOLDEN, n + ".json"))]
    if not names:
        pytest.skip("no stored oracle run of the subsample")
    for g, s, fx, z, repr_ in _batch_full(P, names):
        _assert_t2(z, g, s.name)
        _cmp_samples(fx, g, 1e-3)


# ------------------------------------------------------------------ behaviour

def test_deterministic_and_memory_owner_independent(P):
    s = _small_solve("q37_box", "f32dev", nsteps=30)
    a = _gpu(P, s, state=True, memory="torch")
    b = _gpu(P, s, state=True, memory="library")
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[3], b[3])


@pytest.mark.parametrize("name", ["q37_plate_wall_narrow", "q37_box"])
@pytest.mark.parametrize("storage", ["f64", "f32dev"])
def test_checkpoint_resume(P, storage, name):
    """Run 40 steps straight, versus 20 steps -> checkpoint (raw state +
    lock-in sums) -> a new solver seeks to step 20 -> 20 more steps: bit-exact
    in both representations."""
    s = _small_solve(name, storage, nsteps=40)
    v, w, th = P.lattice(s.Q)
    f0 = _f0(s, w, 5, 1e-3)
    fx, fy, z, fend = _gpu(P, s, f0, state=True)
    p = P.params_from_solve(s)
    with P.Solver(p) as a:
        a.set_populations(f0)
        a.step(20)
        mid = a.get_state()
        sums, _ = a.lockin()
    with P.Solver(p) as b:
        b.seek(20, sums)
        b.set_state(mid)
        b.step(20)
        fx2, _ = b.force_history(20, 20)
        z2 = b.impedance()
        f2 = b.get_populations()
        with pytest.raises(P.LbmError):
            b.force_history(19, 2)
    assert np.array_equal(fx2, fx[20:])
    assert np.array_equal(f2, fend)
    assert z2["Z"] == z["Z"]


def test_unstable_state_is_reported(P):
    s = _small_solve("q9_periodic_bgk", "f64", nsteps=10)
    p = P.params_from_solve(s)
    v, w, th = P.lattice(9)
    f0 = _f0(s, w, 1, 1e-3)
    f0[3, 5, 7] = np.nan
    with P.Solver(p) as sv:
        sv.set_populations(f0)
        sv.step(2)
        with pytest.raises(P.LbmError) as e:
            sv.synchronize()
        assert e.value.code == -5
        sv.get_populations()  # still readable


def test_range_errors_and_history_ring(P):
    s = _small_solve("q9_plate_wall_narrow", "f64", nsteps=50)
    full = _gpu(P, s)[0]
    p = P.params_from_solve(s, history_capacity=16)
    with P.Solver(p) as sv:
        with pytest.raises(P.LbmError) as e:
            sv.step(51)
        assert e.value.code == -4
        sv.step(50)
        fx, _ = sv.force_history(34, 16)
        assert np.array_equal(fx, full[34:])
        with pytest.raises(P.LbmError) as e:
            sv.force_history(33, 2)
        assert e.value.code == -4
        with pytest.raises(P.LbmError):
            sv.step(1)


def test_degenerate_calls(P):
    """Zero steps, read-outs before any step, an empty batch, and a batch
    stepped past its only member's last step: no-ops or range errors, and the
    member's forces are those of the same solve stepped alone."""
    import torch
    s = _small_solve("q37_box", "f32dev", nsteps=12)
    alone = _gpu(P, s)[0]
    stream = torch.cuda.Stream()
    with P.Solver(P.params_from_solve(s), stream=stream) as sv:
        sv.step(0)
        assert sv.steps_done == 0
        with pytest.raises(P.LbmError) as e:
            sv.impedance()
        assert e.value.code == -4
        with pytest.raises(P.LbmError) as e:
            sv.force_history(0, 1)
        assert e.value.code == -4
        assert sv.force_history(0, 0)[0].size == 0
        with P.Batch(stream) as b:
            b.step(5)                 # no members
            b.synchronize()
            assert b.size() == (0, 0)
            b.add(sv)
            b.step(0)
            b.step(12)
            b.step(7)                 # the member is done: nothing more runs
            b.synchronize()
            assert b.size() == (1, 0)
            assert sv.steps_done == 12
            fx, _ = sv.force_history(0, 12)
            b.remove(sv)
        assert np.array_equal(fx, alone)
        with pytest.raises(P.LbmError) as e:
            sv.step(1)
        assert e.value.code == -4


def test_lockin_sums_match_force_series(P):
    s = _small_solve("q37_box", "f64", nsteps=60)
    p = P.params_from_solve(s)
    with P.Solver(p) as sv:
        sv.step(60)
        fx, fy = sv.force_history(0, 60)
        sums, n = sv.lockin()
    assert n == s.window_count
    t = np.arange(s.window_first, s.window_first + s.window_count) + 0.5
    sn, cs = np.sin(s.omega * t), np.cos(s.omega * t)
    wx = fx[s.window_first:]
    assert sums[0] == pytest.approx(np.dot(wx, sn), rel=1e-12)
    assert sums[1] == pytest.approx(np.dot(wx, cs), rel=1e-12)
    assert sums[2] == pytest.approx(wx.sum(), rel=1e-12, abs=1e-18)


def test_periodic_mass_and_momentum_conserved(P):
    s = _small_solve("q37_periodic", "f64", nsteps=25)
    v, w, th = P.lattice(37)
    f0 = _f0(s, w, 9, 1e-2)
    _, _, _, f = _gpu(P, s, f0, state=True)
    assert abs(f.sum() - f0.sum()) <= 1e-13 * f0.sum()
    j0 = np.einsum("qyx,qa->a", f0, v.astype(float))
    j1 = np.einsum("qyx,qa->a", f, v.astype(float))
    assert np.max(np.abs(j1 - j0)) <= 1e-13 * f0.sum()


# ------------------------------------------------------------------ batching

def _mix(storage="f32dev"):
    om = 2 * math.pi / 40
    return [
        W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=90, ny=70, tau=0.9, omega=om,
                box=(30, 25, 20, 12), nsteps=60, window_first=20, window_count=40,
                storage=storage, name="box"),
        W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_WALL, nx=4, ny=700, tau=3.0, omega=om,
                nsteps=45, window_first=5, window_count=40, storage=storage, name="plate"),
        W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_EQ, nx=130, ny=50, tau=0.55, omega=om,
                nsteps=70, window_first=30, window_count=40, storage=storage, name="wide"),
    ]


def _alone(P, s, stream):
    with P.Solver(P.params_from_solve(s), stream=stream) as sv:
        sv.step(s.nsteps)
        fx, fy = sv.force_history(0, s.nsteps)
        return fx, fy, sv.get_populations()


def test_batch_sweep_subsample_matches_oracle(P):
    """The 256-solve sweep draw, on a seeded subsample: its smallest and its
    largest solve and two drawn at random, each from a perturbed rest state,
    truncated to 24 steps and advanced as one batch (FP32 deviation storage,
    the representation the library picks); every step's force against the
    FP64 oracle within the short-run FP32 bound."""
    import torch
    draw = W.batch_sweep()
    cells = [s.nx * s.ny for s in draw]
    rng = np.random.default_rng(4)
    pick = {int(np.argmin(cells)), int(np.argmax(cells))}
    while len(pick) < 4:
        pick.add(int(rng.integers(0, len(draw))))
    solves = [draw[i].scaled(24, 16) for i in sorted(pick)]
    v, w, th = P.lattice(37)
    stream = torch.cuda.Stream()
    f0s, svs = [], []
    for k, s in enumerate(solves):
        print(f"case {s.name} {s.nx}x{s.ny} box {s.box} tau {s.tau:.4g}", flush=True)
        f0s.append(_f0(s, w, seed=100 + k, amp=1e-3))
        sv = P.Solver(P.params_from_solve(s), stream=stream)
        sv.set_populations(f0s[-1])
        svs.append(sv)
    b = P.Batch(stream)
    try:
        for sv in svs:
            b.add(sv)
        b.step(24)
        b.synchronize()
        for s, sv, f0 in zip(solves, svs, f0s):
            fx, fy = sv.force_history(0, s.nsteps)
            ox, oy, _ = O.run(_oracle_params(s), s.nsteps, f0=f0)
            fscale = max(np.max(np.abs(ox)), np.max(np.abs(oy)))
            assert np.max(np.abs(fx - ox)) <= 2e-5 * fscale, s.name
            assert np.max(np.abs(fy - oy)) <= 2e-5 * fscale, s.name
    finally:
        b.close()
        for sv in svs:
            sv.close()


@pytest.mark.parametrize("graphs", [0, 8])
def test_batch_alone_equals_mix(P, graphs):
    """Uneven lattices in one fused launch, one member joining late and one
    finishing early: every member's forces and populations are bit-identical
    to the same solve stepped alone."""
    import torch
    stream = torch.cuda.Stream()
    solves = _mix()
    ref = [_alone(P, s, stream) for s in solves]
    svs = [P.Solver(P.params_from_solve(s), stream=stream) for s in solves]
    b = P.Batch(stream)
    b.set_graphs(graphs)
    b.add(svs[0])
    b.add(svs[1])
    b.step(10)
    b.add(svs[2])                 # joins at its own step 0
    b.step(100)                   # plate stops at 45, box at 60, wide after 70 of its own
    assert b.size() == (3, 0)
    b.synchronize()
    for s, sv, (rx, ry, rf) in zip(solves, svs, ref):
        fx, fy = sv.force_history(0, s.nsteps)
        assert np.array_equal(fx, rx) and np.array_equal(fy, ry), s.name
        assert np.array_equal(sv.get_populations(), rf), s.name
    b.close()
    for sv in svs:
        sv.close()


def test_batch_alone_equals_mix_with_diffuse_walls(P):
    """Diffuse and Maxwell walls beside bounce-back members, in both device
    representations: the launch then runs the kernels that carry the diffuse
    wall, and every member's forces and populations are still bit-identical
    to the same solve stepped alone."""
    import torch
    stream = torch.cuda.Stream()
    om = 2 * math.pi / 40
    solves = [
        W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_WALL, nx=4, ny=300, tau=3.0, omega=om,
                nsteps=45, window_first=5, window_count=40, wall="ds", name="plate_ds"),
        W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_EQ, nx=4, ny=200, tau=0.7, omega=om,
                nsteps=45, window_first=5, window_count=40, name="plate_bb"),
        W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_EQ, nx=130, ny=50, tau=0.55, omega=om,
                nsteps=45, window_first=5, window_count=40, wall="maxwell",
                accommodation=0.6, name="wide_maxwell"),
        W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=90, ny=70, tau=0.9, omega=om,
                box=(30, 25, 20, 12), nsteps=45, window_first=5, window_count=40, name="box"),
        W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=80, ny=66, tau=0.8, omega=om,
                box=(25, 20, 14, 9), nsteps=45, window_first=5, window_count=40, wall="ds",
                name="box_ds"),
        W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=70, ny=60, tau=1.1, omega=om,
                box=(22, 19, 11, 13), nsteps=45, window_first=5, window_count=40,
                wall="maxwell", accommodation=0.3, name="box_maxwell"),
    ]
    ref = [_alone(P, s, stream) for s in solves]
    svs = [P.Solver(P.params_from_solve(s), stream=stream) for s in solves]
    b = P.Batch(stream)
    for sv in svs:
        b.add(sv)
    b.step(45)
    b.synchronize()
    for s, sv, (rx, ry, rf) in zip(solves, svs, ref):
        fx, fy = sv.force_history(0, s.nsteps)
        assert np.array_equal(fx, rx) and np.array_equal(fy, ry), s.name
        assert np.array_equal(sv.get_populations(), rf), s.name
    b.close()
    for sv in svs:
        sv.close()


def test_large_batch_matches_alone(P):
    """Five perturbed 1024 x 1024 boxes: as one batch their coefficient state
    (about 250 MB) is past the size up to which the tiles go in bands per XCD,
    so the batch runs the row-interleaved work order while each solve alone
    runs the banded one; forces and final states are bit-identical."""
    import torch
    stream = torch.cuda.Stream()
    solves = [W.beam_box(tw).scaled(12, 8) for tw in (0.1, 0.3, 1.0, 3.0, 10.0)]
    v, w, th = P.lattice(37)
    f0 = _f0(solves[0], w, seed=11, amp=1e-3)
    ref = []
    for s in solves:
        with P.Solver(P.params_from_solve(s), stream=stream) as sv:
            sv.set_populations(f0)
            sv.step(1)            # the first step after a load runs alone
            sv.step(s.nsteps - 1)
            fx, fy = sv.force_history(0, s.nsteps)
            ref.append((fx, fy, sv.get_deviations()))
    svs = [P.Solver(P.params_from_solve(s), stream=stream) for s in solves]
    b = P.Batch(stream)
    try:
        for sv in svs:
            sv.set_populations(f0)
            sv.step(1)
            b.add(sv)
        b.step(solves[0].nsteps - 1)
        b.synchronize()
        for s, sv, (rx, ry, rd) in zip(solves, svs, ref):
            fx, fy = sv.force_history(0, s.nsteps)
            assert np.array_equal(fx, rx) and np.array_equal(fy, ry), s.name
            assert np.array_equal(sv.get_deviations(), rd), s.name
    finally:
        b.close()
        for sv in svs:
            sv.close()


def test_graph_replays_match_eager(P):
    """Replays of the captured graph, with eager work and synchronisation
    between them, each agree with plain launches."""
    import torch
    stream = torch.cuda.Stream()
    s = _mix()[0].scaled(64, 40)
    with P.Solver(P.params_from_solve(s), stream=stream) as ref:
        for _ in range(64):
            ref.step(1)   # one step per call: plain launches
        rx, _ = ref.force_history(0, 64)
    with P.Solver(P.params_from_solve(s), stream=stream) as sv:
        b = P.Batch(stream)
        b.add(sv)
        b.set_graphs(16)
        for r in range(4):
            b.step(16)
            with torch.cuda.stream(stream):
                junk = torch.ones(1000, device="cuda") * r   # eager work between replays
            b.synchronize()
            fx, _ = sv.force_history(16 * r, 16)
            assert np.array_equal(fx, rx[16 * r:16 * (r + 1)]), r
            del junk
        b.close()


@pytest.mark.parametrize("repr_", [1, 2], ids=["populations", "coefficients"])
def test_single_solver_graph_replays_match_eager(P, repr_):
    """A single solver's step calls of 32 steps or more replay a captured
    graph: four replays, with eager work and synchronisation between them,
    each agree bit for bit with one-step calls (plain launches), forces and
    final state."""
    import torch
    stream = torch.cuda.Stream()
    s = _mix()[0].scaled(4 * 32, 100)
    v, w, th = P.lattice(s.Q)
    f0 = _f0(s, w, seed=7, amp=1e-3)
    with P.Solver(P.params_from_solve(s, representation=repr_), stream=stream) as ref:
        ref.set_populations(f0)
        for _ in range(4 * 32):
            ref.step(1)
        rx, ry = ref.force_history(0, 4 * 32)
        rf = ref.get_populations()
    with P.Solver(P.params_from_solve(s, representation=repr_), stream=stream) as sv:
        sv.set_populations(f0)
        sv.step(1)                # the first step after a load runs alone
        for r in range(4):
            sv.step(32 if r < 3 else 31)
            with torch.cuda.stream(stream):
                junk = torch.ones(1000, device="cuda") * r   # eager work between replays
            sv.synchronize()
            lo, n = (1 + 32 * r, 32) if r < 3 else (97, 31)
            fx, fy = sv.force_history(lo, n)
            assert np.array_equal(fx, rx[lo:lo + n]) and np.array_equal(fy, ry[lo:lo + n]), r
            del junk
        assert np.array_equal(sv.get_populations(), rf)


def test_batch_rejects_mismatched_members(P):
    import torch
    stream = torch.cuda.Stream()
    a = _mix("f32dev")[0]
    c = _mix("f64")[0]
    sa = P.Solver(P.params_from_solve(a), stream=stream)
    sc = P.Solver(P.params_from_solve(c), stream=stream)
    sd = P.Solver(P.params_from_solve(a), stream=torch.cuda.Stream())
    b = P.Batch(stream)
    b.add(sa)
    for bad in (sc, sd, sa):
        with pytest.raises(P.LbmError):
            b.add(bad)
    b.close()
    for sv in (sa, sc, sd):
        sv.close()


# ------------------------------------------------------------------ serving

def test_served_impedances_match_oracle(P):
    """Requests of the serving loop (boxes and plates arriving over time,
    budget-limited admission) against the oracle: every served impedance
    within T2 of the FP64 oracle run of the same solve from rest."""
    import torch
    from paper_0904_4504_amd import serve
    om = 2 * math.pi / 64
    trace = []
    for k in range(5):
        if k % 2 == 0:
            s = W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=96, ny=72 + 8 * k, tau=0.8 + k,
                        omega=om, box=(40, 30, 14, 9), nsteps=256, window_first=128,
                        window_count=128, name=f"box{k}")
        else:
            s = W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_WALL, nx=4, ny=300 + 50 * k,
                        tau=0.6 + 5.0 * k, omega=om, nsteps=320, window_first=128,
                        window_count=192, name=f"plate{k}")
        trace.append((0.003 * k, s))
    need = sorted(P.required_bytes(P.params_from_solve(s, loads=False)) for _, s in trace)
    reqs, _ = serve.serve(trace, budget_bytes=need[-1] + need[-2] + 2048, chunk=64,
                          stream=torch.cuda.Stream())
    for r in reqs:
        s = r.solve
        fx, _, _ = O.run(_oracle_params(s), s.nsteps)
        zo = O.lockin_fit(fx, s.window_first, s.window_count, s.omega, s.u0)
        _assert_t2(r.result, {"fit": zo}, s.name)


def test_serving_results_same_alone_and_in_mix(P):
    """Requests arriving while others run are admitted as memory frees up (a
    budget of about two requests forces queueing), advance together in the
    running batch, and each impedance equals the same solve run alone."""
    import torch
    from paper_0904_4504_amd import serve
    om = 2 * math.pi / 64
    trace = []
    for k in range(7):
        if k % 3 == 0:
            s = W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=96 + 8 * k, ny=80, tau=0.7 + 0.3 * k,
                        omega=om, box=(40, 32, 16, 10), nsteps=320 + 32 * k, window_first=128,
                        window_count=192 + 32 * k, name=f"box{k}")
        else:
            s = W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_WALL, nx=4, ny=500 + 100 * k,
                        tau=0.6 + 2.0 * k, omega=om, nsteps=256 + 64 * k, window_first=64,
                        window_count=192 + 64 * k, name=f"plate{k}")
        trace.append((0.005 * k, s))
    stream = torch.cuda.Stream()
    need = sorted(P.required_bytes(P.params_from_solve(s, loads=False)) for _, s in trace)
    reqs, summ = serve.serve(trace, budget_bytes=need[-1] + need[-2] + 2048, chunk=48,
                             stream=stream)
    assert summ["requests"] == 7
    assert any(r.admitted > r.arrival + 1e-4 for r in reqs)   # someone had to wait
    for r in reqs:
        with P.Solver(P.params_from_solve(r.solve), stream=stream) as sv:
            sv.step(r.solve.nsteps)
            z = sv.impedance()
        assert r.result["Z"] == z["Z"], r.solve.name


@pytest.mark.parametrize("name,storage,repr_", [
    ("q37_box", "f32dev", 1), ("q9_plate_eq_wide", "f64", 1), ("q37_plate_wall_narrow", "f64", 1),
    ("q37_box", "f32dev", 2), ("q37_box", "f64", 2), ("q9_plate_eq_wide", "f64", 2),
    ("q37_plate_eq_wide", "f32dev", 2)])
def test_tile_variants_agree(P, name, storage, repr_):
    """Kernel tiles agree: cells per thread 1, 2, 4 of the population kernel
    give identical states and forces; the coefficient kernel with 1, 2, 3
    cells per thread sums every cell's contributions in the same order
    wherever the tile boundaries fall, and agrees to the storage rounding."""
    s = _small_solve(name, storage, nsteps=30)
    out = []
    for tile in ((1, 2, 4) if repr_ == 1 else (1, 2, 3)):
        p = P.params_from_solve(s, tile=tile, representation=repr_)
        with P.Solver(p) as sv:
            assert sv.representation == repr_
            sv.step(s.nsteps)
            fx, fy = sv.force_history(0, s.nsteps)
            out.append((fx, sv.get_populations()))
    v, w, th = P.lattice(s.Q)
    dev0 = out[0][1] - w[:, None, None] * s.rho0
    for fx, f in out[1:]:
        if repr_ == 1:
            assert np.array_equal(f, out[0][1])
            assert np.array_equal(fx, out[0][0])
        else:
            # the unrolled copies of the coefficient kernel may contract
            # a*b + c differently: agreement to the storage rounding
            dev = f - w[:, None, None] * s.rho0
            tol = 1e-13 if storage == "f64" else 2e-6
            err = np.max(np.abs(dev - dev0)) / np.max(np.abs(dev0))
            ferr = np.max(np.abs(fx - out[0][0])) / np.max(np.abs(out[0][0]))
            print(f"coefficient tiles {name} {storage}: state {err:.2e} force {ferr:.2e}", flush=True)
            assert err <= tol and ferr <= tol


def test_autotune_picks_a_tile_of_the_representation(P):
    """The autotuner times every tile of the representation the solves use
    and returns the fastest; a solver built with it matches the default."""
    from paper_0904_4504_amd import autotune
    solves = [_small_solve(n, "f32dev", nsteps=40) for n in ("q37_box", "q37_plate_eq_wide")]
    tile, times = autotune.tune(solves, steps=8, warmup=2, use_cache=False)
    assert sorted(times) == [1, 2, 3] and tile == min(times, key=times.get)
    out = []
    for t in (0, tile):
        with P.Solver(P.params_from_solve(solves[0], tile=t)) as sv:
            sv.step(solves[0].nsteps)
            out.append(sv.force_history(0, solves[0].nsteps)[0])
    assert np.max(np.abs(out[1] - out[0])) <= 2e-6 * np.max(np.abs(out[0]))
