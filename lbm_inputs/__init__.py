"""Seeded synthetic workloads for the oscillating-body lattice-BGK solver.

This module is shared by the tests, the benchmark and the smoke check.  It
only *describes* inputs (sizes, relaxation times, drive, seeds) and draws the
random numbers they need; it holds none of the method's arithmetic and
imports neither the oracle nor the HIP library.

Workloads (the paper gives no lattice sizes; these stand in for its
resonators: the thickness-shear quartz plate, AR ~ 0, and beam sections of
finite aspect ratio, Sec. 3 and Table 1, at the tau*omega values of Sec. 6):

  stokes_plate   D2Q9, FP64, 4 x 256 plate, tau = 0.8, Stokes depth
                 sqrt(2 nu / omega) = 16 cells, U0 = 1e-3, noise 1e-9, 20 periods
  plate_sweep    D2Q37, 4 x 2048 plate, stationary far wall, U0 = 1e-3,
                 tau*omega in {0.01, 0.1, 1, 10, 100}, 1024 steps per period,
                 30 periods, lock-in over the last 10
  beam_box       D2Q37, 1024 x 1024 domain, 32 x 16 body (32 along the motion)
                 centred, rest-equilibrium far field, tau*omega in {0.1, 1, 10},
                 10-period transient then a 10-period lock-in window
  batch_sweep    256 solves, sides in [256, 2048], aspect 1:1, 2:1, 4:1,
                 plate or box body (sides 8..64), log-uniform tau*omega in
                 [1e-2, 1e2]
  serving_mix    Poisson arrivals of beam_box-like and plate requests, 1:4

Relaxation time: the lattice relaxation time tau_LB of the discrete update
relates to the gas relaxation time by tau = tau_LB - 1/2 (the viscosity of
the discrete scheme is nu = theta (tau_LB - 1/2)), so a workload point
tau*omega maps to tau_LB = tau*omega / omega + 1/2.
"""
import dataclasses
import math

import numpy as np

PLATE, BOX, PERIODIC = "plate", "box", "periodic"
FAR_WALL, FAR_EQ = "wall", "eq"


@dataclasses.dataclass
class Solve:
    """One solve: geometry, drive, relaxation time, run length and window."""
    Q: int
    geometry: str
    far: str
    nx: int
    ny: int
    tau: float                 # lattice relaxation time tau_LB
    omega: float               # rad per step
    u0: float = 1e-3
    rho0: float = 1.0
    box: tuple = (0, 0, 0, 0)  # x0, y0, lx, ly (solid cells)
    nsteps: int = 0
    window_first: int = 0
    window_count: int = 0
    storage: str = "f32dev"    # "f64" or "f32dev"
    collision: str = "regularized"
    wall: str = "bb"           # moving wall: "bb", or "ds" / "maxwell" (plate only)
    accommodation: float = 1.0  # "maxwell": fraction re-emitted diffusely (0 specular)
    noise: float = 0.0
    seed: int = 0
    tau_omega: float = float("nan")
    name: str = ""

    @property
    def fluid_cells(self):
        return self.nx * self.ny - self.box[2] * self.box[3]

    def scaled(self, nsteps, window_count):
        """Same solve with a shorter run (window at the end)."""
        return dataclasses.replace(self, nsteps=nsteps, window_first=nsteps - window_count,
                                   window_count=window_count)


def tau_lb(tau_omega, omega):
    return tau_omega / omega + 0.5


def periods_steps(omega, periods):
    return int(round(periods * 2 * math.pi / omega))


def stokes_plate(delta=16, periods=20, window_periods=10, nx=4, ny=None):
    """D2Q9 FP64 plate with Stokes depth ``delta`` cells (tau_LB = 0.8, nu = 0.1)."""
    tau = 0.8
    nu = (tau - 0.5) / 3.0
    omega = 2 * nu / delta ** 2
    n = periods_steps(omega, periods)
    w = periods_steps(omega, window_periods)
    return Solve(Q=9, geometry=PLATE, far=FAR_WALL, nx=nx, ny=ny or 16 * delta, tau=tau,
                 omega=omega, u0=1e-3, nsteps=n, window_first=n - w, window_count=w,
                 storage="f64", noise=1e-9, seed=0, tau_omega=omega * (tau - 0.5),
                 name=f"stokes_plate_d{delta}")


PLATE_SWEEP_TAU_OMEGA = (0.01, 0.1, 1.0, 10.0, 100.0)


def plate_sweep(tau_omega, ny=2048, nx=4, period=1024, periods=30, window_periods=10,
                storage="f32dev"):
    omega = 2 * math.pi / period
    n = periods * period
    w = window_periods * period
    return Solve(Q=37, geometry=PLATE, far=FAR_WALL, nx=nx, ny=ny, tau=tau_lb(tau_omega, omega),
                 omega=omega, nsteps=n, window_first=n - w, window_count=w, storage=storage,
                 tau_omega=tau_omega, name=f"plate_sweep_tw{tau_omega:g}")


BEAM_TAU_OMEGA = (0.1, 1.0, 10.0)


def beam_box(tau_omega, n=1024, lx=32, ly=16, period=1024, transient_periods=10,
             window_periods=10, storage="f32dev"):
    omega = 2 * math.pi / period
    x0, y0 = (n - lx) // 2, (n - ly) // 2
    steps = (transient_periods + window_periods) * period
    return Solve(Q=37, geometry=BOX, far=FAR_EQ, nx=n, ny=n, tau=tau_lb(tau_omega, omega),
                 omega=omega, box=(x0, y0, lx, ly), nsteps=steps,
                 window_first=transient_periods * period, window_count=window_periods * period,
                 storage=storage, tau_omega=tau_omega, name=f"beam_box_tw{tau_omega:g}")


def wall_box(tau_omega, wall, accommodation=1.0, n=256, lx=32, ly=16, period=1024,
             transient_periods=10, window_periods=10, storage="f32dev"):
    """The beam-box body with a diffuse ("ds") or Maxwell ("maxwell",
    accommodation 0..1) surface in a smaller n x n domain."""
    s = beam_box(tau_omega, n=n, lx=lx, ly=ly, period=period,
                 transient_periods=transient_periods, window_periods=window_periods,
                 storage=storage)
    tag = wall if wall == "ds" else f"{wall}{accommodation:g}"
    return dataclasses.replace(s, wall=wall, accommodation=accommodation,
                               name=f"wall_box_{tag}_tw{tau_omega:g}")


def batch_sweep(count=256, seed=4, period=1024, transient_periods=10, window_periods=10,
                side_min=256, side_max=2048):
    """Uneven solves drawn from one PCG64 stream in a fixed order:
    aspect a in {1,2,4}; short side S ~ U{side_min .. side_max // a}; long
    side a*S; orientation (long side along x or y); body kind (plate or box,
    1:1); box sides U{8..64} each; log10(tau*omega) ~ U[-2, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = 2 * math.pi / period
    steps = (transient_periods + window_periods) * period
    out = []
    for k in range(count):
        a = int(rng.choice([1, 2, 4]))
        s = int(rng.integers(side_min, side_max // a + 1))
        along_x = bool(rng.integers(0, 2))
        nx, ny = (a * s, s) if along_x else (s, a * s)
        kind = PLATE if rng.integers(0, 2) == 0 else BOX
        lx, ly = int(rng.integers(8, 65)), int(rng.integers(8, 65))
        tw = float(10 ** rng.uniform(-2, 2))
        if kind == PLATE:
            sv = Solve(Q=37, geometry=PLATE, far=FAR_EQ, nx=nx, ny=ny, tau=tau_lb(tw, omega),
                       omega=omega, nsteps=steps, window_first=transient_periods * period,
                       window_count=window_periods * period, tau_omega=tw,
                       name=f"batch{k}_plate")
        else:
            x0, y0 = (nx - lx) // 2, (ny - ly) // 2
            sv = Solve(Q=37, geometry=BOX, far=FAR_EQ, nx=nx, ny=ny, tau=tau_lb(tw, omega),
                       omega=omega, box=(x0, y0, lx, ly), nsteps=steps,
                       window_first=transient_periods * period,
                       window_count=window_periods * period, tau_omega=tw,
                       name=f"batch{k}_box")
        out.append(sv)
    return out


def serving_trace(rate, count, seed=5, period=1024, transient_periods=10, window_periods=10,
                  box_n=1024, plate_ny=(1024, 8192)):
    """Poisson arrivals (rate per second) of requests: 1 box : 4 plates.
    Box requests are beam_box-like with log10(tau*omega) ~ U[-1, 1]; plate
    requests are 4 x U{plate_ny} thickness-shear plates, log10(tau*omega) ~
    U[-3, 3], stationary far wall.  Returns [(arrival_s, Solve)]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    omega = 2 * math.pi / period
    steps = (transient_periods + window_periods) * period
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        if rng.integers(0, 5) == 0:
            tw = float(10 ** rng.uniform(-1, 1))
            sv = beam_box(tw, n=box_n, period=period, transient_periods=transient_periods,
                          window_periods=window_periods)
            sv.name = f"req{k}_box"
        else:
            ny = int(rng.integers(plate_ny[0], plate_ny[1] + 1))
            tw = float(10 ** rng.uniform(-3, 3))
            sv = Solve(Q=37, geometry=PLATE, far=FAR_WALL, nx=4, ny=ny, tau=tau_lb(tw, omega),
                       omega=omega, nsteps=steps, window_first=transient_periods * period,
                       window_count=window_periods * period, tau_omega=tw,
                       name=f"req{k}_plate")
        out.append((t, sv))
    return out


def batch_parity_subsample(seed=40, count=256):
    """Indices into batch_sweep(count) of the seeded parity subsample: the
    solve with the fewest fluid cells, the one with the most, and two more
    drawn without replacement from the rest by PCG64(seed).  Returns
    (smallest, largest, [two drawn], sorted)."""
    solves = batch_sweep(count)
    cells = np.array([s.fluid_cells for s in solves])
    small, large = int(np.argmin(cells)), int(np.argmax(cells))
    rest = [i for i in range(count) if i not in (small, large)]
    rng = np.random.Generator(np.random.PCG64(seed))
    drawn = sorted(int(i) for i in rng.choice(rest, 2, replace=False))
    return small, large, drawn


def wide_plate(tau_omega, far, nx=64, ny=2048, period=1024, transient_periods=10,
               window_periods=10, storage="f32dev", wall="bb", accommodation=1.0):
    """D2Q37 plate wide enough (nx >= 64) to be kept as H2 coefficients, with
    the stationary far wall (far=FAR_WALL) or the rest-equilibrium far field
    (far=FAR_EQ): the plates of the batch sweep run this way.  wall: the
    moving wall's model ("bb", "ds" or "maxwell" with its accommodation)."""
    omega = 2 * math.pi / period
    steps = (transient_periods + window_periods) * period
    tag = "" if wall == "bb" else ("ds_" if wall == "ds" else f"{wall}{accommodation:g}_")
    return Solve(Q=37, geometry=PLATE, far=far, nx=nx, ny=ny, tau=tau_lb(tau_omega, omega),
                 omega=omega, nsteps=steps, window_first=transient_periods * period,
                 window_count=window_periods * period, storage=storage, tau_omega=tau_omega,
                 wall=wall, accommodation=accommodation,
                 name=f"wide_plate_{far}_{tag}tw{tau_omega:g}")


# --------------------------------------------------------------- noise

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea & Flood, OOPSLA 2014) applied
    to a uint64 array: z = x + golden gamma, then the two xor-shift-multiply
    rounds and a final xor-shift.  Wrapping 64-bit arithmetic."""
    z = (np.asarray(x, dtype=np.uint64) + np.uint64(0x9E3779B97F4A7C15)) & _M64
    z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & _M64
    z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & _M64
    return z ^ (z >> np.uint64(31))


def uniform_pm1(seed, n):
    """n draws from U[-1, 1): key k = seed xor index, top 53 bits of splitmix64(k)."""
    keys = np.arange(n, dtype=np.uint64) ^ np.uint64(seed)
    bits = splitmix64(keys) >> np.uint64(11)
    return bits.astype(np.float64) * (2.0 ** -52) - 1.0


def initial_noise(solve):
    """Noise added to the rest state, layout [q][y][x] float64.  Population
    (q, y, x) uses key seed xor ((y*nx + x)*Q + q); solid cells get 0."""
    Q, ny, nx = solve.Q, solve.ny, solve.nx
    u = uniform_pm1(solve.seed, Q * ny * nx).reshape(ny, nx, Q).transpose(2, 0, 1)
    out = np.ascontiguousarray(u * solve.noise)
    if solve.geometry == BOX:
        x0, y0, lx, ly = solve.box
        out[:, y0:y0 + ly, x0:x0 + lx] = 0.0
    return out


def random_state(Q, ny, nx, seed, amp):
    """Arbitrary perturbation field [q][y][x] (for parity tests), U[-amp, amp)."""
    return uniform_pm1(seed, Q * ny * nx).reshape(Q, ny, nx) * amp
