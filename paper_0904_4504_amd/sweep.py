"""Damping sweep and its device-level reading.

The paper characterises a resonator cross-section by the nondimensional
damping gamma_f / (rho sqrt(theta/2) S/m_o) as a function of tau*omega and
the aspect ratio AR = L_y / L_x (Sec. 6, eq. nems_W_tw).  On the lattice the
same quantity is R / (rho0 sqrt(theta/2) P), R the dissipative part of the
impedance per unit span and P the wetted length of the section (the plate:
one side of nx cells; a rectangle: its perimeter 2 (L_x + L_y)).

`run_sweep` computes it for plates (AR = 0) and rectangles (AR >= 1), each
with bounce-back and with diffuse walls, over a tau*omega grid in one batched
run.
`quality_factor` turns a damping curve into the quality factor of a
resonator immersed in nitrogen at pressure p (Sec. 6, the relation
Q = Q_o / (1 + rho sqrt(theta/2) S/(m_o gamma_o) gamma_bar)), with
tau = mu/p, rho = p/c_s^2 and the vacuum characteristics of Table 1.
`gamma_cylinder` is the Newtonian hydrodynamic function of an oscillating
cylinder (Sec. 3, eq. hydro_function), the comparator the paper quotes for
cross-sections of moderate aspect ratio at tau*omega << 1.

    python -m paper_0904_4504_amd.sweep [--period 1024] [--json out.json]
"""
import argparse
import json
import math
import os
import sys

import numpy as np

# Resonators of Table 1: vacuum resonance omega_o / 2 pi (Hz), Q_o, S/m_o
# (m^2/kg), aspect ratio AR = L_y / L_x.
TABLE1 = [
    {"name": "cantilever beam", "f0": 0.078e6, "Q0": 8320, "S_over_m": 688.0, "AR": 26},
    {"name": "cantilever beam (first harmonic)", "f0": 1.97e6, "Q0": 3520, "S_over_m": 405.0,
     "AR": 10},
    {"name": "doubly-clamped beam", "f0": 24.2e6, "Q0": 415, "S_over_m": 8380.0, "AR": 1},
    {"name": "quartz crystal disk", "f0": 32.7e6, "Q0": 40755, "S_over_m": 6.29, "AR": 0},
]

# Nitrogen at room temperature (Sec. 3): speed of sound and viscosity.
C_S = 298.0        # m/s
MU = 1.78e-5       # kg/(m s)
TAU_OMEGA_GRID = (0.001, 0.01, 0.1, 0.5, 1.0, 10.0)
TORR = 133.322368  # Pa


def gamma_bar(R, rho0, theta, perimeter):
    """Nondimensional damping R / (rho0 sqrt(theta/2) P) (eq. nems_W_tw)."""
    return R / (rho0 * math.sqrt(theta / 2.0) * perimeter)


def quality_factor(device, p, gbar):
    """Quality factor at pressure p (Pa) of a Table 1 device given the
    nondimensional damping gbar(tau_omega) of its cross-section."""
    omega0 = 2 * math.pi * device["f0"]
    tau = MU / p
    rho = p / (C_S * C_S)
    gamma0 = omega0 / device["Q0"]
    g = gbar(tau * omega0)
    return device["Q0"] / (1.0 + rho * (C_S / math.sqrt(2.0)) * device["S_over_m"] / gamma0 * g)


def interpolate(tau_omegas, values):
    """Damping curve through the sweep points, linear in log(tau*omega)
    (held constant beyond the ends)."""
    lt = np.log(np.asarray(tau_omegas, dtype=float))
    v = np.asarray(values, dtype=float)
    return lambda tw: float(np.interp(math.log(tw), lt, v))


def gamma_cylinder(beta):
    """Newtonian hydrodynamic function of an oscillating cylinder,
    Gamma = 1 + 4i K1(-i sqrt(i beta)) / (sqrt(i beta) K0(-i sqrt(i beta))),
    beta = omega r^2 / nu (eq. hydro_function)."""
    from scipy.special import kve  # exp(z) K_v(z): the ratio without underflow
    s = np.sqrt(1j * beta)
    return 1 + 4j * kve(1, -1j * s) / (s * kve(0, -1j * s))


def cylinder_impedance(rho0, omega, nu, r):
    """Z = R + iX per unit span of a cylinder of radius r from Gamma_cyl:
    the load i omega m Gamma u_hat (m = rho0 pi r^2, e^{-i omega t} phasors)
    is F = -(R u + (X/omega) du/dt) with R = omega m Im Gamma, X = omega m
    Re Gamma."""
    g = gamma_cylinder(omega * r * r / nu)
    m = rho0 * math.pi * r * r
    return complex(omega * m * g.imag, omega * m * g.real)


def sweep_solves(tau_omegas=TAU_OMEGA_GRID, period=1024, transient_periods=10,
                 window_periods=10, plate_ny=2048, box_n=1024, box_lx={1: 16, 10: 8, 26: 4}):
    """(Solve, AR, wall, wetted length) for every sweep point."""
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import lbm_inputs as W
    omega = 2 * math.pi / period
    steps = (transient_periods + window_periods) * period
    out = []
    for tw in tau_omegas:
        for wall in ("bb", "ds"):
            s = W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_EQ, nx=4, ny=plate_ny,
                        tau=W.tau_lb(tw, omega), omega=omega, nsteps=steps,
                        window_first=transient_periods * period,
                        window_count=window_periods * period, tau_omega=tw, wall=wall,
                        name=f"plate_{wall}_tw{tw:g}")
            out.append((s, 0, wall, s.nx))
        for ar, lx in sorted(box_lx.items()):
            ly = ar * lx
            for wall in ("bb", "ds"):
                s = W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=box_n, ny=box_n,
                            tau=W.tau_lb(tw, omega), omega=omega, nsteps=steps,
                            window_first=transient_periods * period,
                            window_count=window_periods * period, tau_omega=tw,
                            box=((box_n - lx) // 2, (box_n - ly) // 2, lx, ly), wall=wall,
                            name=f"box_ar{ar}_{wall}_tw{tw:g}")
                out.append((s, ar, wall, 2 * (lx + ly)))
    return out


def run_sweep(points, stream=None):
    """Advance every sweep point in one batch; returns one record per point
    with R, X and the nondimensional damping."""
    import torch
    from . import lbm as L
    stream = stream or torch.cuda.Stream()
    v, w, theta = L.lattice(37)
    recs = []
    with torch.cuda.stream(stream):
        solvers = [L.Solver(L.params_from_solve(s, loads=False), stream=stream)
                   for s, _, _, _ in points]
        batch = L.Batch(stream)
        try:
            for sv in solvers:
                batch.add(sv)
            batch.step(max(s.nsteps for s, _, _, _ in points))
            batch.synchronize()
            for (s, ar, wall, perim), sv in zip(points, solvers):
                z = sv.impedance()
                recs.append({"name": s.name, "AR": ar, "wall": wall, "tau_omega": s.tau_omega,
                             "R": z["R"], "X": z["X"], "perimeter": perim,
                             "gamma_bar": gamma_bar(z["R"], s.rho0, theta, perim)})
        finally:
            batch.close()
            for sv in solvers:
                sv.close()
    return recs


def device_curves(recs, pressures_torr=(0.1, 1, 10, 100, 1000)):
    """Q/Q_o of each Table 1 device at the given pressures from the sweep
    curve of its aspect ratio, with the diffuse wall (the model the paper
    compares with experiment) and with bounce-back."""
    out = []
    for dev in TABLE1:
        curves = {}
        for wall in ("ds", "bb"):
            pts = sorted((r["tau_omega"], r["gamma_bar"]) for r in recs
                         if r["AR"] == dev["AR"] and r["wall"] == wall)
            if pts:
                curves[wall] = interpolate([p[0] for p in pts], [p[1] for p in pts])
        for wall, g in curves.items():
            out.append({"device": dev["name"], "AR": dev["AR"], "wall": wall,
                        "Q_over_Q0": {str(pt): quality_factor(dev, pt * TORR, g) / dev["Q0"]
                                      for pt in pressures_torr}})
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--period", type=int, default=1024)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    import time
    import torch
    torch.cuda.set_device(0)
    pts = sweep_solves(period=a.period)
    t0 = time.perf_counter()
    recs = run_sweep(pts)
    wall = time.perf_counter() - t0
    out = {"points": recs, "devices": device_curves(recs),
           "solves": len(pts), "wall_s": wall,
           "glups": sum(s.fluid_cells * s.nsteps for s, _, _, _ in pts) / wall / 1e9}
    text = json.dumps(out)
    if a.json:
        with open(a.json, "w") as fh:
            fh.write(text)
    print(text, flush=True)


if __name__ == "__main__":
    main()
