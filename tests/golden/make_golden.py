"""Write the stored oracle results used by the GPU parity tests.

Calls only the CPU oracle (and the seeded workload definitions).  Each case
is written to tests/golden/<case>.json with the workload parameters, the
lock-in fit (a, b, c, R, X) and the force series sampled every `stride`
steps plus the last 64 steps in full.

  python tests/golden/make_golden.py stokes_plate          # D2Q9 4x256, 160 850 steps
  python tests/golden/make_golden.py plate_sweep           # D2Q37 4x2048, 5 tau*omega
  python tests/golden/make_golden.py beam_box [tw ...]     # D2Q37 1024^2 box, hours
  python tests/golden/make_golden.py batch_subsample       # seeded 4 of the 256-solve batch
  python tests/golden/make_golden.py wide_plate            # 64x2048 plates, tau*omega 0.01, 100
  python tests/golden/make_golden.py wide_plate_walls      # the same with diffuse, Maxwell walls
  python tests/golden/make_golden.py wall_box              # 256^2 box, diffuse and specular faces,
                                                           # tau*omega 0.01, 1, 100
  options: --threads N

The batch subsample runs each drawn solve for its full 20 480 steps, except
the largest (2026 x 2026 cells), which runs 4 periods (4096 steps, lock-in
over the last 2): at the oracle's few MLUPS a full run takes hours.
"""
import argparse
import dataclasses
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import lbm_inputs as W  # noqa: E402
import oracle as O  # noqa: E402


# run length of the largest solve of the batch subsample (4 periods)
LARGEST_STEPS = 4096


def oracle_params(s, threads):
    return O.OracleParams(
        Q=s.Q, nx=s.nx, ny=s.ny, tau=s.tau, omega=s.omega, u0=s.u0, rho0=s.rho0,
        geometry={W.PLATE: O.GEOM_PLATE, W.BOX: O.GEOM_BOX, W.PERIODIC: O.GEOM_PERIODIC}[s.geometry],
        far=O.FAR_WALL if s.far == W.FAR_WALL else O.FAR_EQ,
        collision=O.COLL_REGULARIZED if s.collision == "regularized" else O.COLL_BGK,
        box_x0=s.box[0], box_y0=s.box[1], box_lx=s.box[2], box_ly=s.box[3], nthreads=threads,
        wall={"bb": O.WALL_BB, "ds": O.WALL_DS, "maxwell": O.WALL_MAXWELL}[s.wall],
        sigma=s.accommodation)


def run_case(s, variant, threads, stride):
    p = oracle_params(s, threads)
    v, w, th = O.lattice(s.Q, variant)
    f0 = None
    if s.noise:
        f0 = w[:, None, None] * s.rho0 + W.initial_noise(s)
    t0 = time.time()
    fx, fy, _ = O.run(p, s.nsteps, f0=f0, variant=variant)
    dt = time.time() - t0
    z = O.lockin_fit(fx, s.window_first, s.window_count, s.omega, s.u0)
    zy = O.lockin_fit(fy, s.window_first, s.window_count, s.omega, s.u0)
    idx = sorted(set(range(0, s.nsteps, stride)) | set(range(max(0, s.nsteps - 64), s.nsteps)))
    return {
        "solve": {k: (list(v) if isinstance(v, tuple) else v)
                  for k, v in dataclasses.asdict(s).items()},
        "variant": variant,
        "seconds": dt,
        "threads": threads,
        "fit": {k: z[k] for k in ("a", "b", "c", "R", "X")},
        "fit_y": {k: zy[k] for k in ("a", "b", "c")},
        "max_abs_fx": float(np.max(np.abs(fx))),
        "max_abs_fy": float(np.max(np.abs(fy))),
        "samples": {"step": idx, "fx": [float(fx[i]) for i in idx],
                    "fy": [float(fy[i]) for i in idx]},
    }


def write(name, obj):
    path = os.path.join(HERE, name + ".json")
    with open(path, "w") as fh:
        json.dump(obj, fh, indent=1)
    print("wrote", path, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("case", choices=["stokes_plate", "plate_sweep", "beam_box", "batch_subsample",
                                     "wide_plate", "wide_plate_walls", "wall_box"])
    ap.add_argument("tau_omega", nargs="*", type=float)
    ap.add_argument("--threads", type=int, default=0)
    a = ap.parse_args()
    if a.case == "stokes_plate":
        s = W.stokes_plate()
        out = {"f64": run_case(s, "f64", a.threads, 101), "ld": run_case(s, "ld", a.threads, 101)}
        write("stokes_plate", out)
    elif a.case == "plate_sweep":
        for tw in a.tau_omega or W.PLATE_SWEEP_TAU_OMEGA:
            s = W.plate_sweep(tw, storage="f64")
            write(f"plate_sweep_tw{tw:g}", run_case(s, "f64", a.threads, 97))
    elif a.case == "batch_subsample":
        small, large, drawn = W.batch_parity_subsample()
        solves = W.batch_sweep()
        for i in [small] + drawn + [large]:
            s = dataclasses.replace(solves[i], storage="f64")
            if i == large:
                s = s.scaled(LARGEST_STEPS, LARGEST_STEPS // 2)
            out = run_case(s, "f64", a.threads, 97)
            out["batch_index"] = i
            write(f"batch_{i}", out)
    elif a.case == "wide_plate":
        for far in (W.FAR_WALL, W.FAR_EQ):
            for tw in a.tau_omega or (0.01, 100.0):
                s = W.wide_plate(tw, far, storage="f64")
                write(s.name, run_case(s, "f64", a.threads, 97))
    elif a.case == "wide_plate_walls":
        for tw in a.tau_omega or (0.01, 100.0):
            for wall, sigma in (("ds", 1.0), ("maxwell", 0.6)):
                s = W.wide_plate(tw, W.FAR_EQ, storage="f64", wall=wall, accommodation=sigma)
                write(s.name, run_case(s, "f64", a.threads, 97))
    elif a.case == "wall_box":
        for tw in a.tau_omega or (0.01, 1.0, 100.0):
            for wall, sigma in (("ds", 1.0), ("maxwell", 0.0)):
                s = W.wall_box(tw, wall, sigma, storage="f64")
                write(s.name, run_case(s, "f64", a.threads, 97))
    else:
        for tw in a.tau_omega or W.BEAM_TAU_OMEGA:
            s = W.beam_box(tw, storage="f64")
            write(f"beam_box_tw{tw:g}", run_case(s, "f64", a.threads, 97))


if __name__ == "__main__":
    main()
