"""ctypes front end of the C oracle (lbm_oracle.c).

TEST INFRASTRUCTURE ONLY.  Arrays crossing this interface use the canonical
population layout [q][y][x] in float64 (q in the canonical velocity order:
orbits of the appendix table, members by polar angle).
"""
import ctypes as C
import dataclasses
import math
import os

import numpy as np

from . import build as _build

GEOM_PLATE, GEOM_BOX, GEOM_PERIODIC = 0, 1, 2
FAR_WALL, FAR_EQ = 0, 1
COLL_REGULARIZED, COLL_BGK = 0, 1
WALL_BB, WALL_DS, WALL_MAXWELL = 0, 1, 2


class _CParams(C.Structure):
    _fields_ = [
        ("Q", C.c_int), ("geometry", C.c_int), ("far", C.c_int), ("collision", C.c_int),
        ("nx", C.c_int), ("ny", C.c_int),
        ("box_x0", C.c_int), ("box_y0", C.c_int), ("box_lx", C.c_int), ("box_ly", C.c_int),
        ("tau", C.c_double), ("omega", C.c_double), ("u0", C.c_double), ("rho0", C.c_double),
        ("nthreads", C.c_int), ("wall", C.c_int), ("sigma", C.c_double),
    ]


@dataclasses.dataclass
class OracleParams:
    Q: int = 9
    geometry: int = GEOM_PLATE
    far: int = FAR_WALL
    collision: int = COLL_REGULARIZED
    nx: int = 4
    ny: int = 16
    box_x0: int = 0
    box_y0: int = 0
    box_lx: int = 0
    box_ly: int = 0
    tau: float = 0.8
    omega: float = 0.0
    u0: float = 0.0
    rho0: float = 1.0
    nthreads: int = 0
    wall: int = 0
    sigma: float = 1.0     # WALL_MAXWELL: accommodation, 0 specular .. 1 diffuse

    def c(self):
        return _CParams(**dataclasses.asdict(self))


_LIBS = {}


def _lib(variant):
    if variant not in _LIBS:
        path = _build.lib_path(variant)
        if not os.path.exists(path):
            _build.build(force=False)
        lib = C.CDLL(path)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
        lib.oracle_lattice.argtypes = [C.c_int, ip, ip, dp, C.POINTER(C.c_double)]
        lib.oracle_equilibrium.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, dp]
        lib.oracle_collide.argtypes = [C.c_int, C.c_int, C.c_double, dp, dp]
        lib.oracle_advect.argtypes = [C.POINTER(_CParams), dp, C.c_double, dp,
                                      C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.oracle_run.argtypes = [C.POINTER(_CParams), C.c_void_p, C.c_long, C.c_void_p,
                                   C.c_void_p, C.c_void_p]
        lib.oracle_lockin_fit.argtypes = [dp, C.c_long, C.c_long, C.c_double, C.c_double, dp]
        _LIBS[variant] = lib
    return _LIBS[variant]


def lattice(Q, variant="f64"):
    """(v[Q,2] int, w[Q] float64, theta) in canonical order."""
    vx = np.zeros(Q, np.int32)
    vy = np.zeros(Q, np.int32)
    w = np.zeros(Q)
    th = C.c_double()
    if _lib(variant).oracle_lattice(Q, vx, vy, w, C.byref(th)):
        raise ValueError(f"unknown lattice Q={Q}")
    return np.stack([vx, vy], 1), w, th.value


def equilibrium(Q, rho, ux, uy, variant="f64"):
    out = np.zeros(Q)
    if _lib(variant).oracle_equilibrium(Q, rho, ux, uy, out):
        raise ValueError(Q)
    return out


def collide(Q, fin, tau, collision=COLL_REGULARIZED, variant="f64"):
    fin = np.ascontiguousarray(fin, np.float64)
    out = np.zeros(Q)
    if _lib(variant).oracle_collide(Q, collision, tau, fin, out):
        raise ValueError(Q)
    return out


def advect(params, f, U, variant="f64"):
    """Advection + boundaries only.  Returns (f_adv, Fx, Fy)."""
    f = np.ascontiguousarray(f, np.float64)
    out = np.zeros_like(f)
    fx, fy = C.c_double(), C.c_double()
    cp = params.c()
    if _lib(variant).oracle_advect(C.byref(cp), f, U, out, C.byref(fx), C.byref(fy)):
        raise ValueError("oracle_advect rejected the parameters")
    return out, fx.value, fy.value


def run(params, nsteps, f0=None, want_state=False, variant="f64"):
    """Run nsteps steps.  Returns (Fx[n], Fy[n], f_final or None)."""
    shape = (params.Q, params.ny, params.nx)
    if f0 is not None:
        f0 = np.ascontiguousarray(f0, np.float64)
        if f0.shape != shape:
            raise ValueError(f"f0 shape {f0.shape} != {shape}")
    fx = np.zeros(nsteps)
    fy = np.zeros(nsteps)
    fin = np.zeros(shape) if want_state else None
    cp = params.c()
    rc = _lib(variant).oracle_run(
        C.byref(cp), None if f0 is None else f0.ctypes.data, nsteps, fx.ctypes.data,
        fy.ctypes.data, None if fin is None else fin.ctypes.data)
    if rc:
        raise ValueError(f"oracle_run rejected the parameters ({rc})")
    return fx, fy, fin


def lockin_fit(F, first, count, omega, u0):
    """Fit F_n ~ a sin + b cos + c over the window.  Returns dict a, b, c, R, X, Z."""
    F = np.ascontiguousarray(F, np.float64)
    if first < 0 or first + count > F.size:
        raise ValueError("window outside the force series")
    out = np.zeros(5)
    if _lib("ld").oracle_lockin_fit(F, first, count, omega, u0, out):
        raise ValueError("singular lock-in system")
    a, b, c, R, X = out
    return {"a": a, "b": b, "c": c, "R": R, "X": X, "Z": complex(R, X),
            "absZ": math.hypot(R, X), "phase": math.atan2(X, R)}
