"""The largest lattices the library accepts, where 32-bit offsets would
overflow if any were used for them: a plate with 2^29 cells kept as
populations (2 x 37 x 4 B per cell, 159 GB of state) and the plate whose
coefficient plane is the largest under 2 GiB (6 x 2 planes, 25.8 GB).
Neither fits the oracle; both are checked against properties that hold at
any size: the first-step force from rest (Sec. 6 moving wall, eq. BB) --
every population reaching the wall is at rest, so F_0 = -2 rho0 U_w(1/2)
n_x C_s exactly, with C_s = sum_{v_y < 0} w |v_y| v_x^2 / theta -- and, the
plate being uniform along x, the second step's force per unit length equals
the oracle's on a 4-cell-wide plate."""
import math

import numpy as np
import pytest

import lbm_inputs as W
import oracle as O

pytestmark = pytest.mark.gpu

C_S_37 = 0.290227505117714


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0904_4504_amd as P
    return P


def _first_step(P, s, representation):
    import torch
    torch.cuda.empty_cache()
    p = P.params_from_solve(s, representation=representation)
    print(f"case {s.nx}x{s.ny} repr {representation}: {P.required_bytes(p) / 1e9:.1f} GB",
          flush=True)
    with P.Solver(p) as sv:
        got = sv.representation
        sv.step(2)
        sv.synchronize()
        fx, fy = sv.force_history(0, 2)
    torch.cuda.empty_cache()
    return got, fx, fy


@pytest.mark.parametrize("nx,ny,repr_", [
    (16384, 32768, 1),   # 2^29 cells as populations
    (16384, 32767, 3),   # the largest coefficient plane under 2 GiB (FP32)
])
def test_maximum_size_first_step_force(P, nx, ny, repr_):
    om = 2 * math.pi / 1024
    s = W.Solve(Q=37, geometry=W.PLATE, far=W.FAR_EQ, nx=nx, ny=ny, tau=0.9, omega=om,
                u0=1e-3, nsteps=2, window_first=0, window_count=2, storage="f32dev",
                name=f"max_{nx}x{ny}")
    got, fx, fy = _first_step(P, s, repr_)
    assert got == (1 if repr_ == 1 else 2)
    expect = -2 * s.rho0 * s.u0 * math.sin(0.5 * om) * nx * C_S_37
    assert fx[0] == pytest.approx(expect, rel=1e-12)
    # step 1 per unit length against the oracle on a narrow copy of the plate
    narrow = O.OracleParams(Q=37, nx=4, ny=64, tau=s.tau, omega=om, u0=s.u0,
                            geometry=O.GEOM_PLATE, far=O.FAR_EQ)
    ox = O.run(narrow, 2)[0]
    assert fx[0] / nx == pytest.approx(ox[0] / 4, rel=1e-12)
    assert np.isfinite(fx[1]) and abs(fx[1] / nx - ox[1] / 4) <= 2e-5 * abs(ox[1] / 4)
