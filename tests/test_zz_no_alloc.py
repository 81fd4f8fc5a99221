"""The allocation-free entry point lbm_create_static against lbm_create_in.

A solver created in the library's static scratch array runs the same kernels
on the same layout as one created in a caller's buffer, so its forces,
impedance and final state are bit-identical.  Two creations in a row (the
second with a smaller lattice) check that nothing from the first run leaks
into the second; oversize parameters and a second live static solver are
rejected with LBM_ESCRATCH.
"""
import ctypes as C
import math

import numpy as np
import pytest

import lbm_inputs as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_0904_4504_amd as P
    return P


def _box(nx, ny, box, tw, nsteps):
    om = 2 * math.pi / 64
    return W.Solve(Q=37, geometry=W.BOX, far=W.FAR_EQ, nx=nx, ny=ny,
                   tau=W.tau_lb(tw, om), omega=om, box=box, nsteps=nsteps,
                   window_first=nsteps // 2, window_count=nsteps - nsteps // 2,
                   name=f"static_box_{nx}x{ny}")


def _run(P, s, memory):
    print(f"case {s.name} memory={memory} steps={s.nsteps}", flush=True)
    with P.Solver(P.params_from_solve(s), memory=memory) as sv:
        sv.step(s.nsteps)
        sv.synchronize()
        fx, fy = sv.force_history(0, s.nsteps)
        z = sv.impedance()
        state = sv.get_state()
        repr_ = sv.representation
    return fx, fy, z, state, repr_


@pytest.mark.parametrize("storage", ["f32dev", "f64"])
def test_static_matches_caller_buffer_twice(P, storage):
    import dataclasses
    big = dataclasses.replace(_box(320, 192, (140, 88, 32, 16), 1.0, 96), storage=storage)
    small = dataclasses.replace(_box(128, 96, (50, 40, 20, 12), 0.3, 80), storage=storage)
    for s in (big, small):
        assert P.required_bytes(P.params_from_solve(s)) <= P.lbm.STATIC_SCRATCH_BYTES
        ref = _run(P, s, "torch")
        got = _run(P, s, "static")
        assert got[4] == ref[4] == P.lbm.REPR_COEFFICIENTS
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1])
        assert got[2]["Z"] == ref[2]["Z"]
        assert np.array_equal(got[3], ref[3])
        assert np.max(np.abs(ref[0])) > 0


def test_static_rejects_oversize_and_second_live_solver(P):
    big = _box(2048, 2048, (1000, 1000, 32, 16), 1.0, 8)
    assert P.required_bytes(P.params_from_solve(big)) > P.lbm.STATIC_SCRATCH_BYTES
    with pytest.raises(P.LbmError) as e:
        P.Solver(P.params_from_solve(big), memory="static")
    assert e.value.code == P.lbm.ESCRATCH
    s = _box(128, 96, (50, 40, 20, 12), 0.3, 16)
    with P.Solver(P.params_from_solve(s), memory="static") as first:
        with pytest.raises(P.LbmError) as e:
            P.Solver(P.params_from_solve(s), memory="static")
        assert e.value.code == P.lbm.ESCRATCH
        first.step(16)
        first.synchronize()
    # released by lbm_destroy: usable again
    with P.Solver(P.params_from_solve(s), memory="static") as again:
        again.step(16)
        again.synchronize()
