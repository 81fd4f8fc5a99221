"""Seeded workload generators: shapes, ranges and reproducibility."""
import math

import numpy as np

import lbm_inputs as W


def test_stokes_plate_matches_its_definition():
    s = W.stokes_plate()
    nu = (s.tau - 0.5) / 3
    assert math.sqrt(2 * nu / s.omega) == 16.0
    assert (s.nx, s.ny, s.nsteps, s.window_count) == (4, 256, 160850, 80425)
    assert s.window_first + s.window_count == s.nsteps


def test_plate_sweep_relaxation_times():
    for tw in W.PLATE_SWEEP_TAU_OMEGA:
        s = W.plate_sweep(tw)
        assert (s.tau - 0.5) * s.omega == np.float64(tw) or abs((s.tau - 0.5) * s.omega - tw) < 1e-12
        assert s.nsteps == 30 * 1024 and s.window_count == 10 * 1024


def test_beam_box_is_centred_and_y_symmetric():
    s = W.beam_box(1.0)
    x0, y0, lx, ly = s.box
    assert (lx, ly) == (32, 16)
    assert x0 + lx + x0 == s.nx and y0 + ly + y0 == s.ny
    assert s.fluid_cells == 1024 * 1024 - 512


def test_noise_is_reproducible_and_uniform():
    s = W.stokes_plate()
    a = W.initial_noise(s)
    b = W.initial_noise(s)
    assert np.array_equal(a, b)
    assert a.shape == (9, 256, 4)
    assert np.max(np.abs(a)) < 1e-9 and np.min(a) >= -1e-9
    assert abs(a.mean()) < 2e-11
    u = W.uniform_pm1(0, 200000)
    assert abs(u.mean()) < 0.01 and abs(u.var() - 1 / 3) < 0.01


def test_splitmix64_reference_values():
    # SplitMix64 from state 0: the first outputs of the published generator
    out = W.splitmix64(np.array([0, 0x9E3779B97F4A7C15], dtype=np.uint64))
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4


def test_batch_sweep_ranges():
    solves = W.batch_sweep()
    assert len(solves) == 256
    assert solves[0].name == W.batch_sweep()[0].name  # reproducible
    kinds = {s.geometry for s in solves}
    assert kinds == {W.PLATE, W.BOX}
    for s in solves:
        short, long_ = sorted((s.nx, s.ny))
        assert 256 <= short and long_ <= 2048
        assert long_ % short == 0 and long_ // short in (1, 2, 4)
        assert 1e-2 <= s.tau_omega <= 1e2
        if s.geometry == W.BOX:
            assert 8 <= s.box[2] <= 64 and 8 <= s.box[3] <= 64


def test_serving_trace_rate_and_mix():
    tr = W.serving_trace(rate=4.0, count=2000)
    t = np.array([a for a, _ in tr])
    assert np.all(np.diff(t) > 0)
    assert abs(len(t) / t[-1] - 4.0) < 0.3
    boxes = sum(s.geometry == W.BOX for _, s in tr)
    assert abs(boxes / len(tr) - 0.2) < 0.03
    for _, s in tr:
        if s.geometry == W.PLATE:
            assert s.nx == 4 and 1024 <= s.ny <= 8192
            assert 1e-3 <= s.tau_omega <= 1e3
