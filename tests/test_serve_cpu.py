"""Host logic of the serving loop (no GPU): admission by the HBM budget in
arrival order, device chunks that end at the next completion, retirement
and freeing, and the summary.  The library's solver and batch are replaced
by stand-ins that only count steps."""
import pytest

import lbm_inputs as W
from paper_0904_4504_amd import lbm as L
from paper_0904_4504_amd import serve as S


class _Solver:
    live = []

    def __init__(self, params, stream=None):
        self.max_steps = params.max_steps
        self.steps_done = 0
        self.bytes = L.required_bytes(params)
        _Solver.live.append(self)

    def impedance(self):
        return {"R": 1.0, "X": 2.0, "Z": complex(1.0, 2.0)}

    def close(self):
        _Solver.live.remove(self)


class _Batch:
    def __init__(self, stream=None):
        self.members = []
        self.chunks = []

    def add(self, sv):
        self.members.append(sv)

    def remove(self, sv):
        self.members.remove(sv)

    def step(self, n):
        left = min(sv.max_steps - sv.steps_done for sv in self.members)
        self.chunks.append((n, left))
        for sv in self.members:
            sv.steps_done = min(sv.max_steps, sv.steps_done + n)

    def synchronize(self):
        pass

    def close(self):
        pass


@pytest.fixture
def fakes(monkeypatch):
    batches = []

    def make_batch(stream=None):
        b = _Batch(stream)
        batches.append(b)
        return b

    monkeypatch.setattr(S.L, "Solver", _Solver)
    monkeypatch.setattr(S.L, "Batch", make_batch)
    _Solver.live = []
    return batches


def _trace(n, period=32):
    out = []
    for k, (t, s) in enumerate(W.serving_trace(1.0, n, period=period, box_n=96)):
        out.append((0.0, s.scaled(s.nsteps - 7 * k, s.window_count // 2)))
    return out


def test_admission_respects_the_budget_and_chunks_end_at_completions(fakes):
    trace = _trace(9)
    sizes = [L.required_bytes(L.params_from_solve(s, loads=False)) + 512 for _, s in trace]
    budget = max(sizes) + sorted(sizes)[-2]
    peak = []
    orig_add = _Batch.add

    def add(self, sv):
        orig_add(self, sv)
        peak.append(sum(m.bytes + 512 for m in self.members))

    _Batch.add = add
    try:
        reqs, summ = S.serve(trace, budget_bytes=budget, chunk=64, stream=object(),
                             clock=iter(range(10 ** 6)).__next__)
    finally:
        _Batch.add = orig_add
    assert summ["requests"] == 9 and len(reqs) == 9
    assert max(peak) <= budget
    assert _Solver.live == []  # every solver retired and freed
    b = fakes[0]
    assert all(n == min(64, left) for n, left in b.chunks)
    assert all(r.done >= r.admitted >= r.arrival for r in reqs)
    assert [r.rid for r in reqs] == list(range(9))
    assert 0 <= summ["host_fraction"] <= 1


def test_a_request_larger_than_the_budget_is_refused(fakes):
    trace = _trace(2)
    with pytest.raises(ValueError):
        S.serve(trace, budget_bytes=1000, chunk=64, stream=object())
