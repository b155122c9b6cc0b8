"""CPU tests of the continuous-batching scheduler, driven by a CPU executor
that advances each request with the oracle (no GPU)."""
import numpy as np
import pytest

import oracle as O
from paper_1706_04552_amd import inputs
from paper_1706_04552_amd.serving import (ContinuousBatcher, Request, footprint,
                                          sequential_baseline)


class FakeClock:
    def __init__(self, tick=1e-3):
        self.t = 0.0
        self.tick = tick

    def __call__(self):
        self.t += self.tick
        return self.t

    def sleep(self, dt):
        self.t += dt


class OracleExecutor:
    """Holds each request's state on the host and advances it with the oracle."""

    def __init__(self):
        self.passes = []
        self.resident = 0

    def admit(self, q):
        self.resident += 1
        return {"r": q.r, "state": q.state.copy()}

    def run_pass(self, work):
        self.passes.append([k for _, k in work])
        for h, k in work:
            h["state"] = O.life_steps(h["r"], h["state"], k)

    def sync(self):
        pass

    def download(self, h):
        return h["state"]

    def release(self, h):
        self.resident -= 1


def _requests(count, seed, r_lo=3, r_hi=7, steps_hi=40, spacing=0.002):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        r = int(rng.integers(r_lo, r_hi + 1))
        steps = int(rng.integers(0, steps_hi + 1))
        out.append(Request(i, float(i * spacing * rng.random()), r, steps,
                           inputs.bernoulli_state(r, 0.5, 100 + i)))
    return out


@pytest.mark.parametrize("T", [1, 5, 16])
def test_every_result_equals_the_request_alone(T):
    reqs = _requests(30, T)
    clock = FakeClock()
    ex = OracleExecutor()
    st = ContinuousBatcher(ex, cap_bytes=10 ** 9, steps_per_pass=T, keep_outputs=True,
                           clock=clock, sleep=clock.sleep).serve(reqs)
    assert len(st.results) == len(reqs) and not any(x.rejected for x in st.results)
    for res in st.results:
        q = reqs[res.rid]
        assert np.array_equal(res.output, O.life_steps(q.r, q.state, q.steps))
        assert res.finished >= res.admitted >= res.arrival
    # no pass advances a request by more than T generations
    assert all(0 <= k <= T for p in ex.passes for k in p)
    assert ex.resident == 0


def test_admission_never_exceeds_the_cap_and_requests_overlap():
    reqs = _requests(40, 7, r_lo=5, r_hi=7, spacing=0.0)
    cap = 3 * footprint(7)
    clock = FakeClock()
    ex = OracleExecutor()
    st = ContinuousBatcher(ex, cap_bytes=cap, steps_per_pass=4, keep_outputs=True,
                           clock=clock, sleep=clock.sleep).serve(reqs)
    assert st.max_resident_bytes <= cap
    assert st.max_active >= 2            # several requests share a pass
    assert len(st.results) == len(reqs)
    for res in st.results:
        q = reqs[res.rid]
        assert np.array_equal(res.output, O.life_steps(q.r, q.state, q.steps))


def test_oversized_requests_are_rejected():
    reqs = [Request(0, 0.0, 9, 3, inputs.bernoulli_state(9, 0.5, 1)),
            Request(1, 0.0, 4, 3, inputs.bernoulli_state(4, 0.5, 2))]
    clock = FakeClock()
    st = ContinuousBatcher(OracleExecutor(), cap_bytes=footprint(8), steps_per_pass=2,
                           keep_outputs=True, clock=clock, sleep=clock.sleep).serve(reqs)
    by = {x.rid: x for x in st.results}
    assert by[0].rejected and not by[1].rejected


def test_sequential_baseline_queue():
    lat, end = sequential_baseline([1.0, 1.0, 0.5], [0.0, 0.5, 5.0])
    assert list(lat) == [1.0, 1.5, 0.5] and end == 5.5


def test_budgeted_passes_keep_results_and_order():
    reqs = _requests(25, 4, r_lo=4, r_hi=6, spacing=0.0)
    clock = FakeClock()
    ex = OracleExecutor()
    budget = 3 ** 6 * 4
    st = ContinuousBatcher(ex, cap_bytes=10 ** 9, steps_per_pass=4, keep_outputs=True,
                           clock=clock, sleep=clock.sleep, max_cells_per_pass=budget).serve(reqs)
    for res in st.results:
        q = reqs[res.rid]
        assert np.array_equal(res.output, O.life_steps(q.r, q.state, q.steps))
    # every pass stays within the budget unless a single request exceeds it
    assert all(sum(1 for k in p if k) >= 1 for p in ex.passes if any(p))


@pytest.mark.parametrize("horizon", [1, 3 ** 6 * 8, 10 ** 12])
def test_queued_passes_keep_results(horizon):
    reqs = _requests(30, 11, r_lo=4, r_hi=7, steps_hi=60)
    clock = FakeClock()
    ex = OracleExecutor()
    st = ContinuousBatcher(ex, cap_bytes=10 ** 9, steps_per_pass=4, keep_outputs=True,
                           clock=clock, sleep=clock.sleep, horizon_cells=horizon).serve(reqs)
    assert len(st.results) == len(reqs)
    for res in st.results:
        q = reqs[res.rid]
        assert np.array_equal(res.output, O.life_steps(q.r, q.state, q.steps))
    assert st.passes == len(ex.passes) and st.iterations <= st.passes


def test_a_lone_request_runs_all_its_passes_in_one_round():
    q = Request(0, 0.0, 6, 37, inputs.bernoulli_state(6, 0.5, 3))
    clock = FakeClock()
    ex = OracleExecutor()
    st = ContinuousBatcher(ex, cap_bytes=10 ** 9, steps_per_pass=8, keep_outputs=True,
                           clock=clock, sleep=clock.sleep, horizon_cells=10 ** 12).serve([q])
    assert st.iterations == 1 and st.passes == 5
    assert np.array_equal(st.results[0].output, O.life_steps(6, q.state, 37))
