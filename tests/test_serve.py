"""Serving loop scheduling (CPU, fake executor on a virtual clock): FIFO
admission by HBM footprint, launch-slot limits, continuous batching of requests
that arrive while slots are busy, plan-table accounting, latency report."""
import numpy as np
import pytest

from paper_1003_4984_amd.serve import (Request, Server, PlanCache, report, BYTES_PER_SAMPLE, TABLE_BYTES_BOUND,
                                       BATCH_BYTES_BOUND, TQU_CHUNK)


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeExecutor:
    """Completes a group after 1 ms per 1000 samples; records concurrency."""

    def __init__(self, clock):
        self.clock = clock
        self.live = {}
        self.max_live = 0
        self.groups = []

    def launch(self, group, slot):
        assert slot not in self.live
        dur = 1e-3 * sum(r.samples for r in group) / 1000.0
        self.live[slot] = self.clock() + dur
        self.max_live = max(self.max_live, len(self.live))
        self.groups.append([r.rid for r in group])
        return (slot, self.clock() + dur)

    def done(self, token):
        slot, t_end = token
        if self.clock() >= t_end:
            self.live.pop(slot, None)
            return True
        return False


def _reqs(arrivals, ns, fields="T"):
    return [Request(rid=i, arrival=a, nside=16, lmax=16, K=8, fields=fields, n=n,
                    cl_tt=np.ones(17)) for i, (a, n) in enumerate(zip(arrivals, ns))]


def _serve(reqs, budget, slots, plans=None):
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, budget, slots, plans, clock=clock)

    def idle():
        clock.t += 1e-4
    done = srv.run(reqs, idle=idle)
    return srv, ex, done, clock


def test_all_served_fifo_and_latency():
    reqs = _reqs([0.0, 0.001, 0.002, 0.010, 0.011], [2000, 3000, 1000, 4000, 500])
    srv, ex, done, clock = _serve(reqs, budget=10 ** 9, slots=2)
    assert sorted(r.rid for r in done) == list(range(5))
    adm = [r.admitted for r in sorted(done, key=lambda r: r.rid)]
    assert all(a <= b for a, b in zip(adm, adm[1:]))          # first come first admitted
    for r in done:
        assert r.arrival <= r.admitted <= r.finished
    rep = report(done, clock.t)
    assert rep["requests"] == 5 and rep["samples"] == sum(r.samples for r in reqs)
    assert rep["latency_p50_s"] <= rep["latency_p99_s"]


def test_budget_and_slots_respected():
    ns = [5000] * 12
    reqs = _reqs(np.linspace(0, 0.002, 12), ns)
    budget = 2 * reqs[0].footprint()               # two requests in flight at most
    srv, ex, done, _ = _serve(reqs, budget=budget, slots=3)
    assert len(done) == 12
    assert srv.peak <= budget
    assert ex.max_live <= 3


def test_continuous_batching_groups_waiting_requests():
    # one long request holds the only slot; the ones arriving meanwhile are
    # admitted together when it completes
    reqs = _reqs([0.0, 0.0005, 0.0006, 0.0007], [50000, 100, 100, 100])
    srv, ex, done, _ = _serve(reqs, budget=10 ** 9, slots=1)
    assert ex.groups[0] == [0]
    assert ex.groups[1] == [1, 2, 3]


def test_request_over_budget_rejected():
    reqs = _reqs([0.0], [10 ** 6])
    with pytest.raises(ValueError):
        _serve(reqs, budget=1000, slots=1)


def test_new_plan_tables_count_against_budget():
    made = []
    plans = PlanCache(lambda *a: made.append(a) or object())
    r = _reqs([0.0], [100], fields="TQU")[0]
    r.cl_ee, r.cl_bb = np.ones(17), np.zeros(17)
    assert plans.missing(r) == 2
    maps = 8 * 12 * 16 * 16 * 3                      # T, Q, U at N_side 16
    stencils = 4 * 8 * 100                           # K int32 per target for the shared search
    assert r.footprint(plans.missing(r)) == (maps + 16 * 100 + 3 * 100 * BYTES_PER_SAMPLE + stencils
                                             + BATCH_BYTES_BOUND + 2 * TABLE_BYTES_BOUND)
    plans.get(16, 16, 8, 0, r.cl_tt)
    assert plans.missing(r) == 1 and len(plans) == 1
    plans.get(16, 16, 8, 0, r.cl_tt)
    assert len(made) == 1


def test_group_cap_splits_launches():
    reqs = _reqs([0.0, 0.0001, 0.0002, 0.0003], [50000, 3000, 3000, 3000])
    clock = Clock()
    ex = FakeExecutor(clock)
    srv = Server(ex, 10 ** 9, 1, None, clock=clock, max_group_samples=5000)

    def idle():
        clock.t += 1e-4
    done = srv.run(reqs, idle=idle)
    assert len(done) == 4
    assert ex.groups == [[0], [1], [2], [3]]


def test_tqu_footprint_counts_stencil_buffer():
    """The stencil buffer of the shared-search T+Q+U call is K int32 per target
    of one 2^24-target chunk; without the shared call it is not needed."""
    r = Request(rid=0, arrival=0.0, nside=4096, lmax=4096, K=32, fields="TQU", n=12 * 4096 ** 2)
    base = 8 * 12 * 4096 ** 2 * 3 + 16 * r.n + r.samples * BYTES_PER_SAMPLE + BATCH_BYTES_BOUND
    assert r.footprint(0, tqu_shared=True) == base + 4 * 32 * TQU_CHUNK
    assert r.footprint(0, tqu_shared=False) == base
    t = Request(rid=1, arrival=0.0, nside=4096, lmax=4096, K=32, fields="T", n=1000)
    assert t.footprint(0, True) == t.footprint(0, False)


def test_admission_waits_while_memory_is_held():
    """Budget for one request at a time: the second is refused while the first
    holds its memory and is admitted only after the first has completed."""
    reqs = _reqs([0.0, 0.0001], [5000, 5000])
    budget = int(1.5 * reqs[0].footprint())
    srv, ex, done, _ = _serve(reqs, budget=budget, slots=2)
    a, b = sorted(done, key=lambda r: r.rid)
    assert b.admitted >= a.finished
    assert srv.peak <= budget and ex.max_live == 1


def test_server_sleeps_instead_of_spinning():
    """With no idle hook the loop yields through its sleep function while it
    waits for an arrival or a completion."""
    clock = Clock()
    ex = FakeExecutor(clock)
    slept = []

    def sleep(dt):
        slept.append(dt)
        clock.t += max(dt, 1e-5)

    srv = Server(ex, 10 ** 9, 1, None, clock=clock, sleep=sleep)
    done = srv.run(_reqs([0.0, 0.05], [1000, 1000]))
    assert len(done) == 2 and slept and all(0.0 <= d <= 1e-3 for d in slept)
