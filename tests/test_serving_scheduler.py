"""Serving scheduler (continuous batching) on a simulated device: admission by
HBM footprint, arrival order, slot limit, completion and latency statistics.
No GPU: a fake executor models each request as a fixed-duration job."""
import numpy as np
import pytest

from paper_2505_02438_amd import serving as S


class FakeExecutor:
    """Simulated clock; a request runs for n_cells / rate seconds from launch."""

    def __init__(self, rate=1e8, tick=1e-6):
        self.t, self.rate, self.tick = 0.0, rate, tick
        self.running = {}
        self.max_concurrent = 0
        self.log = []

    def now(self):
        self.t += self.tick
        return self.t

    def wait_until(self, t):
        self.t = max(self.t, t)

    def launch(self, req, slot):
        assert slot not in [s for (s, _) in self.running.values()], "slot reused while busy"
        self.running[req.rid] = (slot, self.t + req.n_cells / self.rate)
        self.max_concurrent = max(self.max_concurrent, len(self.running))
        self.log.append(("launch", req.rid, self.t))
        return req.rid

    def done(self, h):
        return self.t >= self.running[h][1]

    def wait(self, h):
        self.t = max(self.t, self.running[h][1])

    def finish(self, h):
        self.running.pop(h)
        self.log.append(("finish", h, self.t))
        return f"dc{h}", f"c{h}"


def _reqs(count=64, rate=None):
    return S.make_requests(count, rate_elems_per_s=rate)


def test_all_requests_complete_with_their_outputs():
    reqs = _reqs(40, rate=5e7)
    ex = FakeExecutor()
    res = S.Scheduler(ex, slots=4, hbm_budget=8 << 30).run(reqs)
    assert [r.rid for r in res] == sorted(r.rid for r in reqs)
    assert all(r.dc == f"dc{r.rid}" and r.c == f"c{r.rid}" for r in res)
    assert all(r.finish >= r.start >= r.arrival for r in res)


@pytest.mark.parametrize("budget_gb", [2, 4, 32])
def test_admission_never_exceeds_hbm_budget(budget_gb):
    reqs = _reqs(80)  # burst: everything arrives at t = 0
    ex = FakeExecutor()
    sch = S.Scheduler(ex, slots=8, hbm_budget=budget_gb << 30)
    sch.run(reqs)
    assert max(b for _, b in sch.admission_log) <= budget_gb << 30
    assert sch.in_use == 0 and sorted(sch.free_slots) == list(range(8))


def test_admission_in_arrival_order_and_slot_limit():
    reqs = _reqs(60, rate=2e8)
    ex = FakeExecutor()
    sch = S.Scheduler(ex, slots=3, hbm_budget=32 << 30)
    sch.run(reqs)
    order = [rid for rid, _ in sch.admission_log]
    by_arrival = [r.rid for r in sorted(reqs, key=lambda r: (r.arrival, r.rid))]
    assert order == by_arrival
    assert ex.max_concurrent <= 3


def test_work_overlaps_when_slots_allow():
    reqs = _reqs(16)
    ex = FakeExecutor()
    S.Scheduler(ex, slots=4, hbm_budget=64 << 30).run(reqs)
    assert ex.max_concurrent == 4


def test_request_larger_than_budget_is_rejected():
    reqs = [S.Request(0, "hex", 96, 3.0)]
    with pytest.raises(ValueError):
        S.Scheduler(FakeExecutor(), slots=2, hbm_budget=1 << 30).run(reqs)


def test_footprint_counts_csr_values():
    # K values dominate: 9 (3n+1)^3 doubles for an n^3 hex grid
    fp = S.request_footprint("hex", 96)
    assert 9 * 289 ** 3 * 8 < fp < 9 * 289 ** 3 * 8 * 1.1
    assert S.request_footprint("quad", 32) > 4 * 97 ** 2 * 8


def test_make_requests_seeded_and_poisson():
    a = _reqs(100, rate=1e8)
    b = _reqs(100, rate=1e8)
    assert [(r.kind, r.n, r.p, r.arrival) for r in a] == [(r.kind, r.n, r.p, r.arrival) for r in b]
    t = np.array([r.arrival for r in a])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    mean_elems = np.mean([r.n_cells for r in a])
    assert 0.5 < (t[-1] / 99) / (mean_elems / 1e8) < 2.0  # mean gap ~ mean work / rate
    assert {r.kind for r in a} == {"quad", "hex"} and {r.p for r in a} <= {3.0, 4.0}


def test_latency_stats():
    res = [S.Result(i, 100, 0.0, 0.0, (i + 1) * 1e-3) for i in range(100)]
    st = S.latency_stats(res)
    assert abs(st["p50_ms"] - 50.5) < 1e-9 and abs(st["p99_ms"] - 99.01) < 1e-9
    assert abs(st["elements_per_s"] - 100 * 100 / 0.1) < 1e-6
