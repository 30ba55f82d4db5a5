"""Host logic of the continuous-batching server, driven by a fake executor."""

import threading
import time

from paper_2304_08159_amd.serving import Executor, Request, Server, make_requests, summarize


class FakeExecutor(Executor):
    def __init__(self, unit_s=0.002):
        self.unit = unit_s
        self.lock = threading.Lock()
        self.active = 0
        self.peak = 0
        self.bytes = 0
        self.peak_bytes = 0
        self.order = []

    def footprint(self, r):
        c = 1
        for m in r.n:
            c *= m
        return c * 100

    def run(self, r):
        with self.lock:
            self.active += 1
            self.bytes += r.footprint
            self.peak = max(self.peak, self.active)
            self.peak_bytes = max(self.peak_bytes, self.bytes)
            self.order.append(r.id)
        time.sleep(self.unit * (1 + sum(r.n) / 256))
        if r.kind == "boom":
            with self.lock:
                self.active -= 1
                self.bytes -= r.footprint
            raise RuntimeError("planted failure")
        with self.lock:
            self.active -= 1
            self.bytes -= r.footprint
        return ("ok", r.id)


def test_all_requests_complete_within_budget_and_slots():
    ex = FakeExecutor()
    reqs = make_requests(count=60, seed=1, rate=2000.0)
    budget = 2 * 128 ** 3 * 100          # two of the largest requests at most
    srv = Server(ex, budget, slots=4)
    out = srv.run(reqs)
    s = summarize(out)
    assert s["done"] == 60 and s["failed"] == 0 and s["rejected"] == 0
    assert ex.peak <= 4 and ex.peak_bytes <= budget
    for r in out:
        assert r.arrival <= r.admitted + 1e-9 <= r.done + 1e-9
    assert s["p50_ms"] <= s["p99_ms"]


def test_overlap_happens_and_fifo_for_equal_sizes():
    ex = FakeExecutor(unit_s=0.01)
    reqs = [Request(id=k, kind="poisson", n=(64, 64), arrival=0.0) for k in range(12)]
    out = Server(ex, 10 ** 12, slots=4).run(reqs)
    assert ex.peak == 4
    assert ex.order[:4] == sorted(ex.order[:4]) and set(ex.order) == set(range(12))
    assert sorted(r.admitted for r in out) == [r.admitted for r in sorted(out, key=lambda r: r.id)]


def test_oversized_rejected_and_failures_recorded():
    ex = FakeExecutor()
    reqs = [Request(id=0, kind="poisson", n=(512, 512, 512)),
            Request(id=1, kind="boom", n=(64, 64)),
            Request(id=2, kind="ns", n=(64, 64))]
    out = {r.id: r for r in Server(ex, 10 ** 9, slots=2).run(reqs)}
    assert out[0].status == "rejected" and "budget" in out[0].error
    assert out[1].status == "failed" and "planted" in out[1].error
    assert out[2].status == "done"


def test_large_request_is_not_starved():
    ex = FakeExecutor(unit_s=0.004)
    small = 64 * 64 * 100
    big = Request(id=0, kind="poisson", n=(64, 64, 8), arrival=0.0005)
    reqs = [Request(id=k, kind="poisson", n=(64, 64), arrival=0.0002 * k) for k in range(1, 40)]
    budget = 64 * 64 * 8 * 100 + small      # big fits only when at most one small runs
    out = {r.id: r for r in Server(ex, budget, slots=4, max_overtakes=3).run(reqs + [big])}
    assert out[0].status == "done"
    later = [r for r in out.values() if r.id > 0 and r.arrival > big.arrival]
    # once it has been overtaken three times it goes before the rest of the queue
    assert sum(r.admitted < out[0].admitted for r in later) <= 3 + 4


class FakeBatchExecutor(FakeExecutor):
    """Batches 2D requests; records the units it ran."""

    def __init__(self):
        super().__init__(unit_s=0.003)
        self.units = []

    def batchable(self, r):
        return len(r.n) == 2 and r.kind == "poisson"

    def run_batch(self, rs):
        with self.lock:
            self.units.append([r.id for r in rs])
            self.active += 1
            self.bytes += sum(r.footprint for r in rs)
            self.peak = max(self.peak, self.active)
            self.peak_bytes = max(self.peak_bytes, self.bytes)
        time.sleep(self.unit)
        with self.lock:
            self.active -= 1
            self.bytes -= sum(r.footprint for r in rs)
        return [("ok", r.id) if r.id % 17 else RuntimeError("planted") for r in rs]


def test_small_requests_are_batched_within_budget():
    ex = FakeBatchExecutor()
    reqs = [Request(id=k, kind="poisson" if k % 3 else "ns", n=(64, 64) if k % 2 else (32, 32, 32),
                    arrival=0.0) for k in range(80)]
    budget = 40 * 64 * 64 * 100 + 2 * 32 ** 3 * 100
    srv = Server(ex, budget, slots=3, batch_max=8)
    out = {r.id: r for r in srv.run(reqs)}
    assert all(r.status in ("done", "failed") for r in out.values())
    assert all(out[k].status == ("failed" if (k % 17 == 0 and ex.batchable(out[k])) else "done")
               for k in out)
    sizes = [len(u) for u in ex.units]
    assert max(sizes) > 1 and max(sizes) <= 8
    # every batched unit holds only batchable requests, each exactly once
    ids = [i for u in ex.units for i in u]
    assert len(ids) == len(set(ids)) and all(ex.batchable(out[i]) for i in ids)
    assert ex.peak <= 3 and ex.peak_bytes <= budget
