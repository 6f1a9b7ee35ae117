"""Host logic of the serving loop (pool allocator, admission, continuous batching),
driven by a simulated executor on a virtual clock.  No GPU."""
import random

import numpy as np
import pytest

from paper_1911_05633_amd import serve
from synthcell import Request, request_stream


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class SimExecutor:
    """Each request occupies its slot for a fixed service time per kind; footprints per kind.

    Records the concurrency (slots in use, bytes in use) at every launch so the tests can
    check the server's invariants."""

    def __init__(self, clock, service, footprint, fail_launch=()):
        self.clock = clock
        self.service = service
        self.footprint = footprint
        self.fail_launch = set(fail_launch)
        self.live = {}
        self.max_live = 0
        self.max_bytes = 0
        self.launched = []
        self.t0 = 0.0

    def sizes(self, req):
        return [self.footprint[req.kind], 1000]

    def start(self):
        self.t0 = self.clock()

    def launch(self, req, slot, offs):
        if req.request_id in self.fail_launch:
            raise RuntimeError("launch failed")
        assert slot not in self.live, "slot handed out twice"
        h = {"req": req, "slot": slot, "t": self.clock() - self.t0, "end": self.clock() - self.t0 + self.service[req.kind],
             "offs": offs}
        self.live[slot] = h
        self.max_live = max(self.max_live, len(self.live))
        self.max_bytes = max(self.max_bytes, sum(serve._align(self.footprint[x["req"].kind]) + serve._align(1000)
                                                 for x in self.live.values()))
        self.launched.append((req.request_id, h["t"]))
        return h

    def poll(self, h):
        return self.clock() - self.t0 >= h["end"]

    def completion(self, h):
        return h["end"]

    def finish(self, h, rec):
        rec.result["slot"] = h["slot"]
        rec.result["start"] = h["t"]

    def release(self, h):
        del self.live[h["slot"]]

    def wait(self, seconds):
        # advance the virtual clock to the next event (arrival or completion)
        ends = [h["end"] for h in self.live.values()]
        nxt = min(ends) - (self.clock() - self.t0) if ends else None
        cands = [x for x in (seconds, nxt) if x is not None and x > 0]
        self.clock.t += min(cands) if cands else 1e-6


def run_sim(reqs, capacity, slots, service, footprint, **kw):
    clock = Clock()
    fail = kw.pop("fail_launch", ())
    ex = SimExecutor(clock, service, footprint, fail_launch=fail)
    srv = serve.Server(ex, capacity, slots=slots, clock=clock, **kw)
    return srv, ex, srv.run(reqs)


SERVICE = {"s": 1.0, "m": 3.0, "l": 10.0}
FOOT = {"s": 10 << 20, "m": 40 << 20, "l": 100 << 20}


def test_pool_best_fit_alignment_and_coalescing():
    p = serve.Pool(10_000)
    assert p.capacity == 10_000 // 256 * 256
    a = p.alloc(100)
    b = p.alloc(300)
    c = p.alloc(256)
    assert (a, b, c) == (0, 256, 768)
    assert p.used == 256 + 512 + 256
    p.free(b)
    # best fit: a 200-byte request goes into the 512-byte hole, not the tail
    d = p.alloc(200)
    assert d == 256
    p.free(a)
    p.free(d)
    p.free(c)
    assert p.used == 0 and p._free == [(0, p.capacity)] and p.largest_free == p.capacity
    assert p.peak == 1024


def test_pool_alloc_all_is_all_or_nothing():
    p = serve.Pool(4096)
    assert p.alloc_all([1024, 1024, 4096]) is None
    assert p.used == 0 and p.largest_free == 4096
    offs = p.alloc_all([1024, 1024])
    assert offs == [0, 1024]
    p.fail_next = 1
    with pytest.raises(MemoryError):
        p.alloc_all([256])
    assert p.used == 2048


def test_pool_random_alloc_free_keeps_the_free_list_consistent():
    rng = random.Random(3)
    p = serve.Pool(1 << 20)
    live = []
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = live.pop(rng.randrange(len(live)))
            p.free(off)
        else:
            off = p.alloc(rng.randrange(1, 40_000))
            if off is not None:
                live.append(off)
        # free intervals are sorted, disjoint, never adjacent, and cover capacity - used
        fr = p._free
        assert all(fr[i][0] + fr[i][1] < fr[i + 1][0] for i in range(len(fr) - 1))
        assert sum(s for _, s in fr) == p.capacity - p.used
        spans = sorted((o, p._live[o]) for o in p._live)
        assert all(spans[i][0] + spans[i][1] <= spans[i + 1][0] for i in range(len(spans) - 1))


def test_percentile_is_nearest_rank():
    v = list(np.random.default_rng(0).random(101))
    for q in (1, 50, 90, 99, 100):
        assert serve.percentile(v, q) == sorted(v)[int(np.ceil(q / 100 * len(v))) - 1]
    assert np.isnan(serve.percentile([], 50))


def test_every_request_completes_within_slots_and_memory():
    rng = np.random.default_rng(1)
    reqs = [Request(i, float(t), str(k), 16) for i, (t, k) in
            enumerate(zip(np.cumsum(rng.exponential(0.7, 60)), rng.choice(list("sml"), 60)))]
    cap = 200 << 20
    srv, ex, recs = run_sim(reqs, cap, 3, SERVICE, FOOT)
    assert all(r.status == "done" for r in recs)
    assert ex.max_live <= 3
    assert ex.max_bytes <= cap
    for r in recs:
        assert r.admitted >= r.arrival - 1e-12
        assert r.done == pytest.approx(r.admitted + SERVICE[r.kind])
        assert r.latency >= SERVICE[r.kind] - 1e-12
    assert srv.pool.used == 0


def test_requests_arriving_during_work_join_it():
    """Continuous batching: a request that arrives while another runs starts before that one ends."""
    reqs = [Request(0, 0.0, "l", 16), Request(1, 2.0, "s", 16), Request(2, 4.0, "m", 16)]
    _, ex, recs = run_sim(reqs, 1 << 30, 4, SERVICE, FOOT)
    r0, r1, r2 = recs
    assert r1.admitted == pytest.approx(2.0) and r1.admitted < r0.done
    assert r2.admitted == pytest.approx(4.0) and r2.admitted < r0.done
    assert r1.done < r0.done  # the short one is not held behind the long one


def test_admission_by_footprint_defers_then_backfills():
    # pool fits one "l" (100 MiB) or two "m"; head "l" must wait while the running "m" pair holds memory
    cap = 130 << 20
    reqs = [Request(0, 0.0, "m", 16), Request(1, 0.0, "m", 16), Request(2, 0.1, "l", 16),
            Request(3, 0.2, "s", 16)]
    _, ex, recs = run_sim(reqs, cap, 4, SERVICE, FOOT)
    assert ex.max_bytes <= cap
    r0, r1, r2, r3 = recs
    assert r2.admitted >= min(r0.done, r1.done) - 1e-12  # deferred until memory frees
    assert r3.admitted < r2.admitted  # backfilled past the deferred head
    assert all(r.status == "done" for r in recs)


def test_head_of_line_is_not_starved():
    cap = 110 << 20
    reqs = [Request(0, 0.0, "m", 16), Request(1, 0.01, "l", 16)] + \
           [Request(2 + i, 0.02 + 0.5 * i, "m", 16) for i in range(40)]
    _, ex, recs = run_sim(reqs, cap, 4, SERVICE, FOOT, max_bypass=3)
    big = recs[1]
    assert big.status == "done"
    assert big.bypassed <= 3
    # without backfill the order of admission is the arrival order
    _, ex2, recs2 = run_sim(reqs, cap, 4, SERVICE, FOOT, backfill=False)
    adm = [r.admitted for r in recs2]
    assert adm == sorted(adm)


def test_too_large_request_is_rejected_and_others_still_run():
    reqs = [Request(0, 0.0, "s", 16), Request(1, 0.0, "l", 16), Request(2, 0.5, "s", 16)]
    _, ex, recs = run_sim(reqs, 50 << 20, 2, SERVICE, FOOT)
    assert [r.status for r in recs] == ["done", "rejected", "done"]
    assert "exceeds the pool" in recs[1].error
    assert 1 not in [i for i, _ in ex.launched]


def test_launch_failure_and_allocator_failure_end_only_that_request():
    reqs = [Request(i, 0.1 * i, "s", 16) for i in range(6)]
    srv, ex, recs = run_sim(reqs, 1 << 30, 2, SERVICE, FOOT, fail_launch={2})
    assert [r.status for r in recs] == ["done", "done", "failed", "done", "done", "done"]
    assert srv.pool.used == 0
    # allocator failure injected on the first admission
    clock = Clock()
    ex = SimExecutor(clock, SERVICE, FOOT)
    srv = serve.Server(ex, 1 << 30, slots=2, clock=clock)
    srv.pool.fail_next = 1
    recs = srv.run(reqs)
    assert recs[0].status == "failed" and "injected" in recs[0].error
    assert all(r.status == "done" for r in recs[1:])
    assert srv.pool.used == 0


def test_cancel_queued_and_running():
    reqs = [Request(0, 0.0, "l", 16), Request(1, 0.0, "l", 16), Request(2, 0.0, "s", 16)]
    clock = Clock()
    ex = SimExecutor(clock, SERVICE, FOOT)
    srv = serve.Server(ex, 1 << 30, slots=1, clock=clock)
    srv.cancel(1)  # queued behind request 0: never launched
    srv.cancel(0)  # will be running: result discarded
    recs = srv.run(reqs)
    assert [r.status for r in recs] == ["cancelled", "cancelled", "done"]
    assert 1 not in [i for i, _ in ex.launched]
    assert "slot" not in recs[0].result


def test_summary_and_request_stream():
    reqs = request_stream(200, rate=5.0)
    assert len(reqs) == 200
    arr = [r.arrival for r in reqs]
    assert arr == sorted(arr) and arr[0] > 0
    assert {r.kind for r in reqs} <= {"tiny2", "si8", "si24", "si40", "si72"}
    assert {r.n_tau for r in reqs} <= {16, 24, 32, 40, 48}
    assert request_stream(200, rate=5.0)[17] == reqs[17]  # seeded
    burst = request_stream(10, rate=5.0, burst=True)
    assert all(r.arrival == 0.0 for r in burst)
    foot = {k: 1 << 20 for k in ("tiny2", "si8", "si24", "si40", "si72")}
    svc = {"tiny2": 0.001, "si8": 0.01, "si24": 0.02, "si40": 0.05, "si72": 0.13}
    _, _, recs = run_sim(reqs, 1 << 30, 4, svc, foot)
    s = serve.summarize(recs)
    assert s["done"] == 200 and s["rejected"] == 0
    assert s["p50_ms"] <= s["p99_ms"]
    assert s["throughput_req_per_s"] == pytest.approx(200 / s["makespan_s"])
