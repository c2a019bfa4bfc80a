"""Continuous-batching scheduler on the host, driven through a fake executor
(no GPU): admission by footprint, chunking into receiver ranges, newcomers
joining at step boundaries, failure injection and the one-at-a-time mode."""
import threading
import time

import pytest

from paper_2104_00359_amd import serve


class FakeExecutor(serve.Executor):
    """Footprint = scene["bytes"]; a step completes ``delay`` seconds after
    launch; launching a step that holds a request with scene["fail"] raises."""

    def __init__(self, delay=0.002):
        self.delay = delay
        self.lock = threading.Lock()
        self.admitted = []
        self.released = []
        self.used_at_admit = []

    def footprint(self, req):
        return req.scene["bytes"]

    def admit(self, req):
        with self.lock:
            self.admitted.append(req.rid)

    def launch(self, items):
        if any(r.scene.get("fail") for r, *_ in items):
            raise RuntimeError("injected launch failure")
        return time.perf_counter() + self.delay

    def done(self, token):
        return time.perf_counter() >= token

    def release(self, req):
        with self.lock:
            self.released.append(req.rid)


def _scene(nbytes=100, fail=False):
    return {"bytes": nbytes, "fail": fail}


def test_ranges_cover_scene_aligned_and_bounded():
    for P, S, cap in [(262144, 512, 8 << 20), (20000, 128, 1 << 20), (1000, 10, 1 << 20), (5000, 3000, 1000),
                      (0, 5, 100)]:
        rs = serve.ranges_for(P, S, cap)
        assert rs[0][0] == 0 and rs[-1][1] == P
        for (a, e), (a2, _) in zip(rs, rs[1:]):
            assert e == a2
        for a, e in rs:
            assert a % serve.RANGE_ALIGN == 0
            assert e == P or e % serve.RANGE_ALIGN == 0
            assert (e - a) * S <= cap or e - a <= serve.RANGE_ALIGN or P * S <= cap
    assert serve.ranges_for(262144, 512, None) == [(0, 262144)]
    assert len(serve.ranges_for(262144, 512, 8 << 20)) == 16


def test_all_requests_complete_and_budget_holds():
    ex = FakeExecutor()
    s = serve.Scheduler(ex, memory_budget=1000, chunk_pairs=10_000, record_steps=True).start()
    futs = [s.submit(_scene(300), P=1000, S=50) for _ in range(12)]
    reqs = [f.result(timeout=10) for f in futs]
    s.stop(timeout=10)
    assert [r.rid for r in reqs] == list(range(12))
    assert s.peak_used <= 1000 and s.used == 0
    assert sorted(ex.released) == list(range(12))
    assert ex.admitted == sorted(ex.admitted)          # admitted in arrival order
    for r in reqs:
        assert r.arrival <= r.admitted <= r.done
    # at most 3 requests of 300 bytes fit the budget at once
    for step in s.step_log:
        assert len({rid for rid, *_ in step}) <= 3


def test_large_request_is_chunked_and_newcomers_join_at_step_boundaries():
    ex = FakeExecutor(delay=0.005)
    s = serve.Scheduler(ex, memory_budget=10**9, chunk_pairs=256 * 100, max_inflight=1, record_steps=True).start()
    big = s.submit(_scene(), P=256 * 40, S=100)
    time.sleep(0.03)
    small = s.submit(_scene(), P=300, S=10)
    rb, rs = big.result(timeout=10), small.result(timeout=10)
    s.stop(timeout=10)
    big_items = [(a, e, d) for step in s.step_log for rid, a, e, d in step if rid == rb.rid]
    assert len(big_items) == 40
    assert [a for a, _, _ in big_items] == list(range(0, 256 * 40, 256))
    assert all(d for *_, d in big_items[:-1]) and not big_items[-1][2]
    first_small = next(i for i, step in enumerate(s.step_log) if any(rid == rs.rid for rid, *_ in step))
    last_big = max(i for i, step in enumerate(s.step_log) if any(rid == rb.rid for rid, *_ in step))
    assert 0 < first_small < last_big                   # joined while the big request was running
    assert rs.done < rb.done


def test_request_larger_than_budget_fails_and_others_proceed():
    ex = FakeExecutor()
    s = serve.Scheduler(ex, memory_budget=500).start()
    too_big = s.submit(_scene(501), P=10, S=10)
    ok = s.submit(_scene(400), P=10, S=10)
    with pytest.raises(MemoryError):
        too_big.result(timeout=10)
    assert ok.result(timeout=10).done > 0
    s.stop(timeout=10)


def test_failed_step_fails_its_requests_and_returns_memory():
    ex = FakeExecutor()
    s = serve.Scheduler(ex, memory_budget=10_000, max_active=1).start()
    a = s.submit(_scene(100), P=10, S=10)
    b = s.submit(_scene(100, fail=True), P=10, S=10)
    c = s.submit(_scene(100), P=10, S=10)
    assert a.result(timeout=10).done > 0
    with pytest.raises(RuntimeError, match="injected"):
        b.result(timeout=10)
    assert c.result(timeout=10).done > 0
    s.stop(timeout=10)
    assert s.used == 0 and s.error is None


def test_one_request_at_a_time_mode():
    ex = FakeExecutor()
    s = serve.Scheduler(ex, memory_budget=10**9, chunk_pairs=None, max_active=1, max_inflight=1,
                        record_steps=True).start()
    futs = [s.submit(_scene(), P=5000, S=300) for _ in range(5)]
    reqs = [f.result(timeout=10) for f in futs]
    s.stop(timeout=10)
    assert all(len(step) == 1 for step in s.step_log)
    assert all(a == 0 and e == 5000 and not d for step in s.step_log for _, a, e, d in step)
    for r1, r2 in zip(reqs, reqs[1:]):
        assert r2.admitted >= r1.done


def test_poisson_arrivals_rate():
    t = serve.poisson_arrivals(1000.0, 2.0, seed=7)
    assert 1800 < len(t) < 2200 and t[-1] < 2.0 and (t[1:] >= t[:-1]).all()


def test_admission_window_limits_admitted_work():
    ex = FakeExecutor(delay=0.003)
    s = serve.Scheduler(ex, memory_budget=10**12, chunk_pairs=None, step_pairs=1000, max_inflight=1,
                        admit_ahead=2000, record_steps=True).start()
    futs = [s.submit(_scene(), P=10, S=100) for _ in range(30)]   # 1000 pairs each
    for f in futs:
        f.result(timeout=20)
    s.stop(timeout=10)
    assert s.used == 0
    assert all(len(step) == 1 for step in s.step_log)          # the step bound holds
    assert s.peak_used <= 3 * 100                               # at most ~3 admitted at once


def test_ranges_merge_when_the_step_has_room():
    ex = FakeExecutor(delay=0.002)
    s = serve.Scheduler(ex, memory_budget=10**9, chunk_pairs=256 * 10, step_pairs=256 * 10 * 4, max_inflight=1,
                        record_steps=True).start()
    big = s.submit(_scene(), P=256 * 10, S=10)         # 10 ranges of 256 receivers
    r = big.result(timeout=10)
    s.stop(timeout=10)
    items = [(a, e, d) for step in s.step_log for rid, a, e, d in step if rid == r.rid]
    assert [(a, e) for a, e, _ in items] == [(0, 1024), (1024, 2048), (2048, 2560)]   # 4 ranges per step
    assert [d for *_, d in items] == [True, True, False]
