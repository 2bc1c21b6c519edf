"""Host logic of the serving loop, on the CPU with stand-in executors:
first-come-first-served admission against the HBM budget, the budget never
exceeded under concurrency, refusal of oversized requests, failures that
reach their request while the slots and the budget are returned, and the
latency statistics."""
import threading
import time

import numpy as np
import pytest

from paper_2603_26968_amd import serve


def test_admission_fifo_and_budget():
    a = serve.Admission(100)
    assert a.acquire(60)
    order = []

    def take(tag, n):
        a.acquire(n)
        order.append(tag)

    t1 = threading.Thread(target=take, args=("big", 80))
    t1.start()
    time.sleep(0.05)
    t2 = threading.Thread(target=take, args=("small", 10))  # fits, but queued behind big
    t2.start()
    time.sleep(0.05)
    assert order == []
    a.release(60)
    t1.join(2)
    t2.join(2)
    assert sorted(order) == ["big", "small"] and a.in_use == 90
    assert not a.acquire(50, timeout=0.05)
    with pytest.raises(MemoryError):
        a.acquire(101)
    a.release(90)
    assert a.in_use == 0 and a.peak == 90


def test_budget_holds_under_concurrency():
    budget = 1000
    live = [0]
    peak = [0]
    lock = threading.Lock()
    rng = np.random.default_rng(1)

    def execute(slot, req):
        with lock:
            live[0] += req.footprint
            peak[0] = max(peak[0], live[0])
        time.sleep(float(rng.uniform(0, 0.003)))
        with lock:
            live[0] -= req.footprint
        return req.tag

    sizes = rng.integers(1, 600, size=200)
    with serve.Server(budget, slots=6, execute=execute,
                      footprint=lambda r: r.data) as srv:
        reqs = [srv.submit(serve.Request("compress", int(s), tag=i)) for i, s in enumerate(sizes)]
        for r in reqs:
            r.done.wait(10)
    assert all(r.result == r.tag and r.error is None for r in reqs)
    assert peak[0] <= budget
    assert srv.admission.in_use == 0 and srv.admission.peak <= budget


def test_failures_reach_their_request_and_free_the_slot():
    def execute(slot, req):
        if req.tag % 3 == 0:
            raise RuntimeError(f"boom {req.tag}")
        return req.tag * 2

    with serve.Server(50, slots=2, execute=execute, footprint=lambda r: r.data) as srv:
        reqs = [srv.submit(serve.Request("compress", 10, tag=i)) for i in range(30)]
        huge = srv.submit(serve.Request("compress", 51, tag=-1))  # refused, line moves on
        after = srv.submit(serve.Request("compress", 10, tag=31))
        for r in reqs + [huge, after]:
            assert r.done.wait(10)
    for r in reqs:
        if r.tag % 3 == 0:
            assert isinstance(r.error, RuntimeError)
            with pytest.raises(RuntimeError):
                r.wait(0)
        else:
            assert r.wait(0) == r.tag * 2
    assert isinstance(huge.error, MemoryError)
    assert after.wait(0) == 62
    assert srv.admission.in_use == 0


def test_poisson_driver_and_stats():
    def execute(slot, req):
        time.sleep(0.001)
        return req.tag

    offs = serve.poisson_arrivals(50, rate=2000.0, seed=3)
    assert np.all(np.diff(offs) > 0) and abs(offs[-1] / 50 - 1 / 2000.0) < 1 / 2000.0
    with serve.Server(10 ** 9, slots=3, execute=execute, footprint=lambda r: 1) as srv:
        reqs = serve.run_arrivals(srv, lambda i: serve.Request("compress", None, tag=i), offs)
    st = serve.latency_stats(reqs, lambda r: 1000)
    assert st["requests"] == 50 and st["failed"] == 0
    assert 1.0 <= st["p50_ms"] <= st["p99_ms"]
    assert st["GBps"] > 0


def test_kept_workspaces_stay_inside_the_budget():
    """Slots that keep workspaces between requests: the keep limit per slot
    is reserved from the budget up front, so the bytes in flight plus the
    kept bytes never exceed the budget (a stand-in executor keeps a
    'workspace' of the request's size when it is within the limit)."""
    budget, slots, limit = 1000, 3, 100
    kept = [0] * slots

    def execute(slot, req):
        time.sleep(0.001 * (req.tag % 3))
        kept[slot] = req.data if req.data <= limit else 0
        return req.data

    with serve.Server(budget, slots=slots, execute=execute, footprint=lambda r: 2 * r.data,
                      keep_limit=limit, kept=lambda: sum(kept)) as srv:
        assert srv.admission.budget == budget - slots * limit
        rng = np.random.default_rng(3)
        reqs = [srv.submit(serve.Request("compress", int(rng.integers(1, 350)), tag=i))
                for i in range(300)]
        for r in reqs:
            r.wait(10)
    assert srv.peak_total <= budget
    assert srv.admission.in_use == 0
    with pytest.raises(ValueError):
        serve.Server(100, slots=2, execute=execute, footprint=lambda r: 1, keep_limit=50)
