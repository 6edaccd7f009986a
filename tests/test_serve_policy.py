"""Serving policy on the CPU: admission, per-shop order, memory budget, deadlines,
the request stream, and the per-shop horizon room (checked against the oracle's
own horizon bound on every event of a served shop)."""
import numpy as np
import pytest

import oracle
from paper_1903_10741_amd import workloads as W
from paper_1903_10741_amd.serve import Admission, horizon_room, percentiles, poisson_schedule


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


def test_admission_fifo_slots_and_shop_order():
    c = Clock()
    a = Admission(n_slots=2, slot_bytes=10, clock=c)
    r0 = a.submit(0)
    r1 = a.submit(0)          # same shop: must wait for r0
    r2 = a.submit(1)
    r3 = a.submit(2)          # no slot left
    got = a.admit()
    assert [r.rid for r in got] == [0, 2]
    assert {r0.slot, r2.slot} == {0, 1}
    assert r1.status == "queued" and r3.status == "queued"
    assert [r.rid for r in a.queue] == [1, 3]
    c.t = 1.0
    a.release(r0)
    got = a.admit()
    assert [r.rid for r in got] == [1]       # r1 first (FIFO), takes r0's slot
    assert r1.slot == r0.slot
    assert r0.status == "done" and r0.latency == 1.0
    a.release(r2)
    assert [r.rid for r in a.admit()] == [3]
    assert a.busy == 2


def test_admission_memory_budget_limits_slots():
    a = Admission(n_slots=64, slot_bytes=1000, memory_budget=3500)
    assert a.n_slots == 3
    for s in range(5):
        a.submit(s)
    assert len(a.admit()) == 3
    with pytest.raises(ValueError):
        Admission(n_slots=4, slot_bytes=1000, memory_budget=999)


def test_admission_deadline_marks_late_and_failures_free_the_slot():
    c = Clock()
    a = Admission(n_slots=1, slot_bytes=1, deadline_s=0.5, clock=c)
    r = a.submit(3)
    a.admit()
    c.t = 0.75
    a.release(r)
    assert r.status == "late"
    r2 = a.submit(3)
    a.admit()
    a.release(r2, "failed", "boom")
    assert r2.status == "failed" and r2.error == "boom" and a.busy == 0 and not a.in_flight


def test_poisson_schedule_counts_and_rate():
    n_events = [3, 1, 4, 2]
    s = poisson_schedule(5, rate_per_s=200.0, n_events=n_events)
    assert len(s) == sum(n_events)
    assert [sum(1 for _, k in s if k == i) for i in range(4)] == n_events
    t = [x for x, _ in s]
    assert all(b > a for a, b in zip(t, t[1:]))
    big = poisson_schedule(6, rate_per_s=100.0, n_events=[2000])
    gaps = np.diff([0.0] + [x for x, _ in big])
    assert abs(gaps.mean() - 0.01) < 0.001          # mean gap 1/rate


def test_percentiles():
    assert percentiles([]) == {"p50": None, "p99": None}
    p = percentiles(list(range(1, 101)))
    assert p["p50"] == 50.5 and abs(p["p99"] - 99.01) < 1e-9


def test_horizon_room_bounds_every_event():
    """The room the server sizes its batch with holds every event's horizon bound
    (the oracle's, computed on the instances of a full event loop)."""
    insts = W.shops(21, 3, jobs=(8, 16), stages=(2, 4), machines=(2, 3), o_max=3)
    for k, inst in enumerate(insts):
        arr = W.shop_arrivals(21, k, inst, 3)
        room = horizon_room(inst, arr)
        ev = oracle.run_events(inst, arr, W.GaParams(1, 2, 2), 2, 9, k)
        for e in ev:
            assert oracle.horizon_bound(e["instance"]) <= room


def test_shop_arrivals_shape():
    inst = W.shops(4, 1)[0]
    arr = W.shop_arrivals(4, 0, inst, 5)
    assert len(arr) == 5
    rs = [a.rs for a in arr]
    assert all(b > a for a, b in zip(rs, rs[1:])) and rs[0] >= 1
    for a in arr:
        k = len(a.release)
        assert a.proc.shape == (k, inst.n_stages, inst.o_max) and (a.proc >= 1).all()
        assert (a.release == a.rs).all() and (a.due > a.rs).all()
        assert (a.power == inst.power[0][None]).all()
