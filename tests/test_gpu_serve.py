"""The rescheduling service on the device: every shop served through the
continuously batched GA gets, event after event, exactly the oracle's
event loop for that shop alone (best objective and executed plan), whatever
else shares the batch."""
import numpy as np
import pytest

import oracle
from paper_1903_10741_amd import workloads as W

pytestmark = pytest.mark.gpu

GA = W.GaParams(2, 2, 4, mig_interval=2, mig_k=1)
GENS = 5


def _say(*a):
    print("[case]", *a, flush=True)


def _shops(seed, n, n_events):
    insts = W.shops(seed, n, jobs=(6, 24), stages=(2, 4), machines=(2, 4), o_max=4)
    arrs = [W.shop_arrivals(seed, k, inst, n_events[k]) for k, inst in enumerate(insts)]
    return insts, arrs


def _serve(insts, arrs, schedule, n_slots, gens_per_tick, **kw):
    from paper_1903_10741_amd.serve import Server
    srv = Server(insts, arrs, GA, generations=GENS, n_slots=n_slots, gens_per_tick=gens_per_tick,
                 seed=17, **kw)
    m = srv.run(schedule)
    return srv, m


def _check_against_oracle(srv, insts, arrs, n_events, shops):
    for k in shops:
        want = oracle.run_events(insts[k], arrs[k], GA, GENS, 17, k, n_threads=4,
                                 events=n_events[k])
        sh = srv.shops[k]
        assert sh.history == [e["best_obj"] for e in want], f"shop {k}"
        n = want[-1]["plan_start"].shape[0]
        assert (sh.plan_start[:n].cpu().numpy() == want[-1]["plan_start"]).all(), f"shop {k} start"
        assert (sh.plan_mach[:n].cpu().numpy() == want[-1]["plan_mach"]).all(), f"shop {k} mach"


@pytest.mark.parametrize("use_graph", [True, False])
def test_serving_matches_oracle_per_shop(use_graph):
    from paper_1903_10741_amd.serve import poisson_schedule
    _say("serving 6 shops, 3 slots, graph", use_graph)
    n_events = [3, 1, 2, 3, 2, 1]
    insts, arrs = _shops(31, 6, n_events)
    sched = poisson_schedule(2, rate_per_s=500.0, n_events=n_events)
    srv, m = _serve(insts, arrs, sched, n_slots=3, gens_per_tick=2,
                    tuning={"use_graph": use_graph, "blocks": 16})
    assert m["done"] == sum(n_events) and m["failed"] == 0 and m["unfinished"] == 0
    assert srv.ticks >= GENS                      # batches of several slots really ran
    _check_against_oracle(srv, insts, arrs, n_events, range(6))
    assert m["latency_p50_s"] > 0 and m["latency_p99_s"] >= m["latency_p50_s"]


def test_shop_alone_equals_shop_in_mix():
    from paper_1903_10741_amd.serve import poisson_schedule
    _say("serving: one shop alone vs in a mix")
    n_events = [2, 3, 2, 2]
    insts, arrs = _shops(44, 4, n_events)
    mix, m = _serve(insts, arrs, poisson_schedule(3, 800.0, n_events), n_slots=4, gens_per_tick=3,
                    tuning={"schedule": 1, "blocks": 8})
    assert m["failed"] == 0
    only = [0, 3, 0, 0]
    alone, m2 = _serve(insts, arrs, poisson_schedule(4, 800.0, only), n_slots=1, gens_per_tick=1)
    assert m2["done"] == 3
    assert alone.shops[1].history == mix.shops[1].history
    n = alone.shops[1].plan_start.shape[0]
    assert (alone.shops[1].plan_start.cpu() == mix.shops[1].plan_start[:n].cpu()).all()


def test_serving_memory_budget_and_rejects_extra_events():
    from paper_1903_10741_amd.serve import Server
    _say("serving: memory budget, request beyond a shop's arrivals")
    insts, arrs = _shops(50, 2, [1, 1])
    srv = Server(insts, arrs, GA, generations=2, n_slots=8, seed=1)
    from dataclasses import replace
    small = Server(insts, arrs, GA, generations=2, n_slots=8, seed=1,
                   memory_budget=replace(srv.cfg, n_slots=2).workspace_bytes())
    assert small.adm.n_slots == 2
    m = small.run([(0.0, 0), (0.0, 0), (0.0, 0), (0.0, 1)])   # shop 0: 3 requests, 2 events
    assert m["done"] == 3 and m["failed"] == 1
    bad = [r for r in small.requests if r.status == "failed"][0]
    assert bad.shop == 0 and "arrival" in bad.error


def test_failed_load_leaves_the_shop_unchanged():
    """A shop whose rescheduled instance outgrows the batch's room: the request
    fails, and the shop keeps its instance, executed plan, pending arrival and
    event count, as if the request had never been admitted."""
    from paper_1903_10741_amd.serve import Server
    _say("serving: failed load rolls the shop back")
    insts, arrs = _shops(61, 1, [1])
    want = oracle.run_events(insts[0], arrs[0], GA, 2, 1, 0, n_threads=4, events=2)
    room = oracle.horizon_bound(insts[0])
    assert oracle.horizon_bound(want[1]["instance"]) > room   # event 1 does not fit
    srv = Server(insts, arrs, GA, generations=2, n_slots=1, seed=1, max_horizon=room)
    m = srv.run([(0.0, 0)])
    assert m["done"] == 1 and m["failed"] == 0
    sh = srv.shops[0]
    inst0, plan_s, plan_m = sh.inst, sh.plan_start.clone(), sh.plan_mach.clone()
    m = srv.run([(0.0, 0)])
    assert m["failed"] == 1
    bad = [r for r in srv.requests if r.status == "failed"][0]
    assert "outside the limits" in bad.error
    assert sh.inst is inst0 and sh.event == 1 and len(sh.arrivals) == 1
    assert sh.history == [want[0]["best_obj"]]
    assert (sh.plan_start == plan_s).all() and (sh.plan_mach == plan_m).all()
    assert srv.adm.busy == 0 and not srv.running
