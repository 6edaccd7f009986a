"""The traditional static approach in the oracle (Section 4.3, Fig. 7;
Section 5.3), pinned to the paper's worked example and to invariants.

The static approach keeps the executed plan of the known jobs in place and
schedules the arrivals after it, stage by stage ("after completing the
operations of the original schedule at each stage"); complete rescheduling
(the method) reschedules every op not started by RS together with the
arrivals.
"""
import itertools

import numpy as np

import oracle
from oracle import validate
from paper_1903_10741_amd import workloads as W
from tests.golden_io import ints, read
from tests.test_oracle_pins import _paper_example


def _static_example():
    e = _paper_example()
    inst0 = W.initial_instance(e["proc"][:6], e["power"][:6], e["release"][:6], e["due"][:6],
                               e["nm"], e["q_max"], e["wt"])
    nxt = oracle.reschedule(inst0, e["plan_start"], e["plan_mach"], e["rs"], e["proc"][6:],
                            e["power"][6:], e["release"][6:], e["due"][6:], static=True)
    return e, W.Instance.from_fields(nxt)


def _full_plan(e, inst, s, m):
    start = np.vstack([e["plan_start"], s[6:]])
    mach = np.vstack([e["plan_mach"], m[6:]])
    return start, mach


def test_static_state_of_the_worked_example():
    """Every original op is frozen; those running at RS = 7 hold power to their end,
    the ones not yet started hold it on their planned window; every machine of a
    stage is free from the stage's planned completion (7.80, 11.91, 15.42)."""
    e, inst = _static_example()
    assert list(inst.active) == [6, 7]
    assert list(inst.first_stage[:6]) == [3] * 6
    ps, pm = e["plan_start"], e["plan_mach"]
    ends = ps + np.array([100, 200, 300])[None, :]
    running = sorted(int(x) for x in inst.running[:, 0])
    assert running == sorted(int(ends[j, s]) for j in range(6) for s in range(3)
                             if ps[j, s] < 700 < ends[j, s]) == [742, 780, 791]
    fixed = sorted(tuple(int(v) for v in r) for r in inst.fixed)
    assert fixed == sorted((int(ps[j, s]), int(ends[j, s]), 1) for j in range(6) for s in range(3)
                           if ps[j, s] >= 700)
    assert [int(inst.machine_free[s][0]) for s in range(3)] == [780, 1191, 1542]
    assert (inst.machine_free[:, 0] == inst.machine_free[:, 1]).all()
    # the frozen objective covers the six original jobs: their makespan is 15.42
    assert inst.frozen_cmax == 1542


def test_static_reproduces_fig7_makespan():
    """Fig. 7: both priority orders of the two arrivals give the printed makespan
    19.91, and so does the best of every X/Y chromosome (every machine choice and
    every order of the six new ops): no placement under the static rule does better."""
    e, inst = _static_example()
    want = ints(read("table4_example.txt")["expect_static_cmax"][0])[0]
    for prio in ([1, 2], [2, 1]):
        obj, s, m, _ = oracle.decode(inst, np.array(prio), want_schedule=True)
        comp = [int(s[j][2]) + 300 for j in (6, 7)]
        assert max(comp) == want == obj          # due dates unprinted: set far, no tardiness
        start, mach = _full_plan(e, inst, s, m)
        assert (start[:6] == e["plan_start"]).all()             # the original plan stays
        validate.check_plan(e["proc"], e["power"], e["release"], e["due"], e["nm"], e["q_max"],
                            e["wt"], start, mach)
    R = oracle.xy_ops(inst)
    assert R == 6
    best = None
    for xs in itertools.product((0, 1), repeat=R):
        for ys in itertools.permutations(range(1, R + 1)):
            o = oracle.decode_xy(inst, np.array(list(xs) + list(ys)))
            best = o if best is None else min(best, o)
    assert best == want


def test_static_arrivals_start_after_each_stage_of_the_plan():
    """Random instances: every arrival's op at stage s starts at or after the last
    planned op of stage s ends, the original plan is untouched and the combined
    schedule meets the model's constraints (power peak included)."""
    for seed in range(6):
        wl = W.config1(seed)
        inst0 = wl.initial
        prio = W.random_population(seed, 1, inst0.n_active)[0]
        _, s0, m0, _ = oracle.decode(inst0, prio, want_schedule=True)
        a = wl.arrivals[0]
        nxt = W.Instance.from_fields(oracle.reschedule(inst0, s0, m0, a.rs, a.proc, a.power,
                                                       a.release, a.due, static=True))
        n0 = inst0.n_jobs
        assert list(nxt.active) == list(range(n0, nxt.n_jobs))
        P = np.asarray(inst0.proc)
        stage_end = [max(int(s0[j, s]) + int(P[j, s, m0[j, s]]) for j in range(n0))
                     for s in range(inst0.n_stages)]
        for p2 in W.random_population(seed + 50, 4, nxt.n_active):
            obj, s, m, _ = oracle.decode(nxt, p2, want_schedule=True)
            for j in nxt.active:
                for st in range(inst0.n_stages):
                    assert s[j, st] >= stage_end[st]
            start = np.vstack([s0, s[n0:]])
            mach = np.vstack([m0, m[n0:]])
            assert (s[:n0] == -1).all()                       # original ops are not re-decoded
            got = validate.check_plan(nxt.proc, nxt.power, nxt.release, nxt.due,
                                      nxt.n_machines, nxt.q_max, nxt.wt, start, mach)
            assert got == obj


def test_static_equals_rescheduling_when_the_plan_has_finished():
    """An arrival after the whole plan has ended leaves nothing to reschedule: the
    static approach and complete rescheduling decode every chromosome alike."""
    for seed in range(4):
        wl = W.config1(seed)
        inst0 = wl.initial
        prio = W.random_population(seed, 1, inst0.n_active)[0]
        _, s0, m0, _ = oracle.decode(inst0, prio, want_schedule=True)
        P = np.asarray(inst0.proc)
        end = max(int(s0[j, s]) + int(P[j, s, m0[j, s]]) for j in range(inst0.n_jobs)
                  for s in range(inst0.n_stages))
        a = wl.arrivals[0]
        args = (inst0, s0, m0, end + 3, a.proc, a.power, np.full(len(a.release), end + 3),
                a.due + end)
        st = W.Instance.from_fields(oracle.reschedule(*args, static=True))
        dy = W.Instance.from_fields(oracle.reschedule(*args))
        assert len(st.fixed) == 0 and len(st.running) == 0
        for p2 in W.random_population(seed + 9, 8, st.n_active):
            assert oracle.decode(st, p2) == oracle.decode(dy, p2)


def test_event_loop_runs_both_ways_from_the_same_first_plan():
    """The oracle's event loop under either approach: event 0 is the same problem
    (the same GA from the same seed gives the same plan); the arrival is then
    handled by the chosen approach."""
    for seed in range(3):
        wl = W.config1(seed)
        st = oracle.run_events(wl.initial, wl.arrivals, wl.ga, 30, wl.seed, wl.shop,
                               n_threads=4, static=True)
        dy = oracle.run_events(wl.initial, wl.arrivals, wl.ga, 30, wl.seed, wl.shop, n_threads=4)
        assert st[0]["best_obj"] == dy[0]["best_obj"]          # event 0 is the same problem
        assert len(st) == len(dy) == 2
