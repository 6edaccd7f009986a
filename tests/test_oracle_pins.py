"""Pins of the CPU oracle against what the paper and the mathematics fix.

Every test here runs on the CPU and checks the oracle against something other
than itself: values printed in the paper (tests/golden/), closed forms of
special cases, an independently written second decoder, the model's
invariants, brute force over all priority vectors, and numpy's Philox.
"""
import itertools

import numpy as np
import pytest

import oracle
from oracle import eventlist, validate
from paper_1903_10741_amd import workloads as W
from tests.golden_io import ints, read


# --------------------------------------------------------------------------
# Philox4x64-10: numpy's Philox is the same generator; its random_raw(4)
# returns the block at the counter after incrementing word 0 once.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("counter,key", [
    ([0, 0, 0, 0], [0, 0]),
    ([5, 7, 11, 2 << 32 | 3], [123456789, 42]),
    ([2**64 - 2, 2**64 - 1, 2**63, 1], [2**64 - 1, 2**64 - 1]),
    ([17, 499, 5, 1 << 32], [0, 7]),
])
def test_philox_matches_numpy(counter, key):
    g = np.random.Philox(counter=np.array(counter, dtype=np.uint64), key=np.array(key, dtype=np.uint64))
    want = g.random_raw(4)
    c = list(counter)
    c[0] = (c[0] + 1) % 2**64
    if c[0] == 0:
        c[1] = (c[1] + 1) % 2**64
    got = oracle.philox4x64_10(c, key)
    assert [int(x) for x in got] == [int(x) for x in want]


# --------------------------------------------------------------------------
# Worked example of Section 4.3 (Table 4, X/Y/Z matrices, Figs. 6-8).
# --------------------------------------------------------------------------
def _paper_example():
    f = read("table4_example.txt")
    q_max = ints(f["q_max"][0])[0]
    wt = ints(f["wt"][0])[0]
    rs = ints(f["rs"][0])[0]
    p_stage = ints(f["proc_per_stage"][0])
    nm = ints(f["machines_per_stage"][0])
    release = ints(f["release"][0])
    g, om = 3, 2
    plan_mach = np.zeros((6, g), np.int32)
    plan_start = np.zeros((6, g), np.int32)
    for row in f["plan_mach"]:
        j, *m = ints(row)
        plan_mach[j] = m
    for row in f["plan_start"]:
        j, *s = ints(row)
        plan_start[j] = s
    proc = np.array([[[p_stage[s]] * om for s in range(g)] for _ in range(8)], np.int32)
    power = np.ones((8, g, om), np.int32)
    due = np.full(8, 10**6, np.int32)  # due dates are not printed: tardiness unpinned
    X = np.array([[int(v) for v in r] for r in f["X"]])
    Z = [[v for v in r] for r in f["Z"]]
    return dict(q_max=q_max, wt=wt, rs=rs, nm=nm, release=release, proc=proc, power=power,
                due=due, plan_mach=plan_mach, plan_start=plan_start, X=X, Z=Z, f=f)


def test_table4_original_plan_is_feasible():
    """T2: the original plan of Table 4 meets eqs. (4)-(9), power peak reached."""
    e = _paper_example()
    validate.check_plan(e["proc"][:6], e["power"][:6], e["release"][:6], e["due"][:6], e["nm"],
                        e["q_max"], e["wt"], e["plan_start"], e["plan_mach"])
    with pytest.raises(AssertionError, match="power"):
        validate.check_plan(e["proc"][:6], e["power"][:6], e["release"][:6], e["due"][:6],
                            e["nm"], e["q_max"] - 1, e["wt"], e["plan_start"], e["plan_mach"])


def _example_rescheduled():
    e = _paper_example()
    inst0 = W.initial_instance(e["proc"][:6], e["power"][:6], e["release"][:6], e["due"][:6],
                               e["nm"], e["q_max"], e["wt"])
    nxt = oracle.reschedule(inst0, e["plan_start"], e["plan_mach"], e["rs"], e["proc"][6:],
                            e["power"][6:], e["release"][6:], e["due"][6:])
    return e, W.Instance.from_fields(nxt)


def test_table4_frozen_state_matches_printed_X_and_Z():
    """Ops started before RS are exactly the -1 entries of the printed X(k); those
    running at RS are exactly the 0 entries of the printed Z(k) (Algorithm 1)."""
    e, inst = _example_rescheduled()
    X, Z = e["X"], e["Z"]
    for j in range(8):
        frozen = [s for s in range(3) if X[j][s] == -1]
        assert frozen == list(range(len(frozen)))           # a stage prefix
        assert inst.first_stage[j] == len(frozen)
    running_ops = {(j, s) for j in range(8) for s in range(3) if Z[j][s] == "0"}
    assert running_ops == {(1, 2), (2, 0), (4, 1)}
    ends = sorted(int(x) for x in inst.running[:, 0])
    want = sorted(int(e["plan_start"][j][s]) + int(e["proc"][j][s][0]) for (j, s) in running_ops)
    assert ends == want == [742, 780, 791]
    assert list(inst.active) == [2, 3, 4, 5, 6, 7]
    # machine (1,1) runs job 4 until 7.91; (0,0) runs job 2 until 7.80
    assert inst.machine_free[1][1] == 791 and inst.machine_free[0][0] == 780
    assert inst.ready[2] == 780 and inst.ready[4] == 791 and inst.ready[6] == 777


def test_table4_rescheduled_plan_reproduces_fig8():
    """T1: decoding the printed Z(k) order on the printed X(k) machines gives the
    makespan of Fig. 8 (20.42) and delays job 7 stage 0 until job 5 stage 2 ends."""
    e, inst = _example_rescheduled()
    X, Z = e["X"], e["Z"]
    ops = sorted((int(Z[j][s]), j, s) for j in range(8) for s in range(3)
                 if Z[j][s] not in ("0", "C"))
    assert [z for z, _, _ in ops] == list(range(1, 14))
    order = [(j, s, int(X[j][s])) for _, j, s in ops]
    start = np.full((8, 3), -1, np.int32)
    mach = np.full((8, 3), -1, np.int32)
    start[:6] = np.where(X[:6] == -1, e["plan_start"], -1)
    mach[:6] = np.where(X[:6] == -1, e["plan_mach"], -1)
    obj, start, mach = oracle.decode_ops(inst, order, start, mach)
    f = e["f"]
    dj, ds = ints(f["expect_delayed_op"][0])
    uj, us = ints(f["expect_delayed_until_op"][0])
    end_until = start[uj][us] + e["proc"][uj][us][0]
    assert start[dj][ds] == end_until == 1391
    assert mach[uj][us] == 0 and us == 2     # "machine 4" = stage 2, machine 0
    comp = [start[j][2] + e["proc"][j][2][0] for j in range(8)]
    assert max(comp) == ints(f["expect_cmax"][0])[0] == 2042
    # the delay is caused by the power peak: machine 0 of stage 0 was free at 780
    assert inst.machine_free[0][0] == 780 and start[dj][ds] > 780
    # the whole rescheduled plan meets the model's constraints
    decoded = X != -1
    validate.check_plan(e["proc"], e["power"], e["release"], e["due"], e["nm"], e["q_max"],
                        e["wt"], start, mach, rs=e["rs"], decoded=decoded)
    # and the objective the oracle reports is eq. (1) of that plan
    tard = sum(max(c - int(d), 0) for c, d in zip(comp, e["due"]))
    assert obj == e["wt"] * tard + max(comp)


# --------------------------------------------------------------------------
# Crossover with correction (Fig. 11) and mutation (Fig. 12).
# --------------------------------------------------------------------------
def _genes(full):
    return [v for v in full if v != -1]


def _expand(full, genes):
    it = iter(genes)
    return [v if v == -1 else next(it) for v in full]


def test_fig11_correction():
    f = read("fig11_crossover.txt")
    for side in ("a", "b"):
        cross = ints(f[f"Y_cross_{side}"][0])
        want = ints(f[f"Y_corrected_{side}"][0])
        got = _expand(cross, oracle.correct(_genes(cross)).tolist())
        assert got == want


def test_fig11_crossover():
    f = read("fig11_crossover.txt")
    a = ints(f["Y_parent_a"][0])
    b = ints(f["Y_parent_b"][0])
    cut_elem = ints(f["cut_elements"][0])[0]
    cut = sum(1 for v in a[:cut_elem] if v != -1)        # same frozen layout in a and b
    ca, cb = oracle.crossover(_genes(a), _genes(b), cut)
    assert _expand(a, ca.tolist()) == ints(f["Y_corrected_a"][0])
    assert _expand(b, cb.tolist()) == ints(f["Y_corrected_b"][0])
    # the splice before correction is the printed "after crossover" pair
    assert a[:cut_elem] + b[cut_elem:] == ints(f["Y_cross_a"][0])
    assert b[:cut_elem] + a[cut_elem:] == ints(f["Y_cross_b"][0])


def test_correction_properties():
    rng = np.random.default_rng(3)
    for n in (1, 2, 3, 7, 64, 65, 300):
        for _ in range(20):
            v = rng.integers(1, n + 1, size=n)
            c = oracle.correct(v)
            assert sorted(c.tolist()) == list(range(1, n + 1))
            seen = set()
            for k in range(n):           # first occurrences are kept in place
                if v[k] not in seen:
                    assert c[k] == v[k]
                    seen.add(int(v[k]))
            missing = sorted(set(range(1, n + 1)) - set(v.tolist()))
            dups = [k for k in range(n) if c[k] != v[k]]
            assert [int(c[k]) for k in dups] == missing   # ascending, in scan order


def _word_for(value, n):
    """A 64-bit draw w with floor(hi32(w) * n / 2^32) == value."""
    hi = -(-(value << 32) // n)
    return hi << 32


def test_fig12_mutation():
    f = read("fig12_mutation.txt")
    before = ints(f["Y_before"][0])
    after = ints(f["Y_after"][0])
    gb, ga = _genes(before), _genes(after)
    diff = [k for k in range(len(gb)) if gb[k] != ga[k]]
    assert len(diff) == 2
    x, y = diff
    n = len(gb)
    got = oracle.mutate(gb, _word_for(x, n), _word_for(y - 1 if y > x else y, n - 1))
    assert _expand(before, got.tolist()) == after


def test_mutation_positions_uniform():
    n = 5
    counts = np.zeros((n, n), np.int64)
    rng = np.random.default_rng(0)
    base = np.arange(1, n + 1)
    for _ in range(20000):
        w1, w2 = (int(x) for x in rng.integers(0, 2**63, size=2, dtype=np.int64) * 2)
        v = oracle.mutate(base, w1, w2)
        d = np.nonzero(v != base)[0]
        assert len(d) == 2 and v[d[0]] == base[d[1]] and v[d[1]] == base[d[0]]
        counts[d[0], d[1]] += 1
    pairs = counts[np.triu_indices(n, 1)]
    assert pairs.min() > 0.8 * pairs.mean() and pairs.max() < 1.2 * pairs.mean()


# --------------------------------------------------------------------------
# Closed forms of special cases of the decoder.
# --------------------------------------------------------------------------
def _order_by_priority(prio, active):
    return [int(active[k]) for k in np.argsort(-np.asarray(prio), kind="stable")]


def test_flow_shop_recurrence_when_power_never_binds():
    """o_s = 1 everywhere and Q_max >= the sum of all powers: a permutation flow
    shop with releases, C_js = max(C_j,s-1, C_prev,s) + p_js, same order at every
    stage (stage-major order of the job priorities)."""
    for seed in range(5):
        inst = W.random_instance(seed, n_jobs=7, n_stages=4, machines=1, release_max=30)
        inst.q_max = int(inst.power.sum())
        rng = np.random.default_rng(seed)
        for _ in range(5):
            prio = rng.permutation(7) + 1
            order = _order_by_priority(prio, inst.active)
            comp_prev_stage = {j: int(inst.release[j]) for j in order}
            for s in range(4):
                t_machine = 0
                for j in order:
                    c = max(comp_prev_stage[j], t_machine) + int(inst.proc[j][s][0])
                    comp_prev_stage[j] = c
                    t_machine = c
            tard = sum(max(comp_prev_stage[j] - int(inst.due[j]), 0) for j in order)
            want = inst.wt * tard + max(comp_prev_stage.values())
            assert oracle.decode(inst, prio) == want


def test_full_serialisation_when_every_op_needs_the_peak():
    """Every Q_jsm = Q_max and releases 0: no two ops overlap, the stages run one
    after the other without idle time, so C_max = sum of all processing times
    and each stage's ops run back to back in priority order."""
    for seed in range(5):
        inst = W.random_instance(seed, n_jobs=6, n_stages=3, machines=2)
        inst.proc[:, :, 1] = inst.proc[:, :, 0]      # identical machines
        inst.power[:] = 4
        inst.q_max = 4
        prio = np.random.default_rng(seed).permutation(6) + 1
        obj, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
        order = _order_by_priority(prio, inst.active)
        t = 0
        for s in range(3):
            for j in order:
                assert start[j][s] == t
                t += int(inst.proc[j][s][0])
        tard = sum(max(int(start[j][2] + inst.proc[j][2][0]) - int(inst.due[j]), 0) for j in order)
        assert obj == inst.wt * tard + int(inst.proc[:, :, 0].sum())


def test_single_machine_sequence():
    """g = 1, o = 1, power slack: jobs run in priority order; the objective is
    WT * sum max(C_j - D_j, 0) + C_max summed directly."""
    inst = W.random_instance(11, n_jobs=6, n_stages=1, machines=1, release_max=10, wt=7)
    inst.q_max = 1000
    prio = np.array([3, 6, 1, 5, 2, 4])
    order = _order_by_priority(prio, inst.active)
    t = 0
    comp = {}
    for j in order:
        t = max(t, int(inst.release[j])) + int(inst.proc[j][0][0])
        comp[j] = t
    want = 7 * sum(max(comp[j] - int(inst.due[j]), 0) for j in comp) + t
    assert oracle.decode(inst, prio) == want


def test_identical_parallel_machines_list_scheduling():
    """g = 1, identical machines, no power limit, releases 0: Graham's list
    scheduling; each job in priority order goes to the machine that frees
    first (lowest index on ties)."""
    for m in (2, 3, 5):
        inst = W.random_instance(m, n_jobs=9, n_stages=1, machines=m)
        inst.proc[:] = inst.proc[:, :, :1]
        inst.q_max = 10**6
        prio = np.random.default_rng(m).permutation(9) + 1
        obj, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
        free = [0] * m
        for j in _order_by_priority(prio, inst.active):
            k = free.index(min(free))
            assert mach[j][0] == k and start[j][0] == free[k]
            free[k] += int(inst.proc[j][0][0])
        assert obj % 1 == 0


def test_machine_choice_is_earliest_completion_on_unrelated_machines():
    """With unrelated machines the chosen machine minimises max(est, free) + P_jsm,
    not the free time: a slow idle machine loses to a fast busy one."""
    inst = W.random_instance(0, n_jobs=2, n_stages=1, machines=2)
    inst.proc[0, 0] = [10, 10]
    inst.proc[1, 0] = [3, 30]      # job 1: fast on machine 0 (busy until 10), slow on 1
    inst.q_max = 100
    prio = np.array([2, 1])        # job 0 first
    obj, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
    assert mach[0][0] == 0 and mach[1][0] == 0 and start[1][0] == 10


# --------------------------------------------------------------------------
# Two independent decoders agree; every plan is valid and earliest.
# --------------------------------------------------------------------------
def _event_instances():
    out = []
    for seed in range(6):
        machines = [1 + (seed + s) % 3 for s in range(3)]
        inst = W.random_instance(seed, n_jobs=6 + seed, n_stages=3, machines=machines,
                                 release_max=seed * 5, percent=40 + 10 * (seed % 4))
        out.append(inst)
        # a later event: freeze a decoded plan at a point inside it
        prio = W.random_population(seed, 1, inst.n_active)[0]
        obj, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
        cm = int((start + 1).max())
        rs = cm // 3
        arr = W.random_arrival(seed + 100, inst, rs, 3)
        nxt = oracle.reschedule(inst, start, mach, rs, arr.proc, arr.power, arr.release, arr.due)
        out.append(W.Instance.from_fields(nxt))
    return out


def test_dense_and_event_list_decoders_agree():
    for inst in _event_instances():
        pop = W.random_population(7, 12, inst.n_active)
        for prio in pop:
            o1, s1, m1, _ = oracle.decode(inst, prio, want_schedule=True)
            o2, s2, m2 = eventlist.decode(inst, prio)
            dec = np.zeros_like(s1, bool)
            for j in inst.active:
                dec[j, inst.first_stage[j]:] = True
            assert o1 == o2
            assert (s1[dec] == s2[dec]).all() and (m1[dec] == m2[dec]).all()


def test_decoded_plans_meet_invariants_and_are_earliest():
    for inst in _event_instances()[:6]:
        if inst.rs != 0:
            continue
        pop = W.random_population(9, 10, inst.n_active)
        for prio in pop:
            obj, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
            got = validate.check_plan(inst.proc, inst.power, inst.release, inst.due,
                                      inst.n_machines, inst.q_max, inst.wt, start, mach)
            assert got == obj
            # replay in decode order: each op starts at its earliest feasible slot
            intervals = []
            free = np.zeros_like(inst.machine_free)
            done = {int(j): int(inst.release[j]) for j in inst.active}
            for s in range(inst.n_stages):
                for j in _order_by_priority(prio, inst.active):
                    m = int(mach[j][s])
                    p = int(inst.proc[j][s][m])
                    q = int(inst.power[j][s][m])
                    t0 = max(done[j], int(free[s][m]))
                    ends = [max(done[j], int(free[s][k])) + int(inst.proc[j][s][k])
                            for k in range(inst.n_machines[s])]
                    assert ends[m] == min(ends) and ends.index(min(ends)) == m
                    st = int(start[j][s])
                    assert st >= t0 and eventlist._feasible(intervals, st, p, q, inst.q_max)
                    for t in range(t0, st):
                        assert not eventlist._feasible(intervals, t, p, q, inst.q_max)
                    intervals.append((st, st + p, q))
                    free[s][m] = st + p
                    done[j] = st + p


def test_rescheduled_plans_meet_invariants():
    for inst0_seed in range(4):
        inst = W.random_instance(inst0_seed, n_jobs=8, n_stages=3, machines=2, percent=50)
        prio = W.random_population(inst0_seed, 1, 8)[0]
        _, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
        rs = int(start.max()) // 2
        arr = W.random_arrival(inst0_seed, inst, rs, 3)
        nxt = W.Instance.from_fields(oracle.reschedule(inst, start, mach, rs, arr.proc, arr.power,
                                                       arr.release, arr.due))
        full_s = np.vstack([start, np.full((3, 3), -1, np.int32)])
        full_m = np.vstack([mach, np.full((3, 3), -1, np.int32)])
        for prio2 in W.random_population(1, 5, nxt.n_active):
            obj, s2, m2, _ = oracle.decode(nxt, prio2, want_schedule=True)
            plan_s = np.where(s2 >= 0, s2, full_s)
            plan_m = np.where(m2 >= 0, m2, full_m)
            plan_s = full_s.copy()
            plan_m = full_m.copy()
            for j in nxt.active:
                f = nxt.first_stage[j]
                plan_s[j, f:] = s2[j, f:]
                plan_m[j, f:] = m2[j, f:]
            decoded = np.zeros_like(plan_s, bool)
            for j in nxt.active:
                decoded[j, nxt.first_stage[j]:] = True
            got = validate.check_plan(nxt.proc, nxt.power, nxt.release, nxt.due, nxt.n_machines,
                                      nxt.q_max, nxt.wt, plan_s, plan_m, rs=rs, decoded=decoded)
            assert got == obj


def test_infeasible_power_is_reported():
    inst = W.random_instance(0, n_jobs=3, n_stages=2, machines=2)
    inst.power[1, 1, 0] = inst.q_max + 1
    with pytest.raises(oracle.OracleError) as e:
        oracle.decode(inst, np.array([1, 2, 3]))
    assert e.value.code == oracle.E_INFEASIBLE


def test_non_permutation_is_rejected():
    inst = W.random_instance(0, n_jobs=3, n_stages=2, machines=2)
    with pytest.raises(oracle.OracleError):
        oracle.decode(inst, np.array([1, 1, 3]))


def test_empty_active_set():
    inst = W.random_instance(0, n_jobs=3, n_stages=2, machines=2)
    prio = np.array([1, 2, 3])
    _, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
    rs = int(start.max()) + 1000
    nxt = W.Instance.from_fields(oracle.reschedule(inst, start, mach, rs, np.zeros((0, 2, 2)),
                                                   np.zeros((0, 2, 2)), [], []))
    assert nxt.n_active == 0 and len(nxt.running) == 0
    comp = [int(start[j][1] + inst.proc[j][1][mach[j][1]]) for j in range(3)]
    want = inst.wt * sum(max(c - int(d), 0) for c, d in zip(comp, inst.due)) + max(comp)
    assert oracle.decode(nxt, np.zeros(0, np.int32)) == want


# --------------------------------------------------------------------------
# Brute force over all priority vectors; the GA never reports better.
# --------------------------------------------------------------------------
def test_bruteforce_bounds_the_ga():
    for seed, n in ((0, 5), (1, 6), (2, 7)):
        inst = W.random_instance(seed, n_jobs=n, n_stages=3, machines=2, percent=50)
        perms = np.array(list(itertools.permutations(range(1, n + 1))), np.int32)
        best = int(oracle.decode_pop(inst, perms, n_threads=4).min())
        ga = W.GaParams(2, 4, 4, mig_k=1)
        st = oracle.ga_run(inst, ga, seed=seed, shop=0, event=0, generations=30, n_threads=4)
        prio, obj = oracle.ga_best(st)
        assert obj >= best
        assert oracle.decode(inst, prio) == obj        # the reported fitness is exact
        assert obj == best                              # tiny case: the GA finds the optimum


# --------------------------------------------------------------------------
# GA: elitism, migration snapshot, selection neighbourhood, determinism.
# --------------------------------------------------------------------------
def test_elite_is_monotone_and_best_in_history():
    inst = W.random_instance(4, n_jobs=12, n_stages=3, machines=2, percent=50)
    ga = W.GaParams(4, 4, 4, mig_interval=5, mig_k=2)
    st = oracle.ga_init(inst, ga, 1, 0, 0)
    best_seen = st["obj"].reshape(4, 16).min(axis=1)
    for k in range(1, 21):
        nxt = oracle.ga_generation(inst, ga, 1, 0, 0, k, st)
        assert (nxt["elite_obj"] <= st["elite_obj"]).all()
        for I in range(4):
            assert oracle.decode(inst, nxt["elite"][I]) == nxt["elite_obj"][I]
            assert nxt["elite_obj"][I] in nxt["obj"][I * 16:(I + 1) * 16]
        best_seen = np.minimum(best_seen, nxt["obj"].reshape(4, 16).min(axis=1))
        st = nxt
    assert (st["elite_obj"] <= best_seen).all()


def test_migration_moves_best_of_predecessor_into_worst():
    inst = W.random_instance(5, n_jobs=10, n_stages=3, machines=2, percent=50)
    K = 8
    ga_mig = W.GaParams(3, 2, 4, mig_interval=1, mig_k=2)
    ga_none = W.GaParams(3, 2, 4, mig_interval=1, mig_k=0)
    st = oracle.ga_init(inst, ga_mig, 2, 0, 0)
    a = oracle.ga_generation(inst, ga_mig, 2, 0, 0, 1, st)
    b = oracle.ga_generation(inst, ga_none, 2, 0, 0, 1, st)   # same state before migration
    for I in range(3):
        src = (I - 1) % 3
        so = b["obj"][src * K:(src + 1) * K]
        best = sorted(range(K), key=lambda i: (so[i], i))[:2]
        do = b["obj"][I * K:(I + 1) * K]
        worst = sorted(range(K), key=lambda i: (-do[i], i))[:2]
        for r in range(2):
            assert (a["prio"][I * K + worst[r]] == b["prio"][src * K + best[r]]).all()
            assert a["obj"][I * K + worst[r]] == b["obj"][src * K + best[r]]
        others = [i for i in range(K) if i not in worst]
        assert (a["prio"][[I * K + i for i in others]] == b["prio"][[I * K + i for i in others]]).all()
        assert a["elite_obj"][I] == min(b["elite_obj"][I], b["obj"][src * K + best[0]])


def test_selection_neighbourhood_fixture():
    """With crossover and mutation off, each slot holds the best of itself and its
    four torus neighbours in the order self, up, down, left, right (first on
    ties), except the island's worst child, which the elite overwrites.
    Worked by hand on a 3x4 island whose objectives include ties between self
    and neighbours and between two neighbours."""
    inst = W.random_instance(6, n_jobs=9, n_stages=2, machines=2)
    ga = W.GaParams(1, 3, 4, pc=0, pm=0, mig_k=0)
    st = oracle.ga_init(inst, ga, 3, 0, 0)
    grid = np.array([[10, 40, 60, 10],
                     [70, 30, 80, 20],
                     [10, 45, 35, 40]], np.int64)
    # by hand, e.g. (1,0): up (0,0)=10 and down (2,0)=10 tie, up wins -> slot 0;
    # (2,3): down (0,3)=10 and right (2,0)=10 tie, down wins -> slot 3;
    # (0,0): self 10 ties up and left, self wins -> slot 0.
    winners = [[0, 0, 3, 3],
               [0, 5, 7, 3],
               [8, 8, 10, 3]]
    st["obj"] = grid.reshape(-1)
    out = oracle.ga_generation(inst, ga, 3, 0, 0, 1, st)
    child_obj = [oracle.decode(inst, st["prio"][winners[i // 4][i % 4]]) for i in range(12)]
    worst = int(np.argmax(child_obj))           # first slot of maximal objective
    best = int(np.argmin(child_obj))
    elite = st["elite"][0]
    if child_obj[best] < st["elite_obj"][0]:    # the elite is refreshed before it replaces
        elite = st["prio"][winners[best // 4][best % 4]]
    for i in range(12):
        r, c = divmod(i, 4)
        want = elite if i == worst else st["prio"][winners[r][c]]
        assert (out["prio"][i] == want).all(), (r, c)


def test_crossover_pairs_follow_generation_parity():
    """Odd generations pair (r,2c)-(r,2c+1), even ones (2r,c)-(2r+1,c); the lower
    slot's purpose-1 draw decides and cuts. With selection neutralised (equal
    objectives keep every slot's own chromosome) and mutation off, every child
    is its own parent's head plus its partner's tail, corrected."""
    inst = W.random_instance(8, n_jobs=10, n_stages=2, machines=2)
    ga = W.GaParams(1, 4, 4, pc=2**32 - 1, pm=0, mig_k=0)
    st = oracle.ga_init(inst, ga, 4, 9, 2)
    st["obj"] = np.zeros(16, np.int64)
    for gen in (1, 2):
        out = oracle.ga_generation(inst, ga, 4, 9, 2, gen, st)
        wants = []
        for i in range(16):
            r, c = divmod(i, 4)
            if gen % 2 == 1:
                lead = r * 4 + (c // 2) * 2
                partner = lead + 1 if i == lead else lead
            else:
                lead = (r // 2) * 8 + c
                partner = lead + 4 if i == lead else lead
            w = oracle.philox4x64_10([lead, gen, 2, 1 << 32], [4, 9])
            cut = 1 + ((int(w[1]) >> 32) * 9 >> 32)
            mine = st["prio"][i]
            other = st["prio"][partner]
            wants.append(oracle.correct(np.concatenate([mine[:cut], other[cut:]])))
        objs = [oracle.decode(inst, w) for w in wants]
        worst = int(np.argmax(objs))
        best = int(np.argmin(objs))
        elite = wants[best] if objs[best] < st["elite_obj"][0] else st["elite"][0]
        for i in range(16):
            want = elite if i == worst else wants[i]
            assert (out["prio"][i] == want).all(), (gen, i)


def test_ga_is_deterministic_and_seed_sensitive():
    inst = W.random_instance(7, n_jobs=10, n_stages=3, machines=2, percent=50)
    ga = W.GaParams(2, 4, 4, mig_k=1)
    a = oracle.ga_run(inst, ga, 5, 0, 0, 12)
    b = oracle.ga_run(inst, ga, 5, 0, 0, 12, n_threads=4)
    c = oracle.ga_run(inst, ga, 6, 0, 0, 12)
    assert all((a[k] == b[k]).all() for k in a)
    assert not (a["prio"] == c["prio"]).all()


def test_island_subset_generation_matches_full():
    inst = W.random_instance(9, n_jobs=11, n_stages=3, machines=2, percent=50)
    ga = W.GaParams(5, 2, 4, mig_interval=2, mig_k=2)
    st = oracle.ga_run(inst, ga, 8, 0, 1, 3)
    for gen in (4, 5):   # a migrating and a plain generation
        full = oracle.ga_generation(inst, ga, 8, 0, 1, gen, st)
        sel = np.zeros(5, bool)
        sel[[0, 3]] = True
        part = oracle.ga_generation(inst, ga, 8, 0, 1, gen, st, island_sel=sel)
        for I in (0, 3):
            sl = slice(I * 8, (I + 1) * 8)
            assert (part["prio"][sl] == full["prio"][sl]).all()
            assert (part["obj"][sl] == full["obj"][sl]).all()
            assert part["elite_obj"][I] == full["elite_obj"][I]


def test_freeze_boundaries_follow_algorithm1():
    """Algorithm 1: an op is running at RS iff S < RS < S + P (z = 0); an op that
    started before RS and ended by RS is finished (z = C); an op starting at RS
    or later is rescheduled (x = y = -1 only for ops started before RS)."""
    # 3 jobs, 2 stages, 1 machine each, P = 10 everywhere, Q = 1, release 0
    proc = np.full((3, 2, 1), 10, np.int32)
    inst = W.initial_instance(proc, np.ones((3, 2, 1)), [0, 0, 0], [100, 100, 100], [1, 1], 5, 1)
    rs = 20
    start = np.array([[0, 10],    # job 0: stage 1 ends exactly at RS -> finished
                      [10, 20],   # job 1: stage 0 ends at RS (finished), stage 1 starts at RS
                      [15, 30]],  # job 2: stage 0 runs over RS -> running until 25
                     np.int32)
    mach = np.zeros((3, 2), np.int32)
    nxt = W.Instance.from_fields(oracle.reschedule(inst, start, mach, rs, np.zeros((0, 2, 1)),
                                                   np.zeros((0, 2, 1)), [], []))
    assert list(nxt.first_stage) == [2, 1, 1]
    assert nxt.running.tolist() == [[25, 1]]
    assert list(nxt.active) == [1, 2]
    assert nxt.ready[1] == 20 and nxt.ready[2] == 25
    assert nxt.frozen_cmax == 20 and nxt.frozen_tardiness == 0
    assert nxt.machine_free[0][0] == 25 and nxt.machine_free[1][0] == 20


def test_island_subset_runs_follow_the_migration_cone():
    """oracle_islands (the tests' subset runs) equals the whole run on its target
    islands, across migrating generations."""
    from oracle_helpers import oracle_islands
    inst = W.random_instance(31, n_jobs=9, n_stages=2, machines=2)
    ga = W.GaParams(8, 2, 4, mig_interval=3, mig_k=2)
    full = oracle.ga_run(inst, ga, 4, 1, 0, 7)
    K = ga.rows * ga.cols
    for islands in ([0], [3, 6], [7]):
        part = oracle_islands(inst, ga, 4, 1, 0, islands, 7)
        for I in islands:
            sl = slice(I * K, (I + 1) * K)
            assert (part["prio"][sl] == full["prio"][sl]).all()
            assert (part["obj"][sl] == full["obj"][sl]).all()
            assert (part["elite"][I] == full["elite"][I]).all()
            assert part["elite_obj"][I] == full["elite_obj"][I]
