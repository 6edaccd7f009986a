"""Pins of the oracle's decode variants (FIFO stage order, power-aware machine
choice) and of the Table 5-shaped instance preset. CPU only."""
import dataclasses
import itertools

import numpy as np

import oracle
from oracle import validate
from paper_1903_10741_amd import workloads as W


def _with(inst, rules):
    return dataclasses.replace(inst, decode_rules=rules)


def _earliest_fit(prof, q_max, t0, p, q):
    """Brute force: the first t >= t0 whose whole window [t, t+p) fits under Q_max."""
    t = t0
    while any(prof.get(x, 0) + q > q_max for x in range(t, t + p)):
        t += 1
    return t


def test_power_ect_equals_ect_when_power_never_binds():
    """With Q_max at least the total power of every op, no push-right moves an op
    and the power-aware choice is the plain earliest-completion choice."""
    for seed in range(4):
        inst = W.config2(seed).initial
        big = dataclasses.replace(inst, q_max=int(np.asarray(inst.power).sum()))
        for prio in W.random_population(seed, 5, inst.n_active):
            a = oracle.decode(big, prio, want_schedule=True)
            b = oracle.decode(_with(big, oracle.RULE_POWER_ECT), prio, want_schedule=True)
            assert a[0] == b[0] and (a[1] == b[1]).all() and (a[2] == b[2]).all()


def test_power_ect_equals_ect_on_identical_machines():
    """Machines of a stage identical in P and Q: both rules take the machine that
    frees first (the push-right is monotone in its lower bound)."""
    rng = np.random.default_rng(3)
    n, g, o = 8, 3, 3
    p_js = rng.integers(1, 15, size=(n, g))
    proc = np.repeat(p_js[:, :, None], o, axis=2).astype(np.int32)
    q_s = rng.integers(1, 6, size=g)
    power = np.broadcast_to(q_s[None, :, None], (n, g, o)).astype(np.int32).copy()
    inst = W.initial_instance(proc, power, np.zeros(n, np.int32), np.full(n, 40, np.int32),
                              np.full(g, o, np.int32), int(q_s.max()) + 2, 10)
    for prio in W.random_population(1, 20, n):
        a = oracle.decode(inst, prio, want_schedule=True)
        b = oracle.decode(_with(inst, oracle.RULE_POWER_ECT), prio, want_schedule=True)
        assert a[0] == b[0] and (a[1] == b[1]).all()


def test_power_ect_takes_the_machine_of_earliest_feasible_completion():
    """Brute force on the decoded plans: replaying the ops in decode order, each op's
    machine gives the earliest completion over all machines of its stage, each
    placed at its first window that fits (ties to the lowest machine), and the op
    starts exactly there. The work count follows the pruned search: 3 per machine,
    then the examined slots and p of the machine of least bound max(est, free) + p
    and of every other machine whose (bound, index) is below the best (completion,
    index) so far, then p updated."""
    for seed in range(6):
        inst = W.random_instance(seed, n_jobs=6, n_stages=2, machines=[2, 3], p_max=9,
                                 q_range=(1, 6), percent=45)
        rules = _with(inst, oracle.RULE_POWER_ECT)
        for prio in W.random_population(seed, 8, inst.n_active):
            obj, start, mach, work = oracle.decode(rules, prio, want_schedule=True)
            want_work = 0
            validate.check_plan(inst.proc, inst.power, inst.release, inst.due, inst.n_machines,
                                inst.q_max, inst.wt, start, mach)
            order = [j for _, j in sorted((-int(prio[k]), int(j)) for k, j in enumerate(inst.active))]
            prof, free = {}, {}
            done = {int(j): int(inst.release[j]) for j in inst.active}
            for s in range(inst.n_stages):
                for j in order:
                    best, fits = None, {}
                    o_s = int(inst.n_machines[s])
                    for m in range(o_s):
                        p, q = int(inst.proc[j][s][m]), int(inst.power[j][s][m])
                        t0 = max(done[j], free.get((s, m), 0))
                        t = _earliest_fit(prof, inst.q_max, t0, p, q)
                        fits[m] = (t0 + p, t - t0 + p)  # bound, examined slots + p
                        if best is None or t + p < best[0]:
                            best = (t + p, m, t)
                    assert mach[j][s] == best[1] and start[j][s] == best[2]
                    first = min(range(o_s), key=lambda m: (fits[m][0], m))
                    done_best = None
                    want_work += 3 * o_s
                    for m in [first] + [m for m in range(o_s) if m != first]:
                        if done_best is not None and (fits[m][0], m) >= done_best:
                            continue
                        want_work += fits[m][1]
                        end = fits[m][0] - int(inst.proc[j][s][m]) + fits[m][1]
                        if done_best is None or (end, m) < done_best:
                            done_best = (end, m)
                    p, q = int(inst.proc[j][s][best[1]]), int(inst.power[j][s][best[1]])
                    want_work += p
                    for x in range(best[2], best[2] + p):
                        prof[x] = prof.get(x, 0) + q
                    free[(s, best[1])] = done[j] = best[2] + p
            assert work == want_work


def test_fifo_orders_each_stage_by_previous_completion():
    """FIFO: replaying the plan with stage 0 in priority order and each later stage
    sorted by the previous stage's completion (ties by priority) through the
    op-list decoder gives the same plan; with one stage FIFO is the priority order."""
    for cfg, seed in ((1, 0), (1, 2), (2, 1)):
        inst = W.CONFIGS[cfg](seed).initial
        fifo = _with(inst, oracle.RULE_FIFO)
        for prio in W.random_population(seed, 5, inst.n_active):
            obj, start, mach, _ = oracle.decode(fifo, prio, want_schedule=True)
            rank = {int(j): -int(prio[k]) for k, j in enumerate(inst.active)}
            ops = []
            done = {j: int(inst.release[j]) for j in rank}
            for s in range(inst.n_stages):
                for j in sorted(rank, key=lambda j: (done[j], rank[j])):
                    ops.append((j, s, -1))
                for j in rank:
                    done[j] = int(start[j][s] + inst.proc[j][s][mach[j][s]])
            obj2, st2, mc2 = oracle.decode_ops(inst, ops)
            assert obj2 == obj and (st2 == start).all() and (mc2 == mach).all()
    one = W.random_instance(4, n_jobs=7, n_stages=1, machines=2)
    for prio in itertools.islice(itertools.permutations(range(1, 8)), 0, 200, 17):
        assert oracle.decode(_with(one, oracle.RULE_FIFO), prio) == oracle.decode(one, prio)


def test_rules_on_frozen_prefixes_and_both_rules_together():
    """Later events (frozen prefixes, running ops): every rule combination gives
    valid plans and the X/Y decode ignores the rules."""
    wl = W.config1(1)
    inst = wl.initial
    st, mc = oracle.decode(inst, W.random_population(0, 1, inst.n_active)[0], want_schedule=True)[1:3]
    a = wl.arrivals[0]
    nxt = W.Instance.from_fields(oracle.reschedule(inst, st, mc, a.rs, a.proc, a.power, a.release,
                                                   a.due))
    genes = W.random_xy_population(1, 3, nxt)
    base_xy = oracle.decode_xy_pop(nxt, genes)
    for rules in range(4):
        r = _with(nxt, rules)
        for prio in W.random_population(rules, 6, r.n_active):
            obj, start, mach, work = oracle.decode(r, prio, want_schedule=True)
            assert obj > 0 and work > 0
        assert (oracle.decode_xy_pop(r, genes) == base_xy).all()


def test_table5_preset_shape():
    for seed in range(5):
        inst = W.table5_instance(seed)
        proc = np.asarray(inst.proc)
        assert (proc == proc[0]).all() and (np.asarray(inst.power) == 1).all()
        assert inst.wt == 100 and inst.q_max == 4 and proc.min() >= 1 and proc.max() <= 5
        p_bar = proc[0].mean(axis=1).sum()
        assert (np.asarray(inst.release) >= 0).all() and (np.asarray(inst.release) < p_bar).all()
        slack = (np.asarray(inst.due) - np.asarray(inst.release)) / p_bar
        assert (slack >= 1 - 1e-9).all() and (slack <= 3 + 1 / p_bar).all()
        oracle.decode(inst, list(range(1, 11)))
