"""Second, independently written decoder: event-list form, pure Python.

TEST INFRASTRUCTURE ONLY. It computes the same schedule as the C oracle's
dense-timeline decoder by a different route, so the two pin each other.

The power profile is kept as a list of intervals (start, end, q) rather than
an array of slots. The earliest power-feasible start of an op with processing
time p and power q, no earlier than t0, is found among the candidates t0 and
every interval end after t0: the power over [t, t+p) is piecewise constant
and only falls where an interval ends, so a window that is infeasible at t
can only become feasible by moving its start to such an end (eqs. (7)-(9),
Algorithm 2's "delay until the earliest finishing operation ends").
A window [t, t+p) is feasible iff the power at t and at every interval start
inside (t, t+p) stays within Q_max - q.
"""
import numpy as np


def _power_at(intervals, x):
    return sum(q for (a, b, q) in intervals if a <= x < b)


def _feasible(intervals, t, p, q, q_max):
    points = [t] + [a for (a, b, _q) in intervals if t < a < t + p]
    return all(_power_at(intervals, x) + q <= q_max for x in points)


def earliest_start(intervals, t0, p, q, q_max):
    candidates = sorted({t0} | {b for (a, b, _q) in intervals if b > t0})
    for t in candidates:
        if _feasible(intervals, t, p, q, q_max):
            return t
    raise AssertionError("unreachable: past every interval the profile is empty")


def decode(inst, prio):
    """Decode a job-priority vector. Returns (obj, start[n_jobs][g], mach[n_jobs][g]).

    Reading (job-priority chromosome): jobs are taken by decreasing priority,
    stage by stage; each op goes to the machine of its stage that completes it
    earliest ignoring power (ties to the lowest machine), after the last op
    already placed on that machine, then is pushed right until the power fits.
    """
    g = int(inst.n_stages)
    active = [int(j) for j in np.asarray(inst.active).reshape(-1)]
    prio = [int(x) for x in np.asarray(prio).reshape(-1)]
    assert sorted(prio) == list(range(1, len(active) + 1))
    order = [j for _p, j in sorted(zip(prio, active), key=lambda t: -t[0])]
    proc = np.asarray(inst.proc)
    power = np.asarray(inst.power)
    n_mach = [int(x) for x in np.asarray(inst.n_machines)]
    rs = int(inst.rs)
    q_max = int(inst.q_max)
    free = np.asarray(inst.machine_free).astype(np.int64).copy()
    first = np.asarray(inst.first_stage)
    done = {j: int(np.asarray(inst.ready)[j]) for j in active}
    intervals = [(rs, int(e), int(q)) for (e, q) in np.asarray(inst.running).reshape(-1, 2) if e > rs]
    n = int(inst.n_jobs)
    start = np.full((n, g), -1, np.int64)
    mach = np.full((n, g), -1, np.int64)
    for s in range(g):
        for j in order:
            if first[j] > s:
                continue
            est = max(rs, done[j])
            ends = [max(est, int(free[s][m])) + int(proc[j][s][m]) for m in range(n_mach[s])]
            m = ends.index(min(ends))
            p = int(proc[j][s][m])
            q = int(power[j][s][m])
            t = earliest_start(intervals, max(est, int(free[s][m])), p, q, q_max)
            intervals.append((t, t + p, q))
            free[s][m] = t + p
            done[j] = t + p
            start[j][s] = t
            mach[j][s] = m
    due = np.asarray(inst.due)
    tard = int(inst.frozen_tardiness) + sum(max(done[j] - int(due[j]), 0) for j in active)
    cmax = max([int(inst.frozen_cmax)] + [done[j] for j in active])
    return int(inst.wt) * tard + cmax, start, mach
