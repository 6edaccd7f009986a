"""Invariant checks on a schedule (Table 1; eqs. (1)-(10)).

TEST INFRASTRUCTURE ONLY. Given every job's processing and power data and a
complete plan (start, machine for every op of every job), checks the model's
constraints directly, and recomputes the objective from its definition.
"""
import numpy as np


def check_plan(proc, power, release, due, n_machines, q_max, wt, start, mach, rs=0,
               decoded=None):
    """Raise AssertionError on any violated constraint; return the objective eq. (1).

    decoded: optional bool [n_jobs][g] marking ops scheduled at this event;
    those must start at or after rs (eq. (10)).
    """
    proc = np.asarray(proc)
    power = np.asarray(power)
    start = np.asarray(start).astype(np.int64)
    mach = np.asarray(mach)
    n, g = start.shape
    ops = []
    for j in range(n):
        prev_end = int(release[j])
        for s in range(g):
            m = int(mach[j][s])
            assert 0 <= m < int(n_machines[s]), f"op ({j},{s}) machine {m} out of range"
            st = int(start[j][s])
            p = int(proc[j][s][m])
            assert st >= prev_end, f"op ({j},{s}) starts {st} before {prev_end} (eqs. 4-5)"
            if decoded is not None and decoded[j][s]:
                assert st >= rs, f"op ({j},{s}) starts {st} before RS {rs} (eq. 10)"
            prev_end = st + p
            ops.append((st, st + p, int(power[j][s][m]), s, m, j))
    # eq. (6): one op at a time per machine
    by_machine = {}
    for (a, b, _q, s, m, j) in ops:
        by_machine.setdefault((s, m), []).append((a, b, j))
    for key, lst in by_machine.items():
        lst.sort()
        for (a0, b0, j0), (a1, b1, j1) in zip(lst, lst[1:]):
            assert b0 <= a1, f"machine {key}: jobs {j0} and {j1} overlap"
    # eqs. (7)-(9): power at every instant within Q_max; u is 1 on [S, S+P)
    events = {}
    for (a, b, q, _s, _m, _j) in ops:
        events[a] = events.get(a, 0) + q
        events[b] = events.get(b, 0) - q
    level = 0
    for t in sorted(events):
        level += events[t]
        assert level <= q_max, f"power {level} > Q_max {q_max} from t={t}"
    # eqs. (1)-(3)
    comp = [int(start[j][g - 1]) + int(proc[j][g - 1][int(mach[j][g - 1])]) for j in range(n)]
    tard = sum(max(c - int(due[j]), 0) for j, c in enumerate(comp))
    return int(wt) * tard + (max(comp) if comp else 0)
