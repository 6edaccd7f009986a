"""Oracle runs shared by tests (calls only the oracle)."""
import numpy as np

import oracle
from paper_1903_10741_amd import workloads as W


def rescheduled_instance(wl, k_events=1, seed=3):
    """The instance after k_events arrivals, each frozen on an oracle-decoded
    random plan (the oracle's own rescheduling; no GPU output involved)."""
    inst = wl.initial
    g = inst.n_stages
    plan_s = np.full((inst.n_jobs, g), -1, np.int32)
    plan_m = np.full((inst.n_jobs, g), -1, np.int32)
    for e in range(k_events):
        prio = W.random_population(seed + e, 1, inst.n_active)[0]
        _, s, m, _ = oracle.decode(inst, prio, want_schedule=True)
        for j in inst.active:
            f = inst.first_stage[j]
            plan_s[j, f:] = s[j, f:]
            plan_m[j, f:] = m[j, f:]
        a = wl.arrivals[e]
        inst = W.Instance.from_fields(oracle.reschedule(inst, plan_s, plan_m, a.rs, a.proc, a.power,
                                                        a.release, a.due))
        plan_s = np.vstack([plan_s, np.full((len(a.release), g), -1, np.int32)])
        plan_m = np.vstack([plan_m, np.full((len(a.release), g), -1, np.int32)])
    return inst


def oracle_islands(inst, gacfg, seed, shop, event, islands, generations, checkpoints=()):
    """The oracle's own state after `generations`, valid for `islands`: generation 0
    whole, then each generation only for the islands the targets depend on (a
    migrating generation makes island I depend on its ring predecessor). With
    checkpoints, returns {generation: state} for them and `generations`."""
    I_n = gacfg.islands
    need = [None] * (generations + 1)
    cur = set(islands)
    for g in range(generations, 0, -1):
        need[g] = set(cur)
        if gacfg.mig_interval > 0 and gacfg.mig_k > 0 and I_n > 1 and g % gacfg.mig_interval == 0:
            cur = cur | {(i - 1) % I_n for i in cur}
    st = oracle.ga_init(inst, gacfg, seed, shop, event, n_threads=8)
    kept = {}
    for g in range(1, generations + 1):
        sel = np.zeros(I_n, bool)
        sel[sorted(need[g])] = True
        st = oracle.ga_generation(inst, gacfg, seed, shop, event, g, st, island_sel=sel, n_threads=8)
        if g in checkpoints:
            kept[g] = {k: np.array(v, copy=True) for k, v in st.items()}
    if checkpoints:
        kept[generations] = st
        return kept
    return st
