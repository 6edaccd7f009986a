"""Oracle runs shared by tests (calls only the oracle)."""
import numpy as np

import oracle


def oracle_islands(inst, gacfg, seed, shop, event, islands, generations):
    """The oracle's own state after `generations`, valid for `islands`: generation 0
    whole, then each generation only for the islands the targets depend on (a
    migrating generation makes island I depend on its ring predecessor)."""
    I_n = gacfg.islands
    need = [None] * (generations + 1)
    cur = set(islands)
    for g in range(generations, 0, -1):
        need[g] = set(cur)
        if gacfg.mig_interval > 0 and gacfg.mig_k > 0 and I_n > 1 and g % gacfg.mig_interval == 0:
            cur = cur | {(i - 1) % I_n for i in cur}
    st = oracle.ga_init(inst, gacfg, seed, shop, event, n_threads=8)
    for g in range(1, generations + 1):
        sel = np.zeros(I_n, bool)
        sel[sorted(need[g])] = True
        st = oracle.ga_generation(inst, gacfg, seed, shop, event, g, st, island_sel=sel, n_threads=8)
    return st
