"""Pins of the oracle's X/Y chromosome (Section 4.3, eqs. (10)-(12), Algorithms
1-2; Section 4.4, Figs. 11-12) against the paper's printed example and against
independent formulations. CPU only."""
import itertools
import random

import numpy as np

import oracle
from oracle import validate
from paper_1903_10741_amd import workloads as W
from tests.golden_io import ints, read
from tests.test_oracle_pins import _example_rescheduled


def _genes_of(inst, M):
    """Row-major genes of a printed matrix over the unfrozen ops."""
    return [int(M[j][s]) for j in inst.active for s in range(int(inst.first_stage[j]), inst.n_stages)]


def _printed_y():
    return np.array([ints(r) for r in read("table4_example.txt")["Y"]])


def _greedy_by_prefix_min(inst, y):
    """The greedy Z written differently: sort ops by (min of y over the job's
    unfrozen stages up to this one, descending; then stage)."""
    keys, k = [], 0
    for j in inst.active:
        m = None
        for s in range(int(inst.first_stage[j]), inst.n_stages):
            m = y[k] if m is None else min(m, y[k])
            keys.append((-m, s, int(j)))
            k += 1
    return [(j, s) for _, s, j in sorted(keys)]


def test_printed_y_gives_printed_z_but_one_op():
    """Greedy Z from the printed Y(k) is the printed Z(k) with one op moved:
    the paper prints z(3,2) = 4, the greedy rule orders (3,2) seventh (the two
    rules of Algorithm 1 disagree there); every other op keeps its printed
    relative order."""
    e, inst = _example_rescheduled()
    yg = _genes_of(inst, _printed_y())
    assert sorted(yg) == list(range(1, 14))
    got = [tuple(map(int, r)) for r in oracle.xy_order(inst, yg)]
    Z = e["Z"]
    printed = [op for _, op in sorted((int(Z[j][s]), (j, s)) for j in range(8) for s in range(3)
                                      if Z[j][s] not in ("0", "C"))]
    assert printed.index((3, 2)) == 3 and got.index((3, 2)) == 6
    assert [o for o in got if o != (3, 2)] == [o for o in printed if o != (3, 2)]


def test_printed_x_y_decode_to_fig8_makespan():
    """Decoding the printed X(k) and Y(k) (greedy Z) gives the makespan of
    Fig. 8's caption, 20.42, a plan meeting every constraint, on X's machines."""
    e, inst = _example_rescheduled()
    xg = _genes_of(inst, e["X"])
    yg = _genes_of(inst, _printed_y())
    obj, start, mach, work = oracle.decode_xy(inst, xg + yg, want_schedule=True, want_work=True)
    k = 0
    for j in inst.active:
        for s in range(int(inst.first_stage[j]), 3):
            assert mach[j][s] == xg[k]
            k += 1
    full_start, full_mach = start.copy(), mach.copy()
    full_start[:6] = np.where(e["X"][:6] == -1, e["plan_start"], start[:6])
    full_mach[:6] = np.where(e["X"][:6] == -1, e["plan_mach"], mach[:6])
    comp = [int(full_start[j][2] + e["proc"][j][2][0]) for j in range(8)]
    assert max(comp) == ints(read("table4_example.txt")["expect_cmax"][0])[0] == 2042
    validate.check_plan(e["proc"], e["power"], e["release"], e["due"], e["nm"], e["q_max"],
                        e["wt"], full_start, full_mach, rs=e["rs"], decoded=e["X"] != -1)
    assert obj == e["wt"] * sum(max(c - int(d), 0) for c, d in zip(comp, e["due"])) + max(comp)


def test_greedy_order_equals_prefix_min_sort():
    """The oracle's literal greedy rule against an independent formulation,
    on random instances with frozen prefixes (later events)."""
    rng = random.Random(3)
    for seed in range(40):
        wl = W.config1(seed % 5)
        inst = wl.initial
        if seed % 2:
            st, mc = oracle.decode(inst, W.random_population(seed, 1, inst.n_active)[0],
                                   want_schedule=True)[1:3]
            arr = wl.arrivals[0]
            nxt = oracle.reschedule(inst, st, mc, arr.rs, arr.proc, arr.power, arr.release, arr.due)
            inst = W.Instance.from_fields(nxt)
        R = oracle.xy_ops(inst)
        y = rng.sample(range(1, R + 1), R)
        got = [tuple(map(int, r)) for r in oracle.xy_order(inst, y)]
        assert got == _greedy_by_prefix_min(inst, y)


def _stage_major_y(inst, prio):
    """Y ranking every stage-s op above every stage-(s+1) op, and within a stage
    the jobs by their priority (the job-vector decode's order)."""
    order = sorted(range(inst.n_active), key=lambda k: -int(prio[k]))
    ops = [(s, int(inst.active[k])) for s in range(inst.n_stages) for k in order
           if int(inst.first_stage[inst.active[k]]) <= s]
    rank = {op: len(ops) - i for i, op in enumerate(ops)}
    return [rank[(s, int(j))] for j in inst.active
            for s in range(int(inst.first_stage[j]), inst.n_stages)]


def test_xy_with_stage_major_y_and_ect_machines_equals_job_vector_decode():
    """The job-vector decode is the X/Y decode whose Y is stage-major by the job
    priorities and whose X holds the machines the job decode chose: the two
    decoders (independent code paths) must give the same plan."""
    for cfg, seed in ((1, 0), (1, 4), (2, 1)):
        wl = W.CONFIGS[cfg](seed)
        inst = wl.initial
        for prio in W.random_population(seed, 6, inst.n_active):
            obj, start, mach, _ = oracle.decode(inst, prio, want_schedule=True)
            xg = [int(mach[j][s]) for j in inst.active
                  for s in range(int(inst.first_stage[j]), inst.n_stages)]
            yg = _stage_major_y(inst, prio)
            obj2, start2, mach2, _ = oracle.decode_xy(inst, xg + yg, want_schedule=True)
            assert obj2 == obj
            assert (start2 == start).all() and (mach2 == mach).all()


def test_fig11_xy_crossover():
    """Fig. 11: one single-point cut on both matrices, then the Y correction."""
    f = read("fig11_crossover.txt")
    cut_elem = ints(f["cut_elements"][0])[0]
    xa, xb = ints(f["X_parent_a"][0]), ints(f["X_parent_b"][0])
    ya, yb = ints(f["Y_parent_a"][0]), ints(f["Y_parent_b"][0])
    free = [k for k, v in enumerate(ya) if v != -1]
    assert free == [k for k, v in enumerate(xa) if v != -1]

    def compact(v):
        return [v[k] for k in free]

    def expand(full, genes):
        out = list(full)
        for k, g in zip(free, genes):
            out[k] = g
        return out

    cut = sum(1 for k in free if k < cut_elem)
    ca, cb = oracle.crossover_xy(compact(xa) + compact(ya), compact(xb) + compact(yb), cut)
    R = len(free)
    assert expand(xa, ca[:R]) == ints(f["X_child_a"][0])
    assert expand(xb, cb[:R]) == ints(f["X_child_b"][0])
    assert expand(ya, ca[R:]) == ints(f["Y_corrected_a"][0])
    assert expand(yb, cb[R:]) == ints(f["Y_corrected_b"][0])


def test_fig12_xy_mutation_rule():
    """Fig. 12: every X entry takes another machine (two per stage here, so all
    flip) and two Y entries swap. The oracle's mutation, forced on every
    individual with crossover off, does exactly that to each selected parent."""
    f = read("fig12_mutation.txt")
    xb, xa = ints(f["X_before"][0]), ints(f["X_after"][0])
    assert all((a == -1) == (b == -1) and (b == -1 or a == 1 - b) for a, b in zip(xa, xb))
    yb, ya = ints(f["Y_before"][0]), ints(f["Y_after"][0])
    diff = [k for k in range(len(yb)) if yb[k] != ya[k]]
    assert len(diff) == 2 and yb[diff[0]] == ya[diff[1]] and yb[diff[1]] == ya[diff[0]]

    wl = W.config1(2)
    inst = wl.initial
    ga = W.GaParams(1, 4, 4, pc=0, pm=2**32 - 1, encoding=1)
    st = oracle.ga_init(inst, ga, 9, 0, 0)
    kids = oracle.ga_breed(inst, ga, 9, 0, 0, 1, 0, st)
    R = oracle.xy_ops(inst)
    K = 16
    for i in range(K):
        r, c = divmod(i, 4)
        cand = [i, ((r - 1) % 4) * 4 + c, ((r + 1) % 4) * 4 + c, r * 4 + (c - 1) % 4,
                r * 4 + (c + 1) % 4]
        w = cand[0]
        for k in cand[1:]:
            if st["obj"][k] < st["obj"][w]:
                w = k
        par, kid = st["prio"][w], kids[i]
        assert (kid[:R] == 1 - par[:R]).all()          # config 1: two machines per stage
        d = np.nonzero(kid[R:] != par[R:])[0]
        assert len(d) == 2 and kid[R + d[0]] == par[R + d[1]] and kid[R + d[1]] == par[R + d[0]]


def test_xy_best_over_all_chromosomes_not_worse_than_job_vectors():
    """Brute force on a tiny instance: every X/Y chromosome decodes to a valid
    plan, and the best X/Y objective is at most the best job-vector one (X/Y
    expresses every job-vector plan)."""
    inst = W.random_instance(5, n_jobs=3, n_stages=2, machines=2, percent=60)
    R = oracle.xy_ops(inst)
    assert R == 6
    best_job = min(oracle.decode(inst, p) for p in itertools.permutations(range(1, 4)))
    best_xy = None
    rng = random.Random(0)
    ys = list(itertools.permutations(range(1, R + 1)))
    for x in itertools.product((0, 1), repeat=R):
        for y in rng.sample(ys, 40):
            obj, st, mc, _ = oracle.decode_xy(inst, list(x) + list(y), want_schedule=True)
            if best_xy is None or obj < best_xy:
                best_xy = obj
            validate.check_plan(inst.proc, inst.power, inst.release, inst.due, inst.n_machines,
                                inst.q_max, inst.wt, st, mc)
    full = [oracle.decode_xy(inst, list(x) + _stage_major_y(inst, p))
            for p in itertools.permutations(range(1, 4)) for x in itertools.product((0, 1), repeat=R)]
    assert min(full) <= best_job and best_xy is not None


def test_xy_ga_elites_never_worsen_and_chromosomes_stay_valid():
    wl = W.config1(1)
    inst = wl.initial
    ga = W.GaParams(2, 4, 4, mig_interval=3, mig_k=1, encoding=1)
    R = oracle.xy_ops(inst)
    st = oracle.ga_init(inst, ga, 5, 1, 0)
    prev = st["elite_obj"].copy()
    for k in range(1, 13):
        st = oracle.ga_generation(inst, ga, 5, 1, 0, k, st)
        assert (st["elite_obj"] <= prev).all()
        prev = st["elite_obj"].copy()
        for v in st["prio"]:
            assert sorted(v[R:]) == list(range(1, R + 1))
            assert ((v[:R] >= 0) & (v[:R] < 2)).all()
    assert (oracle.decode_xy_pop(inst, st["elite"]) == st["elite_obj"]).all()
