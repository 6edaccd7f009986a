"""The comparison GAs of Section 5.2 in the oracle (classical and cellular),
pinned to their definitions: eq. (13)'s E_max, fitness-proportional
selection (chi-square), the cellular replacement as a neighbourhood minimum,
and brute force on tiny instances."""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1903_10741_amd import workloads as W

NO_OPS = dict(pc=0, pm=0)   # selection and replacement alone


@pytest.mark.parametrize("objs,want", [([1], 10), ([9], 10), ([10], 100), ([5, 99, 3], 100),
                                       ([100], 1000), ([529121, 703624], 1000000),
                                       ([999999999], 1000000000)])
def test_emax_is_the_least_power_of_ten_above_every_objective(objs, want):
    """Section 5.1: a increases from 1 until every initial objective is below 10^a."""
    assert oracle.emax(np.array(objs, np.int64)) == want


def _identical_jobs(n):
    """n identical jobs: every priority vector decodes to the same objective, so the
    replacement's worst child is always slot 0 (lowest slot on ties), whatever
    its parent."""
    proc = np.full((n, 2, 2), 5, np.int32)
    return W.initial_instance(proc, np.ones((n, 2, 2), np.int32), np.zeros(n, np.int32),
                              np.full(n, 40, np.int32), [2, 2], 2, 10)


def _state(pop, n, obj, seed=0):
    rng = np.random.default_rng(seed)
    prio = np.stack([rng.permutation(n) + 1 for _ in range(pop)]).astype(np.int32)
    return {"prio": prio, "obj": np.asarray(obj, np.int64),
            "elite": np.arange(n, 0, -1, dtype=np.int32)[None], "elite_obj": np.array([0])}


def test_roulette_selects_in_proportion_to_eq13_fitness():
    """Classical GA without crossover and mutation: each slot copies the parent its
    spin picks; over many generations the picks follow F_i / sum F with
    F_i = max(E_max - obj_i, 0), and an individual of fitness 0 is never picked."""
    inst = _identical_jobs(12)
    ga = W.GaParams(1, 4, 8, **NO_OPS)
    pop, n, e_max = 32, 12, 1000
    obj = np.array([1000, 1500] + list(np.linspace(100, 990, pop - 2).astype(np.int64)))
    st = _state(pop, n, obj)
    rows = {tuple(r): i for i, r in enumerate(st["prio"])}
    counts = np.zeros(pop)
    for g in range(1, 601):
        out = oracle.ga_generation_scheme(inst, ga, oracle.GA_CLASSICAL, e_max, 5, 0, 0, g, st)
        for r in out["prio"]:
            i = rows.get(tuple(r))
            if i is not None:          # slot 0 holds the elite, no population row
                counts[i] += 1
    fit = np.maximum(e_max - obj, 0).astype(np.float64)
    assert counts[0] == 0 and counts[1] == 0
    exp = fit[2:] / fit.sum() * counts.sum()
    chi2, p = stats.chisquare(counts[2:], exp)
    assert p > 1e-3, (chi2, p)


def test_roulette_with_zero_total_fitness_is_uniform():
    inst = _identical_jobs(10)
    ga = W.GaParams(1, 4, 4, **NO_OPS)
    st = _state(16, 10, [5000] * 16, seed=1)
    rows = {tuple(r): i for i, r in enumerate(st["prio"])}
    counts = np.zeros(16)
    for g in range(1, 401):
        out = oracle.ga_generation_scheme(inst, ga, oracle.GA_CLASSICAL, 100, 7, 0, 0, g, st)
        for r in out["prio"]:
            if tuple(r) in rows:
                counts[rows[tuple(r)]] += 1
    assert stats.chisquare(counts).pvalue > 1e-3


def test_classical_pairs_exchange_tails_of_two_population_members():
    """With crossover always on and no mutation, each pair (2k, 2k+1) of children is
    the corrected head/tail exchange of two members of the previous population at
    one cut (Fig. 11's operator), and every child is a permutation."""
    inst = W.random_instance(4, n_jobs=9, n_stages=2, machines=2)
    ga = W.GaParams(1, 4, 4, pc=2**32 - 1, pm=0)
    st = oracle.ga_init(inst, ga, 3, 0, 0)
    out = oracle.ga_generation_scheme(inst, ga, oracle.GA_CLASSICAL, oracle.emax(st["obj"]), 3, 0,
                                      0, 1, st)
    members = [tuple(r) for r in st["prio"]]
    for k in range(0, 16, 2):
        a, b = out["prio"][k], out["prio"][k + 1]
        for v in (a, b):
            assert sorted(v) == list(range(1, 10))
        ok = False
        for pa, pb in itertools.product(members, repeat=2):
            for cut in range(1, 9):
                ca = oracle.correct(np.array(pa[:cut] + pb[cut:]))
                cb = oracle.correct(np.array(pb[:cut] + pa[cut:]))
                if (ca == a).all() and (cb == b).all():
                    ok = True
                    break
            if ok:
                break
        # the elite may have been written over one slot of this pair
        assert ok or any((out["prio"][s] == out["elite"][0]).all() for s in (k, k + 1)), k


def test_cellular_generation_is_a_neighbourhood_minimum():
    """Cellular GA without crossover and mutation: each cell's child is its best
    neighbour (self, up, down, left, right on the torus) and replaces the cell only
    if strictly better, so the new objectives are the five-point minimum filter of
    the old ones; the elite is the grid's best."""
    inst = W.random_instance(5, n_jobs=10, n_stages=2, machines=2)
    R, C = 4, 6
    ga = W.GaParams(1, R, C, **NO_OPS)
    st = oracle.ga_init(inst, ga, 9, 0, 0)
    for g in range(1, 4):
        out = oracle.ga_generation_scheme(inst, ga, oracle.GA_CELLULAR, 0, 9, 0, 0, g, st)
        o = st["obj"].reshape(R, C)
        want = np.minimum.reduce([o, np.roll(o, 1, 0), np.roll(o, -1, 0), np.roll(o, 1, 1),
                                  np.roll(o, -1, 1)])
        assert (out["obj"].reshape(R, C) == want).all()
        assert out["elite_obj"][0] == min(st["elite_obj"][0], want.min())
        for i in range(R * C):
            assert oracle.decode(inst, out["prio"][i]) == out["obj"][i]
        st = out


def test_cellular_never_loses_a_cell():
    inst = W.random_instance(6, n_jobs=11, n_stages=3, machines=2, percent=50)
    ga = W.GaParams(1, 6, 6)
    st = oracle.ga_init(inst, ga, 2, 0, 0)
    for g in range(1, 16):
        out = oracle.ga_generation_scheme(inst, ga, oracle.GA_CELLULAR, 0, 2, 0, 0, g, st)
        assert (out["obj"] <= st["obj"]).all()
        st = out


@pytest.mark.parametrize("scheme", [oracle.GA_CLASSICAL, oracle.GA_CELLULAR])
def test_bruteforce_bounds_the_comparison_gas(scheme):
    """Neither GA reports better than the optimum over all priority vectors, and the
    reported fitness is the exact decode. The cellular GA reaches the optimum on
    these tiny cases; the classical GA need not: with E_max = 10^a far above the
    objectives' spread, eq. (13) gives nearly equal fitness to everyone and the
    roulette's selection pressure is weak (Section 5.2 finds it the weakest)."""
    for seed, n in ((0, 5), (1, 6)):
        inst = W.random_instance(seed, n_jobs=n, n_stages=3, machines=2, percent=50)
        perms = np.array(list(itertools.permutations(range(1, n + 1))), np.int32)
        best = int(oracle.decode_pop(inst, perms, n_threads=4).min())
        st = oracle.ga_run_scheme(inst, W.GaParams(1, 6, 6), scheme, seed, 0, 0, 40, n_threads=4)
        prio, obj = oracle.ga_best(st)
        assert obj >= best and oracle.decode(inst, prio) == obj
        if scheme == oracle.GA_CELLULAR:
            assert obj == best


def test_cellular_keeps_the_cell_on_a_tie():
    """Identical jobs make every priority vector decode alike, so every child ties
    with its cell: "replaces the target individual if its solution is better"
    leaves every cell as it was, even with crossover and mutation always on."""
    inst = _identical_jobs(9)
    ga = W.GaParams(1, 4, 4, pc=2**32 - 1, pm=2**32 - 1)
    st = oracle.ga_init(inst, ga, 4, 0, 0)
    for g in range(1, 4):
        out = oracle.ga_generation_scheme(inst, ga, oracle.GA_CELLULAR, 0, 4, 0, 0, g, st)
        assert (out["prio"] == st["prio"]).all() and (out["obj"] == st["obj"]).all()
        st = out
