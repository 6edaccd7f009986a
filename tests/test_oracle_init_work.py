"""Pins of the oracle's population initialisation and of its work count.

* Initialisation (Section 4.3: unique priorities, generated randomly): a
  Durstenfeld shuffle worked by hand from numpy's Philox words
  (tests/golden/fisher_yates_init.txt), and a chi-square test that every
  permutation of four genes is equally likely — a Sattolo-type slip (draws
  on 0..pos-1) never yields the identity and only reaches the 6 cyclic
  permutations; a wrong draw range skews the counts.
* Work count W, the numerator of the roofline: per placed op, 3 * o_s for the
  machine choice, the slots from the op's first candidate start t0 up to its
  start, and 2p (p slots of the window examined, p slots updated); the X/Y
  decode has no machine choice. Recomputed here from the decoded plan alone:
  t0 = max(RS, end of the job's previous stage or its ready time, end of the
  op before it on its machine). Machines are append-only, so the op before it
  is the one of latest start below its own, or the frozen free time.
"""
import itertools

import numpy as np
import pytest
from scipy import stats

import oracle
from paper_1903_10741_amd import workloads as W
from tests.golden_io import read


def _fixture():
    f = read("fisher_yates_init.txt")
    key = [int(v) for v in f["key"][0]]
    words = {int(r[0]): int(r[1], 16) for r in f["word"]}
    steps = [r for r in f["step"]]
    return dict(key=key, individual=int(f["individual"][0][0]), event=int(f["event"][0][0]),
                n=int(f["n"][0][0]), words=words, steps=steps,
                result=[int(v) for v in f["result"][0]])


def test_fisher_yates_fixture_words_are_numpy_philox():
    fx = _fixture()
    for d, w in fx["words"].items():
        ctr = np.array([fx["individual"] - 1, 0, fx["event"], d // 4], dtype=np.uint64)
        g = np.random.Philox(counter=ctr, key=np.array(fx["key"], dtype=np.uint64))
        assert int(g.random_raw(4)[d % 4]) == w


def test_fisher_yates_fixture_is_a_consistent_hand_replay():
    """Each recorded step swaps entries pos and r of the previous array, and
    its quotient column rounds down to r (a check of the worked fixture)."""
    fx = _fixture()
    n = fx["n"]
    arr = list(range(1, n + 1))
    for row in fx["steps"]:
        d, pos, hi, quo, r = int(row[0]), int(row[1]), int(row[2]), float(row[3]), int(row[4])
        after = [int(v) for v in row[5:]]
        assert pos == n - 1 - d and hi == fx["words"][d] >> 32
        assert abs(quo - hi * (pos + 1) / 2**32) < 1e-3 and r == int(quo) and 0 <= r <= pos
        arr[pos], arr[r] = arr[r], arr[pos]
        assert arr == after
    assert arr == fx["result"]


def _tiny_instance(n, seed=0):
    return W.random_instance(seed, n_jobs=n, n_stages=2, machines=2)


def test_oracle_init_replays_the_fixture():
    fx = _fixture()
    inst = _tiny_instance(fx["n"])
    ga = W.GaParams(1, 2, 4)
    st = oracle.ga_init(inst, ga, fx["key"][0], fx["key"][1], fx["event"])
    assert st["prio"][fx["individual"]].tolist() == fx["result"]


def test_init_is_uniform_over_all_permutations():
    n = 4
    inst = _tiny_instance(n, seed=1)
    ga = W.GaParams(192, 8, 16)   # 24 576 individuals
    st = oracle.ga_init(inst, ga, 11, 0, 0, n_threads=8)
    perms = {p: k for k, p in enumerate(itertools.permutations(range(1, n + 1)))}
    counts = np.zeros(len(perms), np.int64)
    for row in st["prio"]:
        counts[perms[tuple(int(v) for v in row)]] += 1
    assert counts.min() > 0, "some permutation never drawn (a Sattolo-type shuffle reaches 6 of 24)"
    _, pval = stats.chisquare(counts)
    assert pval > 1e-4, (counts, pval)


def test_init_differs_per_individual_event_and_key():
    inst = _tiny_instance(12, seed=2)
    ga = W.GaParams(2, 2, 4)
    a = oracle.ga_init(inst, ga, 5, 0, 0)["prio"]
    assert len({tuple(r) for r in a.tolist()}) == len(a)
    for other in (oracle.ga_init(inst, ga, 5, 0, 1)["prio"], oracle.ga_init(inst, ga, 6, 0, 0)["prio"],
                  oracle.ga_init(inst, ga, 5, 1, 0)["prio"]):
        assert (other != a).any(axis=1).all()
    for row in a:
        assert sorted(row.tolist()) == list(range(1, 13))


# --------------------------------------------------------------------------
# Work count recomputed from decoded plans.
# --------------------------------------------------------------------------
def _work_from_plan(inst, start, mach, machine_choice):
    g = int(inst.n_stages)
    nm = np.asarray(inst.n_machines)
    proc = np.asarray(inst.proc).reshape(int(inst.n_jobs), g, -1)
    mfree = np.asarray(inst.machine_free).reshape(g, -1)
    first = np.asarray(inst.first_stage)
    ready = np.asarray(inst.ready)
    rs = int(inst.rs)
    ops = [(int(j), s) for j in inst.active for s in range(int(first[j]), g)]
    total = 0
    for j, s in ops:
        S, m = int(start[j, s]), int(mach[j, s])
        p = int(proc[j, s, m])
        prev_end = int(ready[j]) if s == first[j] else int(start[j, s - 1] + proc[j, s - 1, mach[j, s - 1]])
        before = [int(start[k, s] + proc[k, s, mach[k, s]]) for k, t in ops
                  if t == s and mach[k, t] == m and start[k, t] < S]
        free = max(before) if before else int(mfree[s, m])
        t0 = max(rs, prev_end, free)
        assert S >= t0
        total += (3 * int(nm[s]) if machine_choice else 0) + (S - t0) + 2 * p
    return total


def _instances():
    out = [W.config1(0).initial, W.config2(3).initial,
           W.random_instance(4, n_jobs=9, n_stages=3, machines=[2, 3, 1], percent=45)]
    # rescheduled instances: frozen ops, running ops holding power, busy machines
    for sd in range(3):
        inst = W.random_instance(10 + sd, n_jobs=8, n_stages=3, machines=2, percent=50)
        _, start, mach, _ = oracle.decode(inst, W.random_population(sd, 1, 8)[0], want_schedule=True)
        rs = int(start.max()) // 2
        arr = W.random_arrival(sd, inst, rs, 3)
        out.append(W.Instance.from_fields(oracle.reschedule(inst, start, mach, rs, arr.proc,
                                                            arr.power, arr.release, arr.due)))
    return out


@pytest.mark.parametrize("k", range(6))
def test_work_count_recomputed_from_plan(k):
    inst = _instances()[k]
    assert inst.n_active > 0
    for prio in W.random_population(100 + k, 4, inst.n_active):
        _, start, mach, work = oracle.decode(inst, prio, want_schedule=True, want_work=True)
        assert work == _work_from_plan(inst, start, mach, True)


@pytest.mark.parametrize("k", range(6))
def test_xy_work_count_recomputed_from_plan(k):
    inst = _instances()[k]
    for genes in W.random_xy_population(200 + k, 3, inst):
        _, start, mach, work = oracle.decode_xy(inst, genes, want_schedule=True, want_work=True)
        assert work == _work_from_plan(inst, start, mach, False)


def test_work_count_on_a_long_horizon_with_many_pushes():
    """Tight peak and long ops: many delayed starts, a work sum past 2^31 is not
    needed but the per-op gaps are large."""
    inst = W.random_instance(21, n_jobs=40, n_stages=4, machines=3, p_max=400, q_range=(5, 10),
                             percent=30)
    for prio in W.random_population(5, 3, inst.n_active):
        _, start, mach, work = oracle.decode(inst, prio, want_schedule=True, want_work=True)
        assert work == _work_from_plan(inst, start, mach, True)
        assert work > 40 * 4 * 400


def test_initial_elite_is_the_best_in_history():
    """Generation 0 is the whole history of an island (Section 4.4, replacement keeps
    the best in history): each island's elite is its best initial individual."""
    inst = W.config2(1).initial
    ga = W.GaParams(4, 4, 8)
    st = oracle.ga_init(inst, ga, 3, 0, 0, n_threads=8)
    K = ga.rows * ga.cols
    for I in range(ga.islands):
        objs = st["obj"][I * K:(I + 1) * K]
        assert st["elite_obj"][I] == objs.min()
        assert oracle.decode(inst, st["elite"][I]) == objs.min()
        assert any((st["prio"][I * K + k] == st["elite"][I]).all() for k in range(K))
