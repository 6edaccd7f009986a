"""Seeded synthetic EDFFS workloads.

This module only draws inputs: instances, arrival events, GA parameters and
random priority populations. It holds none of the method's arithmetic (no
decoding, no GA operator, no rescheduling) and serves the GPU path, the
tests and the benchmark alike.

The paper's experiments use random instances drawn from its Table 5
distributions, with no seeds published and no public benchmark; the recipes
below are synthetic stand-ins with the shapes of the configurations this
project measures (job counts, stages, machines per stage, processing-time
and power distributions, peak-power fraction, arrival events).

Draws use numpy's PCG64 generator (``numpy.random.default_rng(seed)``) in the
order written in each recipe. Rounding is half-up: ``floor(x + 0.5)``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

PC_09 = 3865470566   # floor(0.9 * 2^32): crossover threshold on hi32 of a draw
PM_01 = 429496729    # floor(0.1 * 2^32): mutation threshold


@dataclass
class Instance:
    """One event's EDFFS instance (field meanings follow the C header)."""
    n_jobs: int
    n_stages: int
    o_max: int
    n_machines: np.ndarray   # int32 [g]
    proc: np.ndarray         # int32 [n_jobs, g, o_max]
    power: np.ndarray        # int32 [n_jobs, g, o_max]
    release: np.ndarray      # int32 [n_jobs]
    due: np.ndarray          # int32 [n_jobs]
    q_max: int
    wt: int
    rs: int
    first_stage: np.ndarray  # int32 [n_jobs]
    ready: np.ndarray        # int32 [n_jobs]
    machine_free: np.ndarray  # int32 [g, o_max]
    running: np.ndarray      # int32 [n_running, 2] (end, q)
    frozen_tardiness: int
    frozen_cmax: int
    active: np.ndarray       # int32 [n_active]
    decode_rules: int = 0    # job-vector decode variants: 1 FIFO stage order, 2 power-aware ECT
    fixed: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), np.int32))
    # int32 [n_fixed, 3] (start, end, q): planned ops kept in place (static approach)

    @property
    def n_active(self) -> int:
        return int(len(self.active))

    @classmethod
    def from_fields(cls, d: dict) -> "Instance":
        return cls(**{k: d[k] for k in cls.__dataclass_fields__ if k in d})


@dataclass
class Arrival:
    """New jobs arriving at rescheduling point rs."""
    rs: int
    proc: np.ndarray     # int32 [n_new, g, o_max]
    power: np.ndarray    # int32 [n_new, g, o_max]
    release: np.ndarray  # int32 [n_new]
    due: np.ndarray      # int32 [n_new]


@dataclass
class GaParams:
    islands: int
    rows: int
    cols: int
    pc: int = PC_09
    pm: int = PM_01
    mig_interval: int = 10
    mig_k: int = 1
    encoding: int = 0   # 0: one priority per job; 1: X/Y matrices over the operations

    @property
    def pop(self) -> int:
        return self.islands * self.rows * self.cols


@dataclass
class Workload:
    name: str
    initial: Instance
    arrivals: List[Arrival]
    ga: GaParams
    generations: int
    seed: int
    shop: int = 0
    notes: dict = field(default_factory=dict)

    @property
    def decodes_per_run(self) -> int:
        """Decodes in one full run: (generation 0 + generations) per slot per event."""
        return (1 + len(self.arrivals)) * (1 + self.generations) * self.ga.pop


def round_half_up(x):
    return np.floor(np.asarray(x, dtype=np.float64) + 0.5).astype(np.int64)


def initial_instance(proc, power, release, due, n_machines, q_max, wt) -> Instance:
    """The state at time 0: nothing scheduled, every job active from stage 0."""
    proc = np.ascontiguousarray(proc, dtype=np.int32)
    n, g, om = proc.shape
    return Instance(
        n_jobs=n, n_stages=g, o_max=om,
        n_machines=np.ascontiguousarray(n_machines, dtype=np.int32),
        proc=proc, power=np.ascontiguousarray(power, dtype=np.int32),
        release=np.ascontiguousarray(release, dtype=np.int32),
        due=np.ascontiguousarray(due, dtype=np.int32),
        q_max=int(q_max), wt=int(wt), rs=0,
        first_stage=np.zeros(n, np.int32),
        ready=np.ascontiguousarray(release, dtype=np.int32).copy(),
        machine_free=np.zeros((g, om), np.int32),
        running=np.zeros((0, 2), np.int32),
        frozen_tardiness=0, frozen_cmax=0,
        active=np.arange(n, dtype=np.int32),
    )


def peak_limit(machine_power, n_machines, percent):
    """Q_max = max(floor(percent * sum_s max_m Q_sm / 100), max Q_sm).

    The second term keeps every single op placeable (no op may need more than
    the peak on its own)."""
    g = len(n_machines)
    stage_max = [int(machine_power[s, :n_machines[s]].max()) for s in range(g)]
    return max((percent * sum(stage_max)) // 100, max(stage_max))


def mean_proc(proc, n_machines):
    """P-bar_j = sum_s mean_m P_jsm (the paper's Table 5 definition)."""
    g = len(n_machines)
    return np.array([sum(proc[j, s, :n_machines[s]].mean() for s in range(g))
                     for j in range(proc.shape[0])], dtype=np.float64)


def _broadcast_power(machine_power, n_jobs):
    return np.ascontiguousarray(np.broadcast_to(machine_power[None], (n_jobs,) + machine_power.shape),
                                dtype=np.int32)


def _poisson_times(rng, n_events, lb0):
    """Arrival times: floored exponential gaps of mean lb0/(n_events+1), each >= 1."""
    t = 0
    out = []
    mean = lb0 / (n_events + 1)
    for _ in range(n_events):
        t += max(1, int(math.floor(rng.exponential(mean))))
        out.append(t)
    return out


def makespan_lower_bound(proc, machine_power, n_machines, q_max):
    """LB0 = max(max_s ceil(sum_j min_m P_jsm / o_s), ceil(sum_js min_m P_jsm Q_sm / Q_max))."""
    n, g, _ = proc.shape
    per_stage = []
    energy = 0
    for s in range(g):
        o = int(n_machines[s])
        per_stage.append(math.ceil(int(proc[:, s, :o].min(axis=1).sum()) / o))
        energy += int((proc[:, s, :o] * machine_power[s, :o][None]).min(axis=1).sum())
    return max(max(per_stage), math.ceil(energy / q_max))


def config1(seed: int = 0) -> Workload:
    """Tiny: 10 jobs, 2 stages, 2 identical machines; P ~ U{1..20}; Q_sm ~ U{1..10};
    peak 60%; R = 0, D = round(U[1.2,2.0] * P-bar); one event at t=15 adding 3 jobs;
    WT = 10; 64 individuals in one 8x8 island; 50 generations per event."""
    rng = np.random.default_rng(seed)
    n0, g, o = 10, 2, 2
    p_js = rng.integers(1, 21, size=(n0, g))
    proc = np.repeat(p_js[:, :, None], o, axis=2)
    qsm = rng.integers(1, 11, size=(g, o))
    nm = np.full(g, o, np.int32)
    q_max = peak_limit(qsm, nm, 60)
    slack = rng.uniform(1.2, 2.0, size=n0)
    due = round_half_up(slack * mean_proc(proc, nm))
    inst = initial_instance(proc, _broadcast_power(qsm, n0), np.zeros(n0), due, nm, q_max, 10)
    n_new, t = 3, 15
    p_new = np.repeat(rng.integers(1, 21, size=(n_new, g))[:, :, None], o, axis=2)
    slack = rng.uniform(1.2, 2.0, size=n_new)
    arr = Arrival(rs=t, proc=p_new.astype(np.int32), power=_broadcast_power(qsm, n_new),
                  release=np.full(n_new, t, np.int32),
                  due=(t + round_half_up(slack * mean_proc(p_new, nm))).astype(np.int32))
    return Workload("tiny-10x2x2", inst, [arr], GaParams(1, 8, 8, mig_k=1), 50, seed)


def _unrelated(rng, n, speed):
    base = rng.integers(5, 51, size=(n, speed.shape[0]))
    return np.maximum(1, round_half_up(base[:, :, None] * speed[None])).astype(np.int32)


def table5_instance(seed: int, n_jobs: int = 10, n_stages: int = 3, machines: int = 2,
                    q_max: int = 4) -> Instance:
    """An event-0 instance shaped like the paper's small test (Section 5, Table 5):
    P_sm ~ U{1..5} the same for every job, Q = 1, R_j ~ U[0, P-bar), D_j = R_j +
    P-bar * (1 + sigma) with sigma ~ U[0, 2] and P-bar = sum_s mean_m P_sm, WT = 100;
    10 jobs, 3 stages of 2 machines and a power peak of 4 as in the paper's tests 1-3.
    Times are integers: R and D are floored / rounded."""
    rng = np.random.default_rng(seed)
    p_sm = rng.integers(1, 6, size=(n_stages, machines))
    proc = np.repeat(p_sm[None], n_jobs, axis=0).astype(np.int32)
    p_bar = float(p_sm.mean(axis=1).sum())
    release = np.floor(rng.uniform(0, p_bar, size=n_jobs)).astype(np.int32)
    sigma = rng.uniform(0, 2, size=n_jobs)
    due = (release + round_half_up(p_bar * (1 + sigma))).astype(np.int32)
    nm = np.full(n_stages, machines, np.int32)
    power = np.ones((n_jobs, n_stages, machines), np.int32)
    return initial_instance(proc, power, release, due, nm, q_max, 100)


def table5_arrival(seed: int, inst: Instance, rs: int, n_new: int) -> Arrival:
    """New jobs for a Table 5-shaped instance: the instance's stage times (the same
    for every job) and unit power, release RS, D = RS + P-bar * (1 + sigma) with
    sigma ~ U[0, 2], rounded."""
    rng = np.random.default_rng(seed)
    g, om = int(inst.n_stages), int(inst.o_max)
    p_sm = np.asarray(inst.proc)[0]
    proc = np.repeat(p_sm[None], n_new, axis=0).astype(np.int32)
    p_bar = float(sum(p_sm[s, :int(inst.n_machines[s])].mean() for s in range(g)))
    sigma = rng.uniform(0, 2, size=n_new)
    due = (rs + round_half_up(p_bar * (1 + sigma))).astype(np.int32)
    return Arrival(int(rs), proc, np.ones((n_new, g, om), np.int32), np.full(n_new, rs, np.int32),
                   due)


TABLE5_GA = GaParams(64, 8, 8)   # 64 x 64 = 4096 individuals in 8 x 8 islands (Section 5.1)


def config2(seed: int = 0, generations: int = 500) -> Workload:
    """Paper-shaped: 50 jobs, 5 stages, 3 unrelated machines, P = max(1, round(base*speed)),
    base ~ U{5..50}, speed_sm ~ U[0.8,1.5]; Q_sm ~ U{2..15}; peak 55%; R = 0;
    5 Poisson arrival events of U{5..10} jobs (due slack U[1.2,2.0]);
    population 4096 = 32 islands x (8x16), 2 best migrate every 10 generations."""
    rng = np.random.default_rng(seed)
    n0, g, o, n_events = 50, 5, 3, 5
    speed = rng.uniform(0.8, 1.5, size=(g, o))
    proc = _unrelated(rng, n0, speed)
    qsm = rng.integers(2, 16, size=(g, o))
    nm = np.full(g, o, np.int32)
    q_max = peak_limit(qsm, nm, 55)
    slack = rng.uniform(1.2, 2.0, size=n0)
    due = round_half_up(slack * mean_proc(proc, nm))
    inst = initial_instance(proc, _broadcast_power(qsm, n0), np.zeros(n0), due, nm, q_max, 10)
    times = _poisson_times(rng, n_events, makespan_lower_bound(proc, qsm, nm, q_max))
    arrivals = []
    for t in times:
        k = int(rng.integers(5, 11))
        p_new = _unrelated(rng, k, speed)
        sl = rng.uniform(1.2, 2.0, size=k)
        arrivals.append(Arrival(t, p_new, _broadcast_power(qsm, k), np.full(k, t, np.int32),
                                (t + round_half_up(sl * mean_proc(p_new, nm))).astype(np.int32)))
    return Workload("paper-50x5x3", inst, arrivals, GaParams(32, 8, 16, mig_k=2), generations, seed)


def config3(seed: int = 0, generations: int = 200) -> Workload:
    """Large: 200 jobs, 10 stages, o_s ~ U{4..6} unrelated machines, P ~ U{1..100} i.i.d.,
    Q_sm ~ U{1..20}, peak 50%; 10 events of U{10..30} jobs; 512 islands x (8x16)."""
    rng = np.random.default_rng(seed)
    n0, g, om, n_events = 200, 10, 6, 10
    nm = rng.integers(4, 7, size=g).astype(np.int32)
    proc = rng.integers(1, 101, size=(n0, g, om)).astype(np.int32)
    qsm = rng.integers(1, 21, size=(g, om))
    q_max = peak_limit(qsm, nm, 50)
    slack = rng.uniform(1.2, 2.0, size=n0)
    due = round_half_up(slack * mean_proc(proc, nm))
    inst = initial_instance(proc, _broadcast_power(qsm, n0), np.zeros(n0), due, nm, q_max, 10)
    times = _poisson_times(rng, n_events, makespan_lower_bound(proc, qsm, nm, q_max))
    arrivals = []
    for t in times:
        k = int(rng.integers(10, 31))
        p_new = rng.integers(1, 101, size=(k, g, om)).astype(np.int32)
        sl = rng.uniform(1.2, 2.0, size=k)
        arrivals.append(Arrival(t, p_new, _broadcast_power(qsm, k), np.full(k, t, np.int32),
                                (t + round_half_up(sl * mean_proc(p_new, nm))).astype(np.int32)))
    return Workload("large-200x10x4-6", inst, arrivals, GaParams(512, 8, 16, mig_k=2), generations,
                    seed)


def random_instance(seed: int, n_jobs: int, n_stages: int, machines, p_max: int = 20,
                    q_range=(1, 10), percent: int = 60, release_max: int = 0,
                    wt: int = 10) -> Instance:
    """A small random event-0 instance for tests. `machines` is an int (all stages)
    or a list of per-stage machine counts."""
    rng = np.random.default_rng(seed)
    nm = np.array([machines] * n_stages if np.isscalar(machines) else machines, np.int32)
    om = int(nm.max())
    proc = rng.integers(1, p_max + 1, size=(n_jobs, n_stages, om)).astype(np.int32)
    qsm = rng.integers(q_range[0], q_range[1] + 1, size=(n_stages, om))
    q_max = peak_limit(qsm, nm, percent)
    release = rng.integers(0, release_max + 1, size=n_jobs) if release_max else np.zeros(n_jobs)
    slack = rng.uniform(1.2, 2.0, size=n_jobs)
    due = release + round_half_up(slack * mean_proc(proc, nm))
    return initial_instance(proc, _broadcast_power(qsm, n_jobs), release, due, nm, q_max, wt)


def random_arrival(seed: int, inst: Instance, rs: int, n_new: int, p_max: int = 20) -> Arrival:
    rng = np.random.default_rng(seed)
    g, om = inst.n_stages, inst.o_max
    proc = rng.integers(1, p_max + 1, size=(n_new, g, om)).astype(np.int32)
    power = np.ascontiguousarray(np.broadcast_to(inst.power[0][None], (n_new, g, om))
                                 if inst.n_jobs else np.ones((n_new, g, om)), dtype=np.int32)
    slack = rng.uniform(1.2, 2.0, size=n_new)
    due = rs + round_half_up(slack * mean_proc(proc, inst.n_machines))
    return Arrival(rs, proc, power, np.full(n_new, rs, np.int32), due.astype(np.int32))


def random_population(seed: int, pop: int, n: int) -> np.ndarray:
    """pop random permutations of 1..n, int32 [pop, n]."""
    rng = np.random.default_rng(seed)
    base = np.tile(np.arange(1, n + 1, dtype=np.int32), (pop, 1))
    return np.ascontiguousarray(rng.permuted(base, axis=1), dtype=np.int32)



def random_xy_population(seed: int, pop: int, inst) -> np.ndarray:
    """Seeded X/Y chromosomes [pop, 2R] for `inst`: R = unfrozen ops, row-major over
    the active jobs and their stages from first_stage; a uniform machine of the
    op's stage, then a uniform permutation of 1..R."""
    rng = np.random.default_rng(seed)
    stages = [s for j in inst.active for s in range(int(inst.first_stage[j]), int(inst.n_stages))]
    o = np.asarray(inst.n_machines)[np.asarray(stages, dtype=np.int64)] if stages else np.zeros(0, int)
    R = len(stages)
    out = np.empty((pop, 2 * R), np.int32)
    for i in range(pop):
        out[i, :R] = (rng.random(R) * o).astype(np.int32)
        out[i, R:] = rng.permutation(R) + 1
    return out

def shop_instance(rng, n_jobs, n_stages, machines, wt=10, percent=55):
    """One shop drawn like the paper-shaped recipe: P = max(1, round(U{5..50} x U[0.8,1.5])),
    Q_sm ~ U{2..15}, peak `percent`, R = 0, D = round(U[1.2,2.0] x P-bar)."""
    nm = np.asarray(machines, np.int32)
    om = int(nm.max())
    speed = rng.uniform(0.8, 1.5, size=(n_stages, om))
    proc = _unrelated(rng, n_jobs, speed)
    qsm = rng.integers(2, 16, size=(n_stages, om))
    q_max = peak_limit(qsm, nm, percent)
    slack = rng.uniform(1.2, 2.0, size=n_jobs)
    due = round_half_up(slack * mean_proc(proc, nm))
    return initial_instance(proc, _broadcast_power(qsm, n_jobs), np.zeros(n_jobs), due, nm,
                            q_max, wt)


def shops(seed: int = 0, n_shops: int = 512, jobs=(20, 200), stages=(3, 10), machines=(2, 6),
          o_max: int = 6):
    """Independent shops of uneven size: jobs ~ U{20..200}, stages ~ U{3..10}, machines per
    stage ~ U{2..6}, otherwise the paper-shaped distributions. Every instance is padded to
    o_max machine columns so that shops can share a batch."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n_shops):
        n = int(rng.integers(jobs[0], jobs[1] + 1))
        g = int(rng.integers(stages[0], stages[1] + 1))
        nm = rng.integers(machines[0], machines[1] + 1, size=g)
        inst = shop_instance(rng, n, g, nm)
        pad = o_max - inst.o_max
        if pad > 0:
            inst.proc = np.pad(inst.proc, ((0, 0), (0, 0), (0, pad)), constant_values=1)
            inst.power = np.pad(inst.power, ((0, 0), (0, 0), (0, pad)), constant_values=1)
            inst.machine_free = np.pad(inst.machine_free, ((0, 0), (0, pad)))
            inst.o_max = o_max
        out.append(inst)
    return out


def shop_arrivals(seed: int, index: int, inst: Instance, n_events: int) -> List[Arrival]:
    """Arrival events of one shop: Poisson times over the shop's LB0 like the
    paper-shaped recipe, U{5..10} new jobs each with fresh unrelated-machine
    times, the shop's machine powers and due slack U[1.2, 2.0]."""
    rng = np.random.default_rng([seed, index])
    g, om, nm = int(inst.n_stages), int(inst.o_max), inst.n_machines
    qsm = np.asarray(inst.power[0]) if inst.n_jobs else np.ones((g, om), np.int32)
    times = _poisson_times(rng, n_events, makespan_lower_bound(inst.proc, qsm, nm, inst.q_max))
    out = []
    for t in times:
        k = int(rng.integers(5, 11))
        speed = rng.uniform(0.8, 1.5, size=(g, om))
        p_new = _unrelated(rng, k, speed)
        sl = rng.uniform(1.2, 2.0, size=k)
        out.append(Arrival(t, p_new, _broadcast_power(qsm, k), np.full(k, t, np.int32),
                           (t + round_half_up(sl * mean_proc(p_new, nm))).astype(np.int32)))
    return out


SERVING_GA = GaParams(8, 8, 16, mig_k=2)   # 1024 individuals per request

SURROGATE_HIDDEN = 256


def surrogate_init(seed: int, hidden: int = SURROGATE_HIDDEN) -> np.ndarray:
    """Initial surrogate parameters, float32, flat layout [W1 (4 x H), b1 (H),
    W2 (H x H), b2 (H), w3 (H), b3]: weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)),
    biases 0 (the targets are standardised)."""
    rng = np.random.default_rng([seed, 0x5047])
    h = hidden
    parts = [rng.uniform(-0.5, 0.5, size=4 * h), np.zeros(h),
             rng.uniform(-1, 1, size=h * h) / np.sqrt(h), np.zeros(h),
             rng.uniform(-1, 1, size=h) / np.sqrt(h), np.array([0.0])]
    return np.concatenate(parts).astype(np.float32)


CONFIGS = {1: config1, 2: config2, 3: config3}
