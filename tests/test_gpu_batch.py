"""Batched GA (ga_batch_* through the C ABI): every slot equals its instance run alone.

Slots hold instances of different sizes; each slot's population, objectives
and elites must equal the oracle's GA on that instance with the slot's own
(seed, shop, event), bit for bit, under both schedules, with and without a
captured graph, across slot swaps and off-chip profile redos.
"""
import numpy as np
import pytest

import oracle
from paper_1903_10741_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ffs():
    import torch
    from paper_1903_10741_amd import ffsga
    assert torch.cuda.is_available()
    return torch, ffsga


def _say(*a):
    print("[case]", *a, flush=True)


GA = W.GaParams(2, 4, 4, mig_interval=3, mig_k=2)


def _instances():
    out = []
    for k, (n, g, m) in enumerate(((9, 2, 2), (23, 4, [3, 1, 2, 4]), (14, 3, 3), (40, 5, [2, 4, 3, 2, 4]),
                                   (1, 2, 2), (31, 3, [4, 4, 2]))):
        inst = W.random_instance(100 + k, n_jobs=n, n_stages=g, machines=m, p_max=25, percent=50)
        pad = 4 - inst.o_max
        if pad:
            inst.proc = np.pad(inst.proc, ((0, 0), (0, 0), (0, pad)), constant_values=1)
            inst.power = np.pad(inst.power, ((0, 0), (0, 0), (0, pad)), constant_values=1)
            inst.machine_free = np.pad(inst.machine_free, ((0, 0), (0, pad)))
            inst.o_max = 4
        out.append(inst)
    return out


def _batch(ffsga, insts, schedule, use_graph, blocks=7, lds_slots=0, n_slots=None, classes=1):
    cfg = ffsga.BatchConfig(
        n_slots=n_slots or len(insts), max_jobs=max(i.n_jobs for i in insts),
        max_genes=max(i.n_active for i in insts), max_stages=max(i.n_stages for i in insts),
        o_max=4, max_horizon=max(oracle.horizon_bound(i) for i in insts),
        ga=ffsga.GaConfig.of(GA, lds_slots=lds_slots), schedule=schedule, blocks=blocks,
        use_graph=use_graph, profile_classes=classes)
    return ffsga.Batch(cfg)


def _state(b, slot):
    return {k: t.cpu().numpy() for k, t in b.view(slot).items() if k != "work"}


def _same(a, b, what):
    for k in ("prio", "obj", "elite", "elite_obj"):
        assert (np.asarray(a[k]) == np.asarray(b[k])).all(), (what, k)


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_slots_match_oracle(schedule, use_graph):
    torch, ffsga = _ffs()
    _say("batch schedule", schedule, "graph", use_graph)
    insts = _instances()
    b = _batch(ffsga, insts, schedule, use_graph)
    dev = [ffsga.DeviceInstance.from_host(i) for i in insts]
    for s, d in enumerate(dev):
        b.set(s, d, seed=40 + s, shop=s, event=s % 3)
    want = [oracle.ga_init(i, GA, 40 + s, s, s % 3) for s, i in enumerate(insts)]
    for s in range(len(insts)):
        _same(_state(b, s), want[s], f"slot {s} gen 0")
    for step in (1, 2, 4):     # generations 1, 2..3, 4..7 (3 and 6 migrate)
        b.step(step)
        for s, i in enumerate(insts):
            for k in range(b.generation(s) - step + 1, b.generation(s) + 1):
                want[s] = oracle.ga_generation(i, GA, 40 + s, s, s % 3, k, want[s])
            _same(_state(b, s), want[s], f"slot {s} gen {b.generation(s)}")
    b.status()
    for s, i in enumerate(insts):
        prio, obj = b.best(s)
        bp, bo = oracle.ga_best(want[s])
        assert int(obj.item()) == bo and (prio.cpu().numpy() == bp).all()


def test_batch_graph_replays_match_eager_with_work_between():
    """Replays of the captured generation, with eager work and synchronisation
    between them, equal the eager batch after every replay."""
    torch, ffsga = _ffs()
    _say("batch graph replays vs eager")
    insts = _instances()
    dev = [ffsga.DeviceInstance.from_host(i) for i in insts]
    g = _batch(ffsga, insts, 0, True)
    e = _batch(ffsga, insts, 0, False)
    for s, d in enumerate(dev):
        g.set(s, d, 7, s, 1)
        e.set(s, d, 7, s, 1)
    for r in range(4):
        g.step(1)
        e.step(1)
        x = torch.arange(1000, device="cuda").sum()       # eager work between replays
        torch.cuda.synchronize()
        assert int(x.item()) == 499500
        for s in range(len(insts)):
            _same(_state(g, s), _state(e, s), f"replay {r} slot {s}")


def test_batch_slot_swap_keeps_other_slots():
    torch, ffsga = _ffs()
    _say("batch slot swap")
    insts = _instances()
    dev = [ffsga.DeviceInstance.from_host(i) for i in insts]
    b = _batch(ffsga, insts, 0, True, n_slots=len(insts))
    for s in range(3):
        b.set(s, dev[s], 5, s, 0)
    want = {s: oracle.ga_init(insts[s], GA, 5, s, 0) for s in range(3)}
    b.step(2)
    for s in range(3):
        for k in (1, 2):
            want[s] = oracle.ga_generation(insts[s], GA, 5, s, 0, k, want[s])
    b.clear(1)
    b.set(1, dev[4], 9, 44, 2)       # a different, tiny instance in slot 1
    b.set(4, dev[3], 9, 45, 0)       # and a new slot
    want[1] = oracle.ga_init(insts[4], GA, 9, 44, 2)
    want[4] = oracle.ga_init(insts[3], GA, 9, 45, 0)
    b.step(3)
    for s, inst, seed, shop, ev in ((0, insts[0], 5, 0, 0), (2, insts[2], 5, 2, 0),
                                    (1, insts[4], 9, 44, 2), (4, insts[3], 9, 45, 0)):
        for k in range(b.generation(s) - 2, b.generation(s) + 1):
            want[s] = oracle.ga_generation(inst, GA, seed, shop, ev, k, want[s])
        _same(_state(b, s), want[s], f"slot {s}")
    b.status()


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_off_chip_redo(schedule):
    torch, ffsga = _ffs()
    _say("batch with lds_slots 64, schedule", schedule)
    insts = _instances()
    dev = [ffsga.DeviceInstance.from_host(i) for i in insts]
    b = _batch(ffsga, insts, schedule, False, lds_slots=64)
    for s, d in enumerate(dev):
        b.set(s, d, 3, s, 0)
    b.step(4)
    b.status()
    for s, i in enumerate(insts):
        _same(_state(b, s), oracle.ga_run(i, GA, 3, s, 0, 4), f"slot {s}")


@pytest.mark.parametrize("schedule,use_graph", [(0, True), (1, False)])
def test_batch_profile_classes(schedule, use_graph):
    """Profile size classes 64/128/256 slots: slots of different schedule lengths
    land in different class launches (and long ones still overflow off chip);
    every slot stays bit-exact."""
    torch, ffsga = _ffs()
    _say("batch with profile classes, schedule", schedule, "graph", use_graph)
    insts = _instances()
    dev = [ffsga.DeviceInstance.from_host(i) for i in insts]
    b = _batch(ffsga, insts, schedule, use_graph, lds_slots=256, classes=3)
    for s, d in enumerate(dev):
        b.set(s, d, 12, s, 1)
    b.step(5)
    b.status()
    for s, i in enumerate(insts):
        _same(_state(b, s), oracle.ga_run(i, GA, 12, s, 1, 5), f"slot {s}")


def test_batch_of_shops_sampled():
    """Forty uneven shops of the serving shape, population 1024 each, in the
    launch shape the benchmark uses: sampled slots against the oracle."""
    torch, ffsga = _ffs()
    _say("batch of 40 shops, pop 1024")
    shops = W.shops(3, 40)
    cfg = ffsga.BatchConfig(n_slots=40, max_jobs=200, max_genes=200, max_stages=10, o_max=6,
                            max_horizon=max(oracle.horizon_bound(s) for s in shops),
                            ga=ffsga.GaConfig.of(W.SERVING_GA, lds_slots=16384), use_graph=True,
                            profile_classes=3)
    b = ffsga.Batch(cfg)
    dev = [ffsga.DeviceInstance.from_host(s) for s in shops]
    for s, d in enumerate(dev):
        b.set(s, d, 11, s, 0)
    b.step(10)
    b.status()
    for s in (0, 17, 39):
        want = oracle.ga_run(shops[s], W.SERVING_GA, 11, s, 0, 10, n_threads=8)
        _same(_state(b, s), want, f"shop {s}")


@pytest.mark.parametrize("schedule", [0, 1])
def test_batch_large_instance_both_schedules(schedule):
    """large-200x10x4-6 (512 islands x 8x16 = 65536) in a one-slot batch, in the
    launch shapes its bench times: sampled islands after a migrating generation
    against the oracle's own run of them."""
    from oracle_helpers import oracle_islands
    torch, ffsga = _ffs()
    wl = W.config3(0)
    _say("large instance in a batch, schedule", schedule)
    d = ffsga.DeviceInstance.from_host(wl.initial)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cfg = ffsga.BatchConfig(n_slots=1, max_jobs=wl.initial.n_jobs, max_genes=wl.initial.n_active,
                            max_stages=wl.initial.n_stages, o_max=wl.initial.o_max,
                            max_horizon=d.horizon, ga=ffsga.GaConfig.of(wl.ga, lds_slots=8192),
                            schedule=schedule, blocks=(8 if schedule == 0 else 2) * n_cu,
                            use_graph=True)
    b = ffsga.Batch(cfg)
    b.set(0, d, wl.seed, wl.shop, 0)
    b.step(10)
    b.status()
    islands = [0, 255, 511]
    want = oracle_islands(wl.initial, wl.ga, wl.seed, wl.shop, 0, islands, 10)
    got = _state(b, 0)
    K = wl.ga.rows * wl.ga.cols
    for I in islands:
        sl = slice(I * K, (I + 1) * K)
        assert (got["prio"][sl] == want["prio"][sl]).all(), I
        assert (got["obj"][sl] == want["obj"][sl]).all(), I
        assert (got["elite"][I] == want["elite"][I]).all(), I
        assert got["elite_obj"][I] == want["elite_obj"][I], I
