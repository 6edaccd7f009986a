"""The measured configurations at their full shapes, against the oracle.

Large-200x10x4-6 (65 536 individuals) at a rescheduled event and deep into an
event, the serving shape (512 uneven shops x 1024 individuals x 100
generations), and the paper-shaped event loop at its full 500 generations per
event. Where the oracle cannot run the whole population it runs the sampled
islands and every island they depend on through migration.
"""
import numpy as np
import pytest

import oracle
from oracle_helpers import oracle_islands, rescheduled_instance
from paper_1903_10741_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ffs():
    import torch
    from paper_1903_10741_amd import ffsga
    assert torch.cuda.is_available()
    return torch, ffsga


def _say(*a):
    print("[case]", *a, flush=True)


def _state(v):
    return {k: t.cpu().numpy() for k, t in v.items() if k != "work"}


def _same_islands(got, want, islands, K, what):
    for I in islands:
        sl = slice(I * K, (I + 1) * K)
        assert (got["prio"][sl] == want["prio"][sl]).all(), (what, I)
        assert (got["obj"][sl] == want["obj"][sl]).all(), (what, I)
        assert (got["elite"][I] == want["elite"][I]).all(), (what, I)
        assert got["elite_obj"][I] == want["elite_obj"][I], (what, I)


def test_large_rescheduled_event_sampled_islands():
    """Large-200x10x4-6 after two arrivals (rescheduled on oracle-decoded plans):
    more than 200 active jobs, running ops at RS, a horizon bound far past the
    on-chip slots; 20 generations (two of them migrating) with the on-chip
    profile sized by FFS_LDS_AUTO; sampled islands at generations 10 and 20."""
    torch, ffsga = _ffs()
    wl = W.config3(0)
    inst = rescheduled_instance(wl, k_events=2, seed=5)
    assert inst.n_active >= 200 and len(inst.running) > 0 and inst.rs > 0
    _say("large, event 2, n_active", inst.n_active, "rs", inst.rs)
    d = ffsga.DeviceInstance.from_host(inst)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga, lds_slots=ffsga.FFS_LDS_AUTO), wl.seed, wl.shop, 2)
    assert d.horizon > int(ga.ga.lds_slots)
    islands = [0, 300, 511]
    want = oracle_islands(inst, wl.ga, wl.seed, wl.shop, 2, islands, 20, checkpoints=(10,))
    K = wl.ga.rows * wl.ga.cols
    for G in (10, 20):
        ga.step(G - ga.generation)
        _same_islands(_state(ga.view()), want[G], islands, K, f"gen {G}")
    ga.status()


def test_large_event0_generation_200():
    """Large-200x10x4-6, event 0, the whole event (200 generations, 20 of them
    migrating): islands 0-2, which depend on islands 492-511 through the ring,
    checked at generations 100 and 200."""
    torch, ffsga = _ffs()
    wl = W.config3(0)
    _say("large, event 0, 200 generations, islands 0-2")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga, lds_slots=ffsga.FFS_LDS_AUTO), wl.seed, wl.shop, 0)
    islands = [0, 1, 2]
    want = oracle_islands(wl.initial, wl.ga, wl.seed, wl.shop, 0, islands, 200,
                          checkpoints=(100,))
    K = wl.ga.rows * wl.ga.cols
    for G in (100, 200):
        ga.step(G - ga.generation)
        _same_islands(_state(ga.view()), want[G], islands, K, f"gen {G}")
    ga.status()


def test_serving_shape_512_shops_100_generations():
    """The serving shape in one batch: 512 uneven shops (jobs 20-200, stages
    3-10, machines 2-6), 1024 individuals each, 100 generations, in the launch
    shape the benchmark uses (one wave per child, three profile classes, graph
    replay). The largest and the smallest shop and two seeded random ones
    against the oracle's own 100-generation runs."""
    torch, ffsga = _ffs()
    shops = W.shops(0, 512)
    _say("serving shape: 512 shops x 1024 x 100 generations")
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cfg = ffsga.BatchConfig(n_slots=512, max_jobs=max(s.n_jobs for s in shops),
                            max_genes=max(s.n_active for s in shops),
                            max_stages=max(s.n_stages for s in shops), o_max=6,
                            max_horizon=max(oracle.horizon_bound(s) for s in shops),
                            ga=ffsga.GaConfig.of(W.SERVING_GA, lds_slots=8192),
                            schedule=ffsga.FFS_SCHEDULE_CHROMOSOME, blocks=8 * n_cu,
                            use_graph=True, profile_classes=3)
    b = ffsga.Batch(cfg)
    for k, s in enumerate(shops):
        b.set(k, ffsga.DeviceInstance.from_host(s), 7, k, 0)
    b.step(100)
    b.status()
    size = [s.n_active * s.n_stages for s in shops]
    rng = np.random.default_rng(11)
    check = [int(np.argmax(size)), int(np.argmin(size))]
    check += [int(x) for x in rng.choice([k for k in range(512) if k not in check], 2,
                                         replace=False)]
    for k in check:
        _say("shop", k, "jobs", shops[k].n_active, "stages", shops[k].n_stages)
        want = oracle.ga_run(shops[k], W.SERVING_GA, 7, k, 0, 100, n_threads=8)
        got = _state(b.view(k))
        for key in ("prio", "obj", "elite", "elite_obj"):
            assert (got[key] == np.asarray(want[key])).all(), (k, key)


def test_paper_event_loop_full_500_generations():
    """Paper-50x5x3's whole run at 500 generations per event: every event's best
    objective and plan, and every rescheduled instance, against the oracle's run."""
    torch, ffsga = _ffs()
    from paper_1903_10741_amd.run import run_workload
    wl = W.config2(0)
    _say("paper-shaped event loop, 500 generations per event")
    got = run_workload(wl, keep_instances=True)
    want = oracle.run_events(wl.initial, wl.arrivals, wl.ga, wl.generations, wl.seed, wl.shop,
                             n_threads=8)
    assert len(got.events) == len(want) == 1 + len(wl.arrivals)
    for e, (ge, we) in enumerate(zip(got.events, want)):
        assert ge.best_obj == we["best_obj"], e
        assert (ge.best_prio.cpu().numpy() == we["best_prio"]).all(), e
        gi = ge.instance.to_host()
        wi = we["instance"]
        for k in ("first_stage", "ready", "active", "machine_free", "running"):
            assert np.array_equal(np.asarray(gi[k]).reshape(-1),
                                  np.asarray(getattr(wi, k)).reshape(-1)), (e, k)
    n = got.plan_start.shape[0]
    assert (got.plan_start.cpu().numpy() == want[-1]["plan_start"][:n]).all()
    assert (got.plan_mach.cpu().numpy() == want[-1]["plan_mach"][:n]).all()
