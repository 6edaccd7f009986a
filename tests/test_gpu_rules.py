"""GPU decode variants (FFS_RULE_FIFO, FFS_RULE_POWER_ECT) against the oracle, bit
for bit: ffs_decode on and off chip, the GA, the event loop, the Table 5 preset."""
import dataclasses

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


def _later_event(wl, seed):
    inst = wl.initial
    st, mc = oracle.decode(inst, W.random_population(seed, 1, inst.n_active)[0],
                           want_schedule=True)[1:3]
    arr = wl.arrivals[0]
    return W.Instance.from_fields(oracle.reschedule(inst, st, mc, arr.rs, arr.proc, arr.power,
                                                    arr.release, arr.due))


@pytest.mark.parametrize("rules", [1, 2, 3])
def test_decode_rules_match_oracle(rules):
    torch, ffsga = _ffs()
    for cfg, seed in ((1, 0), (2, 3)):
        wl = W.CONFIGS[cfg](seed)
        for name, base in (("event 0", wl.initial), ("event 1", _later_event(wl, seed))):
            inst = dataclasses.replace(base, decode_rules=rules)
            d = ffsga.DeviceInstance.from_host(inst)
            prio = W.random_population(11, 120, inst.n_active)
            want, wwork = oracle.decode_pop(inst, prio, n_threads=8, want_work=True)
            for lds in (0, 64):
                _say("rules", rules, "cfg", cfg, name, "lds_slots", lds)
                got = ffsga.ffs_decode(d, torch.from_numpy(prio).cuda(), lds_slots=lds,
                                       want_schedule=True, want_work=True)
                assert (got["obj"].cpu().numpy() == want).all()
                assert (got["work"].cpu().numpy() == wwork).all()
                st, mc = got["start"].cpu().numpy(), got["mach"].cpu().numpy()
                for i in (0, 59, 119):
                    _, s2, m2, _ = oracle.decode(inst, prio[i], want_schedule=True)
                    assert (st[i] == s2).all() and (mc[i] == m2).all()


@pytest.mark.parametrize("n_jobs", [60, 100, 150])
def test_fifo_order_for_each_job_count_layout(n_jobs):
    """FIFO stage order with the keys in one register (up to 64 jobs), in two
    (65-128) and in LDS (more), at event 0 and after an arrival, against the oracle."""
    torch, ffsga = _ffs()
    base = W.random_instance(23, n_jobs=n_jobs, n_stages=3, machines=[2, 3, 2], p_max=30, percent=55)
    st, mc = oracle.decode(base, W.random_population(1, 1, base.n_active)[0], want_schedule=True)[1:3]
    arr = W.random_arrival(6, base, 40, 9, p_max=30)
    later = W.Instance.from_fields(oracle.reschedule(base, st, mc, arr.rs, arr.proc, arr.power,
                                                     arr.release, arr.due))
    for name, b in (("event 0", base), ("event 1", later)):
        inst = dataclasses.replace(b, decode_rules=1)
        _say("FIFO", n_jobs, "jobs", name, "n_active", inst.n_active)
        d = ffsga.DeviceInstance.from_host(inst)
        prio = W.random_population(5, 64, inst.n_active)
        want, wwork = oracle.decode_pop(inst, prio, n_threads=8, want_work=True)
        got = ffsga.ffs_decode(d, torch.from_numpy(prio).cuda(), want_schedule=True, want_work=True)
        assert (got["obj"].cpu().numpy() == want).all()
        assert (got["work"].cpu().numpy() == wwork).all()
        st2, mc2 = got["start"].cpu().numpy(), got["mach"].cpu().numpy()
        for i in (0, 63):
            _, s3, m3, _ = oracle.decode(inst, prio[i], want_schedule=True)
            assert (st2[i] == s3).all() and (mc2[i] == m3).all()


def _state(ga):
    v = ga.view()
    return {k: t.cpu().numpy() for k, t in v.items() if k != "work"}


def _same(a, b, what):
    for k in ("prio", "obj", "elite", "elite_obj"):
        assert (np.asarray(a[k]) == np.asarray(b[k])).all(), (what, k)


def test_ga_with_rules_and_table5_preset():
    torch, ffsga = _ffs()
    wl = W.config1(2)
    cases = [("config 1", wl.initial, wl.ga, 30), ("table 5", W.table5_instance(1),
                                                    W.GaParams(2, 8, 8, mig_k=1), 30)]
    for name, base, gp, gens in cases:
        for rules in (0, 3):
            inst = dataclasses.replace(base, decode_rules=rules)
            _say("GA", name, "rules", rules)
            d = ffsga.DeviceInstance.from_host(inst)
            ga = ffsga.GA(d, ffsga.GaConfig.of(gp), 4, 1, 0)
            ga.step(gens)
            ga.status()
            _same(_state(ga), oracle.ga_run(inst, gp, 4, 1, 0, gens, n_threads=8), (name, rules))


def test_event_loop_with_rules():
    """The rules travel with the instance through every rescheduling."""
    torch, ffsga = _ffs()
    from paper_1903_10741_amd.run import run_workload
    wl = W.config1(0)
    wl.initial = dataclasses.replace(wl.initial, decode_rules=3)
    _say("event loop, rules 3")
    got = run_workload(wl, generations=20, keep_instances=True)
    want = oracle.run_events(wl.initial, wl.arrivals, wl.ga, 20, wl.seed, wl.shop, n_threads=8)
    for e, (ge, we) in enumerate(zip(got.events, want)):
        assert ge.best_obj == we["best_obj"], e
        assert int(ge.instance.s.decode_rules) == 3
    n = got.plan_start.shape[0]
    assert (got.plan_start.cpu().numpy() == want[-1]["plan_start"][:n]).all()
