"""Rescheduling on the GPU and the whole predictive-reactive event loop, against the oracle."""
import numpy as np
import pytest

import oracle
from paper_1903_10741_amd import workloads as W
from tests.golden_io import ints, read

pytestmark = pytest.mark.gpu


def _ffs():
    import torch
    from paper_1903_10741_amd import ffsga
    assert torch.cuda.is_available()
    return torch, ffsga


def _say(*a):
    print("[case]", *a, flush=True)


def _check_instance(got, want):
    for k in ("n_jobs", "rs", "frozen_tardiness", "frozen_cmax"):
        assert got[k] == int(want[k]), k
    for k in ("proc", "power", "release", "due", "first_stage", "ready", "machine_free", "running",
              "active"):
        assert np.array_equal(np.asarray(got[k]), np.asarray(want[k])), k
    assert got["horizon"] == oracle.horizon_bound(oracle._Fields(want))


def test_reschedule_paper_example():
    """The worked example of Section 4.3: Table 4's plan frozen at RS = 7."""
    torch, ffsga = _ffs()
    _say("reschedule Table 4")
    f = read("table4_example.txt")
    p_stage = ints(f["proc_per_stage"][0])
    release = ints(f["release"][0])
    proc = np.array([[[p] * 2 for p in p_stage] for _ in range(8)], np.int32)
    power = np.ones((8, 3, 2), np.int32)
    due = np.full(8, 10**6, np.int32)
    ps = np.zeros((6, 3), np.int32)
    pm = np.zeros((6, 3), np.int32)
    for row in f["plan_start"]:
        j, *s = ints(row)
        ps[j] = s
    for row in f["plan_mach"]:
        j, *m = ints(row)
        pm[j] = m
    inst = W.initial_instance(proc[:6], power[:6], release[:6], due[:6], [2, 2, 2], 3, 100)
    arr = W.Arrival(700, proc[6:], power[6:], np.array(release[6:], np.int32), due[6:])
    d = ffsga.DeviceInstance.from_host(inst)
    nxt = ffsga.reschedule(d, torch.from_numpy(ps).cuda(), torch.from_numpy(pm).cuda(), arr)
    want = oracle.reschedule(inst, ps, pm, 700, arr.proc, arr.power, arr.release, arr.due)
    got = nxt.to_host()
    _check_instance(got, want)
    assert list(got["first_stage"]) == [3, 3, 1, 1, 2, 1, 0, 0]
    assert sorted(got["running"][:, 0].tolist()) == [742, 780, 791]


@pytest.mark.parametrize("cfg", [1, 2, 3])
def test_reschedule_random_plans(cfg):
    torch, ffsga = _ffs()
    wl = W.CONFIGS[cfg](4)
    _say("reschedule config", cfg)
    inst = wl.initial
    prio = W.random_population(cfg, 1, inst.n_active)[0]
    _, s, m, _ = oracle.decode(inst, prio, want_schedule=True)
    d = ffsga.DeviceInstance.from_host(inst)
    for a in wl.arrivals[:2]:
        want = oracle.reschedule(inst, s, m, a.rs, a.proc, a.power, a.release, a.due)
        nxt = ffsga.reschedule(d, torch.from_numpy(s).cuda(), torch.from_numpy(m).cuda(), a)
        _check_instance(nxt.to_host(), want)


def test_reschedule_rejects_bad_plan():
    torch, ffsga = _ffs()
    _say("reschedule invalid plan")
    inst = W.random_instance(0, n_jobs=3, n_stages=2, machines=2)
    _, s, m, _ = oracle.decode(inst, np.array([1, 2, 3]), want_schedule=True)
    s = s.copy()
    rs = int(s[:, 1].max())            # every stage-0 op started before rs
    s[0, 0] = rs + 5                   # ...except job 0's, which breaks the prefix rule
    s[0, 1] = 0
    d = ffsga.DeviceInstance.from_host(inst)
    arr = W.Arrival(rs, np.zeros((0, 2, 2), np.int32), np.zeros((0, 2, 2), np.int32),
                    np.zeros(0, np.int32), np.zeros(0, np.int32))
    with pytest.raises(ffsga.FfsError) as e:
        ffsga.reschedule(d, torch.from_numpy(s).cuda(), torch.from_numpy(m).cuda(), arr)
    assert e.value.code == ffsga.FFS_E_INVAL


@pytest.mark.parametrize("cfg,gens", [(1, 50), (2, 20)])
def test_event_loop_matches_oracle(cfg, gens):
    """Every event of the workload: GA, executed plan, freeze, reschedule."""
    torch, ffsga = _ffs()
    from paper_1903_10741_amd.run import run_workload
    wl = W.CONFIGS[cfg](0)
    _say("event loop config", cfg, "generations", gens)
    got = run_workload(wl, generations=gens, keep_instances=True)
    want = oracle.run_events(wl.initial, wl.arrivals, wl.ga, gens, wl.seed, wl.shop, n_threads=8)
    assert len(got.events) == len(want) == 1 + len(wl.arrivals)
    for e, (ge, we) in enumerate(zip(got.events, want)):
        assert ge.best_obj == we["best_obj"], e
        assert (ge.best_prio.cpu().numpy() == we["best_prio"]).all(), e
        gi = ge.instance.to_host()
        wi = we["instance"]
        for k in ("first_stage", "ready", "active", "machine_free"):
            assert np.array_equal(gi[k], np.asarray(getattr(wi, k))), (e, k)
    n = got.plan_start.shape[0]
    assert (got.plan_start.cpu().numpy() == want[-1]["plan_start"][:n]).all()
    assert (got.plan_mach.cpu().numpy() == want[-1]["plan_mach"][:n]).all()
