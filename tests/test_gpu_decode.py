"""GPU decode (ffs_decode through the C ABI) against the CPU oracle, element by element.

Integer path: objectives, start times, machines and algorithmic work counts
must be identical (zero tolerance).
"""
import numpy as np
import pytest

import oracle
from oracle_helpers import rescheduled_instance
from paper_1903_10741_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ffs():
    import torch
    from paper_1903_10741_amd import ffsga
    assert torch.cuda.is_available()
    return torch, ffsga


def _say(*a):
    print("[case]", *a, flush=True)


def _event_instance(wl, k_events=1, seed=3):
    return rescheduled_instance(wl, k_events, seed)


def _compare(inst, pop, lds_slots=0, schedule=True):
    torch, ffsga = _ffs()
    d = ffsga.DeviceInstance.from_host(inst)
    got = ffsga.ffs_decode(d, torch.from_numpy(pop).cuda(), lds_slots=lds_slots,
                           want_schedule=schedule, want_work=True)
    obj = got["obj"].cpu().numpy()
    work = got["work"].cpu().numpy()
    for i, prio in enumerate(pop):
        o, s, m, w = oracle.decode(inst, prio, want_schedule=True)
        assert obj[i] == o, (i, obj[i], o)
        assert work[i] == w, (i, work[i], w)
        if schedule:
            gs = got["start"][i].cpu().numpy()
            gm = got["mach"][i].cpu().numpy()
            for j in inst.active:
                f = inst.first_stage[j]
                assert (gs[j, f:] == s[j, f:]).all() and (gm[j, f:] == m[j, f:]).all(), (i, j)
            frozen = np.ones_like(gs, bool)
            for j in inst.active:
                frozen[j, inst.first_stage[j]:] = False
            assert (gs[frozen] == -1).all()   # frozen entries are not written


@pytest.mark.parametrize("cfg,pop", [(1, 256), (2, 96), (3, 24)])
def test_decode_event0_configs(cfg, pop):
    _say("decode event 0, config", cfg, "pop", pop)
    inst = W.CONFIGS[cfg](0).initial
    _compare(inst, W.random_population(10 + cfg, pop, inst.n_active))


@pytest.mark.parametrize("cfg,k,pop", [(1, 1, 128), (2, 1, 64), (2, 3, 64), (3, 2, 12)])
def test_decode_rescheduled_configs(cfg, k, pop):
    _say("decode after", k, "arrivals, config", cfg)
    inst = _event_instance(W.CONFIGS[cfg](1), k_events=k)
    assert inst.rs > 0 and len(inst.running) > 0
    _compare(inst, W.random_population(20 + cfg, pop, inst.n_active))


@pytest.mark.parametrize("n", [1, 2, 3, 63, 64, 65, 130])
def test_decode_ragged_gene_counts(n):
    _say("decode ragged n =", n)
    inst = W.random_instance(n, n_jobs=n, n_stages=3, machines=[2, 3, 1], p_max=30, percent=50)
    _compare(inst, W.random_population(n, 16, n))


def test_decode_max_gene_count():
    """n_active = 4096, the largest the ABI takes: 16-bit op records hold ranks up to
    4095; the default 4096 on-chip slots overflow, so the decodes go off chip."""
    torch, ffsga = _ffs()
    _say("decode at n = 4096")
    inst = W.random_instance(7, n_jobs=4096, n_stages=2, machines=[3, 2], p_max=6, q_range=(1, 5),
                             percent=60)
    _compare(inst, W.random_population(7, 3, 4096), schedule=False)
    _compare(inst, W.random_population(8, 2, 4096), lds_slots=32768)
    big = W.random_instance(7, n_jobs=4097, n_stages=1, machines=2, p_max=3)
    with pytest.raises(ffsga.FfsError) as e:
        ffsga.DeviceInstance.from_host(big)
    assert e.value.code == ffsga.FFS_E_UNSUPPORTED


def test_decode_long_windows_span_several_chunks():
    _say("decode with p up to 200 (windows of 4 chunks)")
    inst = W.random_instance(5, n_jobs=20, n_stages=4, machines=[3, 5, 2, 4], p_max=200,
                             q_range=(3, 12), percent=45)
    _compare(inst, W.random_population(5, 32, 20))


def test_decode_work_long_horizon_many_delays():
    """Schedules of about 1.8 million slots (off chip) in which every op draws the
    whole peak, so each is pushed right past the ops placed before it on the
    other 15 machines of its stage: objectives, plans and work counts (about
    4e7 examined slots per decode) equal the oracle's."""
    _say("decode long horizon, every op pushed right")
    rng = np.random.default_rng(17)
    n, g, om = 300, 2, 16
    proc = rng.integers(2000, 4001, size=(n, g, om)).astype(np.int32)
    power = np.full((n, g, om), 7, np.int32)
    inst = W.initial_instance(proc, power, np.zeros(n, np.int32), np.full(n, 10**6, np.int32),
                              [om] * g, 7, 3)
    _compare(inst, W.random_population(19, 8, n))


def test_decode_sixteen_machines():
    _say("decode o_max = 16")
    inst = W.random_instance(6, n_jobs=30, n_stages=3, machines=[16, 9, 12], p_max=40, percent=30)
    _compare(inst, W.random_population(6, 32, 30))


@pytest.mark.parametrize("lds_slots", [64, 256, 1024])
def test_decode_overflow_tier(lds_slots):
    """Decodes whose schedule outgrows the on-chip profile are redone with the
    global-memory profile; results are identical."""
    _say("decode overflow tier, lds_slots", lds_slots)
    inst = _event_instance(W.config2(2), k_events=2)
    _compare(inst, W.random_population(7, 48, inst.n_active), lds_slots=lds_slots)


def test_decode_full_population_config2():
    """Full config-2 population (4096) in the launch shape the benchmark uses."""
    _say("decode config 2, pop 4096")
    torch, ffsga = _ffs()
    inst = W.config2(0).initial
    pop = W.random_population(99, 4096, inst.n_active)
    d = ffsga.DeviceInstance.from_host(inst)
    got = ffsga.ffs_decode(d, torch.from_numpy(pop).cuda()).cpu().numpy()
    want = oracle.decode_pop(inst, pop, n_threads=8)
    assert (got == want).all()


def test_decode_full_population_config3_sampled():
    """Config 3 at its full population (65536): a sample of outputs against the oracle."""
    _say("decode config 3, pop 65536, sampled")
    torch, ffsga = _ffs()
    inst = W.config3(0).initial
    pop = W.random_population(98, 65536, inst.n_active)
    d = ffsga.DeviceInstance.from_host(inst)
    got = ffsga.ffs_decode(d, torch.from_numpy(pop).cuda()).cpu().numpy()
    idx = np.random.default_rng(0).choice(65536, 512, replace=False)
    want = oracle.decode_pop(inst, pop[idx], n_threads=8)
    assert (got[idx] == want).all()
    assert (got > 0).all()


@pytest.mark.parametrize("rules", [0, 1])
def test_decode_late_first_stages_of_twenty(rules):
    """20 stages, rescheduled where some jobs have finished 15 or more stages: the
    16-bit job records hold a first stage only up to 15, so from stage 15 on such
    jobs are looked up; with the default rules and with the FIFO stage order (whose
    compaction tests the same records)."""
    _say("decode, 20 stages, late first stages, rules", rules)
    g, om = 20, 2
    inst = W.random_instance(17, n_jobs=40, n_stages=g, machines=om, p_max=10, percent=70)
    prio = W.random_population(18, 1, inst.n_active)[0]
    _, s, m, _ = oracle.decode(inst, prio, want_schedule=True)
    rs = int(np.median(s[:, 16])) + 1
    rng = np.random.default_rng(19)
    k = 6
    proc = rng.integers(1, 11, size=(k, g, om)).astype(np.int32)
    power = np.broadcast_to(np.asarray(inst.power)[:1], (k, g, om)).astype(np.int32)
    nxt = W.Instance.from_fields(oracle.reschedule(inst, s, m, rs, proc, power,
                                                   np.full(k, rs, np.int32),
                                                   np.full(k, rs + 200, np.int32)))
    nxt.decode_rules = rules
    firsts = np.asarray(nxt.first_stage)[np.asarray(nxt.active)]
    assert (firsts >= 15).any() and (firsts < 15).any(), firsts
    _compare(nxt, W.random_population(20 + rules, 48, nxt.n_active))


def test_decode_empty_active_set():
    _say("decode with no active job")
    torch, ffsga = _ffs()
    inst = W.random_instance(0, n_jobs=3, n_stages=2, machines=2)
    _, s, m, _ = oracle.decode(inst, np.array([1, 2, 3]), want_schedule=True)
    nxt = W.Instance.from_fields(oracle.reschedule(inst, s, m, int(s.max()) + 999,
                                                   np.zeros((0, 2, 2)), np.zeros((0, 2, 2)), [], []))
    d = ffsga.DeviceInstance.from_host(nxt)
    got = ffsga.ffs_decode(d, torch.zeros((4, 0), dtype=torch.int32).cuda()).cpu().numpy()
    assert (got == oracle.decode(nxt, np.zeros(0, np.int32))).all()


def test_decode_rejects_non_permutation():
    _say("decode invalid chromosome")
    torch, ffsga = _ffs()
    inst = W.random_instance(1, n_jobs=5, n_stages=2, machines=2)
    d = ffsga.DeviceInstance.from_host(inst)
    prio = torch.tensor([[1, 2, 3, 4, 5], [1, 1, 3, 4, 5], [0, 2, 3, 4, 5]], dtype=torch.int32).cuda()
    with pytest.raises(ffsga.FfsError) as e:
        ffsga.ffs_decode(d, prio)
    assert e.value.code == ffsga.FFS_E_INVAL


def test_prepare_reports_infeasible_power():
    _say("prepare infeasible instance")
    torch, ffsga = _ffs()
    inst = W.random_instance(2, n_jobs=4, n_stages=2, machines=2)
    inst.power[2, 1, 1] = inst.q_max + 1
    with pytest.raises(ffsga.FfsError) as e:
        ffsga.DeviceInstance.from_host(inst)
    assert e.value.code == ffsga.FFS_E_INFEASIBLE


def test_prepare_horizon_matches_oracle_bound():
    _, ffsga = _ffs()
    for cfg in (1, 2, 3):
        inst = _event_instance(W.CONFIGS[cfg](0), k_events=1)
        _say("horizon bound, config", cfg)
        d = ffsga.DeviceInstance.from_host(inst)
        assert d.horizon == oracle.horizon_bound(inst)
