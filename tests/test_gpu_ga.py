"""GPU island GA (ga_init / ga_step / ga_best through the C ABI) against the oracle.

The Philox stream makes every generation recomputable from its predecessor,
so GPU and oracle populations, objectives and elites must agree bit for bit.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle_helpers import oracle_islands
from paper_1903_10741_amd import workloads as W

pytestmark = pytest.mark.gpu


def _ffs():
    import torch
    from paper_1903_10741_amd import ffsga
    assert torch.cuda.is_available()
    return torch, ffsga


def _say(*a):
    print("[case]", *a, flush=True)


def _state(ga):
    v = ga.view()
    return {k: t.cpu().numpy() for k, t in v.items() if k != "work"}


def _same(a, b, what):
    for k in ("prio", "obj", "elite", "elite_obj"):
        assert (np.asarray(a[k]) == np.asarray(b[k])).all(), (what, k)


def test_ga_init_matches_oracle():
    torch, ffsga = _ffs()
    for cfg in (1, 2):
        wl = W.CONFIGS[cfg](0)
        _say("ga_init config", cfg)
        d = ffsga.DeviceInstance.from_host(wl.initial)
        ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
        ga.status()
        want = oracle.ga_init(wl.initial, wl.ga, wl.seed, wl.shop, 0, n_threads=8)
        _same(_state(ga), want, f"init cfg {cfg}")


def test_ga_config1_every_generation():
    torch, ffsga = _ffs()
    wl = W.config1(0)
    _say("config 1, 50 generations, checked every generation")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
    st = oracle.ga_init(wl.initial, wl.ga, wl.seed, wl.shop, 0)
    for k in range(1, wl.generations + 1):
        ga.step(1)
        st = oracle.ga_generation(wl.initial, wl.ga, wl.seed, wl.shop, 0, k, st)
        _same(_state(ga), st, f"gen {k}")
    ga.status()
    prio, obj = ga.best()
    bp, bo = oracle.ga_best(st)
    assert int(obj.item()) == bo and (prio.cpu().numpy() == bp).all()


def test_ga_config2_first_event_prefix():
    """Config 2 at full population (32 islands x 8x16): 30 generations, three
    of them migrating, compared whole."""
    torch, ffsga = _ffs()
    wl = W.config2(0)
    _say("config 2, 30 generations, full population")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
    st = oracle.ga_init(wl.initial, wl.ga, wl.seed, wl.shop, 0, n_threads=8)
    for k in range(1, 31):
        st = oracle.ga_generation(wl.initial, wl.ga, wl.seed, wl.shop, 0, k, st, n_threads=8)
        if k % 10 == 0:
            ga.step(10)
            _same(_state(ga), st, f"gen {k}")
    ga.status()


def _same_islands(got, want, islands, K, what):
    for I in islands:
        sl = slice(I * K, (I + 1) * K)
        assert (got["prio"][sl] == want["prio"][sl]).all(), (what, I)
        assert (got["obj"][sl] == want["obj"][sl]).all(), (what, I)
        assert (got["elite"][I] == want["elite"][I]).all(), (what, I)
        assert got["elite_obj"][I] == want["elite_obj"][I], (what, I)


def test_ga_config2_full_event():
    """Config 2's whole first event (500 generations) against the oracle's own
    500-generation run, compared whole at generations 99, 250 and 500."""
    torch, ffsga = _ffs()
    wl = W.config2(0)
    _say("config 2, 500 generations, whole state at 99, 250, 500")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
    st = oracle.ga_init(wl.initial, wl.ga, wl.seed, wl.shop, 0, n_threads=8)
    for k in range(1, 501):
        st = oracle.ga_generation(wl.initial, wl.ga, wl.seed, wl.shop, 0, k, st, n_threads=8)
        if k in (99, 250, 500):
            ga.step(k - ga.generation)
            _same(_state(ga), st, f"gen {k}")
    assert ga.generation == 500
    ga.status()


def test_ga_config3_sampled_islands():
    """Config 3 (512 islands x 8x16 = 65536): sampled islands against the oracle's
    own run of them (and of what they depend on), at a plain and a migrating
    generation."""
    torch, ffsga = _ffs()
    wl = W.config3(0)
    _say("config 3, pop 65536, sampled islands")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
    want0 = oracle.ga_init(wl.initial, W.GaParams(1, 8, 16), wl.seed, wl.shop, 0, n_threads=8)
    got0 = _state(ga)
    assert (got0["prio"][:128] == want0["prio"]).all() and (got0["obj"][:128] == want0["obj"]).all()
    K = wl.ga.rows * wl.ga.cols
    for G, islands in ((9, [0, 77, 511]), (10, [1, 300, 511])):   # generation 10 migrates
        ga.step(G - ga.generation)
        want = oracle_islands(wl.initial, wl.ga, wl.seed, wl.shop, 0, islands, G)
        _same_islands(_state(ga), want, islands, K, f"gen {G}")
    ga.status()


def test_ga_overflow_tier_in_the_loop():
    """A GA whose decodes mostly overflow the on-chip profile stays bit-exact."""
    torch, ffsga = _ffs()
    wl = W.config1(3)
    _say("GA with lds_slots = 64 (overflow tier)")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga, lds_slots=64), wl.seed, wl.shop, 0)
    ga.step(12)
    ga.status()
    st = oracle.ga_run(wl.initial, wl.ga, wl.seed, wl.shop, 0, 12)
    _same(_state(ga), st, "overflow GA")


def test_ga_auto_size_beyond_the_sizing_decode():
    """Schedules of 20 000-26 000 slots: generation 0's sizing decode keeps 16 384
    slots on chip, so its decodes are redone off chip, and those redos record the
    true lengths: later generations get more slots than the sizing decode had,
    and the populations equal the oracle's."""
    torch, ffsga = _ffs()
    inst = W.random_instance(23, n_jobs=24, n_stages=3, machines=2, p_max=1500, percent=60)
    gp = W.GaParams(2, 4, 8, mig_interval=2, mig_k=1)
    _say("FFS_LDS_AUTO past the sizing decode's 16384 slots")
    d = ffsga.DeviceInstance.from_host(inst)
    ga = ffsga.GA(d, ffsga.GaConfig.of(gp, lds_slots=ffsga.FFS_LDS_AUTO), 5, 0, 0)
    assert ga.overflows() > 0
    assert 20000 < int(ga.ga.lds_slots) <= 32768, int(ga.ga.lds_slots)
    ga.step(4)
    ga.status()
    st = oracle.ga_run(inst, gp, 5, 0, 0, 4)
    _same(_state(ga), st, "auto size beyond the sizing decode")


def test_ga_narrow_layout_with_inline_redo():
    """200 jobs, 6144 individuals and 5440-5760 on-chip slots (about 7.5 KB of LDS
    per wave): 16-bit ready times save 400 bytes a wave, which at some of these
    sizes lets a compute unit hold one more wave, and 6144 individuals are more
    than the chip holds at once, so there the generation kernels take the narrow
    layout (at least one size must). The schedules outgrow the slots and each is
    redone by its own wave in the wide layout over the same LDS (6144 off-chip
    profiles fit the 1 GiB the workspace allows). Whole state against the oracle
    at every size."""
    torch, ffsga = _ffs()
    wl = W.config3(0)
    gp = W.GaParams(48, 8, 16, mig_interval=2, mig_k=2)
    st = oracle.ga_run(wl.initial, gp, wl.seed, wl.shop, 0, 3, n_threads=8)
    d = ffsga.DeviceInstance.from_host(wl.initial)
    narrow = []
    for slots in (5440, 5504, 5568, 5632, 5696, 5760):
        _say("narrow layout, inline redo: 200 jobs, pop 6144, slots", slots)
        ga = ffsga.GA(d, ffsga.GaConfig.of(gp, lds_slots=slots), wl.seed, wl.shop, 0)
        ga.step(3)
        ga.status()
        assert ga.overflows() > 0
        narrow.append(int(ga.ga.narrow_lds))
        _same(_state(ga), st, f"{slots} slots, narrow {narrow[-1]}")
    _say("narrow layout taken at", narrow)
    assert any(narrow)


def test_ga_odd_island_shape_and_tiny_genes():
    """Odd torus sides leave unpaired slots; n_active = 1 and 2 have no or one cut."""
    torch, ffsga = _ffs()
    for n, (isl, r, c) in ((1, (2, 3, 5)), (2, (3, 3, 3)), (7, (2, 5, 3))):
        _say("GA shape", isl, r, c, "genes", n)
        inst = W.random_instance(n, n_jobs=n, n_stages=2, machines=2, percent=50)
        gp = W.GaParams(isl, r, c, mig_interval=3, mig_k=2)
        d = ffsga.DeviceInstance.from_host(inst)
        ga = ffsga.GA(d, ffsga.GaConfig.of(gp), 11, 4, 2)
        ga.step(7)
        ga.status()
        st = oracle.ga_run(inst, gp, 11, 4, 2, 7)
        _same(_state(ga), st, f"shape {isl}x{r}x{c} n={n}")


def test_ga_is_deterministic():
    torch, ffsga = _ffs()
    wl = W.config2(1)
    _say("GA determinism")
    d = ffsga.DeviceInstance.from_host(wl.initial)
    runs = []
    for _ in range(2):
        ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
        ga.step(25)
        runs.append(_state(ga))
    _same(runs[0], runs[1], "determinism")


def test_ga_island_groups_change_nothing():
    """ga_step over 1, 3 and 4 concurrent island groups gives the same populations,
    objectives and elites, for job vectors and X/Y chromosomes. Config 2 has 32
    islands: groups of 10-11 and of 8; the migrations at generations 10 and 20
    join the groups in mid-call and calls of 7 and 18 generations fork and join at
    their ends. The generation launches counted with HIP events show that the
    grouped runs did launch one generation kernel per group."""
    torch, ffsga = _ffs()
    wl = W.config2(3)
    d = ffsga.DeviceInstance.from_host(wl.initial)
    try:
        for enc in (0, 1):
            gp = dataclasses.replace(wl.ga, encoding=enc)
            runs = {}
            for groups in (1, 3, 4):
                _say("island groups", groups, "encoding", enc)
                ffsga.set_island_groups(groups)
                ga = ffsga.GA(d, ffsga.GaConfig.of(gp), wl.seed, wl.shop, 0)
                ffsga.timing_enable(True, families=[ffsga.TIMING_GENERATION], every=1)
                ga.step(7)
                ga.step(18)
                torch.cuda.synchronize()
                _, launches = ffsga.timing_read(ffsga.TIMING_GENERATION)
                ffsga.timing_enable(False)
                assert launches == 25 * groups, (groups, launches)
                ga.status()
                runs[groups] = _state(ga)
            for groups in (3, 4):
                _same(runs[groups], runs[1], f"{groups} island groups, encoding {enc}")
    finally:
        ffsga.timing_enable(False)
        ffsga.set_island_groups(0)
    for bad in (-1, 5):
        with pytest.raises(ffsga.FfsError):
            ffsga.set_island_groups(bad)


def test_ga_auto_sized_profile_changes_nothing():
    """FFS_LDS_AUTO (on-chip slots sized from generation 0's longest schedule)
    gives the same populations as the default slots and the oracle; the chosen
    slots are a multiple of 64 and stay below the horizon."""
    torch, ffsga = _ffs()
    for cfg, gens in ((1, 12), (2, 20)):
        wl = W.CONFIGS[cfg](2)
        _say("GA with FFS_LDS_AUTO, config", cfg)
        d = ffsga.DeviceInstance.from_host(wl.initial)
        ga = ffsga.GA(d, ffsga.GaConfig.of(wl.ga, lds_slots=ffsga.FFS_LDS_AUTO), wl.seed, wl.shop, 0)
        cap = int(ga.ga.lds_slots)
        assert cap % 64 == 0 and 64 <= cap <= (d.horizon + 63) // 64 * 64
        ga.step(gens)
        ga.status()
        ref = ffsga.GA(d, ffsga.GaConfig.of(wl.ga), wl.seed, wl.shop, 0)
        ref.step(gens)
        _same(_state(ga), _state(ref), f"auto vs default cfg {cfg}")
        st = oracle.ga_run(wl.initial, wl.ga, wl.seed, wl.shop, 0, gens, n_threads=8)
        _same(_state(ga), st, f"auto vs oracle cfg {cfg}")
