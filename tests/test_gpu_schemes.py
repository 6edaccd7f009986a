"""The comparison GAs of Section 5.2 (classical and cellular, ffs_ga_params.scheme)
on the GPU against the oracle, whole state, generation by generation."""
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


def _state(ga):
    return {k: t.cpu().numpy() for k, t in ga.view().items() if k != "work"}


def _same(a, b, what):
    for k in ("prio", "obj", "elite", "elite_obj"):
        assert (np.asarray(a[k]) == np.asarray(b[k])).all(), (what, k)


def _run(inst, gp, scheme, seed, gens, lds_slots=0, check_every=1, event=0):
    torch, ffsga = _ffs()
    d = ffsga.DeviceInstance.from_host(inst)
    ga = ffsga.GA(d, ffsga.GaConfig.of(gp, lds_slots=lds_slots, scheme=scheme), seed, 0, event)
    st = oracle.ga_init(inst, gp, seed, 0, event, n_threads=8)
    _same(_state(ga), st, "init")
    e = oracle.emax(st["obj"])
    if scheme == ffsga.FFS_GA_CLASSICAL:
        assert ga.e_max() == e
    for g in range(1, gens + 1):
        st = oracle.ga_generation_scheme(inst, gp, scheme, e, seed, 0, event, g, st, n_threads=8)
        if g % check_every == 0 or g == gens:
            ga.step(g - ga.generation)
            _same(_state(ga), st, f"scheme {scheme} gen {g}")
    ga.status()


@pytest.mark.parametrize("scheme", [1, 2])
def test_scheme_tiny_every_generation(scheme):
    _say("comparison GA", scheme, "tiny-10x2x2, 8x8, 40 generations")
    wl = W.config1(0)
    _run(wl.initial, W.GaParams(1, 8, 8), scheme, 3, 40)


@pytest.mark.parametrize("scheme", [1, 2])
def test_scheme_paper_shaped_64x64(scheme):
    """Table 8's smallest population (64 x 64 = 4096) on the paper-shaped instance."""
    _say("comparison GA", scheme, "paper-50x5x3, 64x64, 20 generations")
    wl = W.config2(1)
    _run(wl.initial, W.GaParams(1, 64, 64), scheme, 5, 20, check_every=5)


@pytest.mark.parametrize("scheme", [1, 2])
def test_scheme_odd_grid_rescheduled_and_off_chip(scheme):
    """A 3 x 5 grid (the classical GA's last slot has no partner), a rescheduled
    instance, and 64 on-chip slots so most decodes are redone off chip before the
    cellular acceptance."""
    _say("comparison GA", scheme, "odd grid, event 1, 64 on-chip slots")
    from oracle_helpers import rescheduled_instance
    inst = rescheduled_instance(W.config1(2), k_events=1)
    _run(inst, W.GaParams(1, 3, 5), scheme, 8, 12, lds_slots=64, event=1)


def test_schemes_reject_what_they_do_not_run():
    torch, ffsga = _ffs()
    _say("comparison GA parameter checks")
    wl = W.config1(0)
    d = ffsga.DeviceInstance.from_host(wl.initial)
    for gp, scheme, enc in ((W.GaParams(2, 4, 4), 1, 0), (W.GaParams(1, 4, 4), 2, 1),
                            (W.GaParams(1, 4, 4), 3, 0)):
        with pytest.raises(ffsga.FfsError) as e:
            ffsga.GA(d, ffsga.GaConfig.of(gp, encoding=enc, scheme=scheme), 1, 0, 0)
        assert e.value.code == ffsga.FFS_E_INVAL
