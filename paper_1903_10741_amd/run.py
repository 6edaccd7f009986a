"""The predictive-reactive event loop on the device (Section 4.1).

For each event: the island GA runs on the current instance, the best elite's
plan is decoded (start and machine of every op) into the executed plan, and
at the next arrival the plan is frozen and the instance rescheduled, all
through the C ABI. Only the host-side bookkeeping (which arrays belong to
which event) lives here.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import torch

from . import ffsga


@dataclass
class EventResult:
    event: int
    rs: int
    n_active: int
    best_obj: int = -1
    best_prio: torch.Tensor = None
    instance: "ffsga.DeviceInstance" = None


@dataclass
class RunResult:
    events: List[EventResult] = field(default_factory=list)
    plan_start: torch.Tensor = None
    plan_mach: torch.Tensor = None
    decodes: int = 0
    ga_decodes: int = 0
    work: int = 0


def run_workload(wl, device="cuda", generations=None, lds_slots=0, keep_instances=False,
                 sync_results=True, keep_work=False) -> RunResult:
    """Run every event of workload `wl` on the device. Returns per-event best objectives."""
    gens = wl.generations if generations is None else generations
    cfg = ffsga.GaConfig.of(wl.ga, lds_slots=lds_slots)
    g = int(wl.initial.n_stages)
    n_final = int(wl.initial.n_jobs) + sum(len(a.release) for a in wl.arrivals)
    plan_s = torch.full((n_final, g), -1, dtype=torch.int32, device=device)
    plan_m = torch.full((n_final, g), -1, dtype=torch.int32, device=device)
    dinst = ffsga.DeviceInstance.from_host(wl.initial, device=device)
    res = RunResult(plan_start=plan_s, plan_mach=plan_m)
    ga_ws = None
    for e in range(1 + len(wl.arrivals)):
        ga = ffsga.GA(dinst, cfg, wl.seed, wl.shop, e, workspace=ga_ws)
        ga_ws = ga.ws
        ga.step(gens)
        prio, obj = ga.best()
        n = int(dinst.s.n_jobs)
        sched = ffsga.ffs_decode(dinst, prio.view(1, -1), lds_slots=lds_slots, want_schedule=True,
                                 xy=cfg.encoding == 1)
        # decoded ops of the best plan overwrite their entries; frozen ones stay
        dec = sched["start"][0] >= 0
        plan_s[:n][dec] = sched["start"][0][dec]
        plan_m[:n][dec] = sched["mach"][0][dec]
        ev = EventResult(e, int(dinst.s.rs), dinst.n_active, best_prio=prio)
        ev.best_obj = obj
        if keep_instances:
            ev.instance = dinst
        res.events.append(ev)
        res.decodes += (1 + gens) * ga.ga.pop + 1
        res.ga_decodes += (1 + gens) * ga.ga.pop
        if keep_work:
            res.work += int(ga.view()["work"].item())
        if e < len(wl.arrivals):
            dinst = ffsga.reschedule(dinst, plan_s[:n], plan_m[:n], wl.arrivals[e])
    if sync_results:
        for ev in res.events:
            ev.best_obj = int(ev.best_obj.item())
    return res
