"""The predictive-reactive event loop on the device (Section 4.1).

For each event: the island GA runs on the current instance, the best elite's
plan is decoded (start and machine of every op) straight into the executed
plan, and at the next arrival the plan is frozen and the instance
rescheduled, all through the C ABI. Only the host-side bookkeeping (which
arrays belong to which event) lives here.
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
    work: torch.Tensor = None      # device int64 [1]: work of every decode of the event's GA
    lds_slots: int = 0             # on-chip profile slots the event's generations used
    decodes: int = 0               # the GA's decodes plus the executed plan's
    overflows: int = 0             # the GA's decodes redone off chip
    island_groups: int = 1         # island groups the event's ga_step ran concurrently
    narrow_lds: int = 0            # 1 if its generations kept ready times in 16 bits


@dataclass
class RunResult:
    events: List[EventResult] = field(default_factory=list)
    plan_start: torch.Tensor = None
    plan_mach: torch.Tensor = None
    decodes: int = 0
    ga_decodes: int = 0
    work: int = 0


class EventLoop:
    """The events of a workload run one at a time, in order: event e's GA (init +
    `generations`), the decode of its best plan into the executed plan, and the
    rescheduling at arrival e. After the last event the loop starts again at
    event 0 from the initial instance, which stays resident on the device.
    static=True handles every arrival by the traditional static approach
    (reschedule_static) instead of complete rescheduling."""

    def __init__(self, wl, device="cuda", generations=None, lds_slots=0, keep_instances=False,
                 static=False):
        self.wl = wl
        self.gens = wl.generations if generations is None else generations
        self.cfg = ffsga.GaConfig.of(wl.ga, lds_slots=lds_slots)
        self.keep_instances = keep_instances
        self.static = static
        g = int(wl.initial.n_stages)
        n_final = int(wl.initial.n_jobs) + sum(len(a.release) for a in wl.arrivals)
        self.plan_s = torch.full((n_final, g), -1, dtype=torch.int32, device=device)
        self.plan_m = torch.full((n_final, g), -1, dtype=torch.int32, device=device)
        self.initial = ffsga.DeviceInstance.from_host(wl.initial, device=device)
        self.ga_ws = None
        self.n_events = 1 + len(wl.arrivals)
        self.event = 0

    def run_event(self) -> EventResult:
        """Run the current event and move on to the next (event 0 after the last;
        the executed plan of the finished cycle stays readable until then)."""
        if self.event == 0:
            self.dinst = self.initial
            self.plan_s.fill_(-1)
            self.plan_m.fill_(-1)
        e, d = self.event, self.dinst
        ga = ffsga.GA(d, self.cfg, self.wl.seed, self.wl.shop, e, workspace=self.ga_ws)
        self.ga_ws = ga.ws
        ga.step(self.gens)
        prio, obj = ga.best()
        n = int(d.s.n_jobs)
        ffsga.ffs_decode(d, prio.view(1, -1), lds_slots=int(ga.ga.lds_slots),
                         xy=self.cfg.encoding == 1, start_out=self.plan_s[:n],
                         mach_out=self.plan_m[:n])
        ev = EventResult(e, int(d.s.rs), d.n_active, best_prio=prio, best_obj=obj,
                         work=ga.view()["work"].clone(), lds_slots=int(ga.ga.lds_slots),
                         decodes=(1 + self.gens) * ga.ga.pop + 1, overflows=ga.overflows(),
                         island_groups=int(ga.ga.island_groups),
                         narrow_lds=int(ga.ga.narrow_lds))
        if self.keep_instances:
            ev.instance = d
        if e + 1 < self.n_events:
            self.dinst = ffsga.reschedule(d, self.plan_s[:n], self.plan_m[:n], self.wl.arrivals[e],
                                          static=self.static)
            self.event = e + 1
        else:
            self.event = 0
        return ev


def run_workload(wl, device="cuda", generations=None, lds_slots=0, keep_instances=False,
                 sync_results=True, keep_work=False, static=False) -> RunResult:
    """Run every event of workload `wl` on the device. Returns per-event best objectives."""
    loop = EventLoop(wl, device, generations, lds_slots, keep_instances, static)
    res = RunResult()
    for _ in range(loop.n_events):
        ev = loop.run_event()
        res.events.append(ev)
        res.decodes += ev.decodes
        res.ga_decodes += ev.decodes - 1
    res.plan_start, res.plan_mach = loop.plan_s, loop.plan_m
    if keep_work:
        res.work = int(sum(int(ev.work.item()) for ev in res.events))
    if sync_results:
        for ev in res.events:
            ev.best_obj = int(ev.best_obj.item())
    return res
