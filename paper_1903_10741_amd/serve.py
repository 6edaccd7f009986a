"""Rescheduling service: arrival events of many shops, continuously batched on one GPU.

Each request is one shop's next event (Section 4.1): its first plan, or the
arrival of new jobs at the shop's next rescheduling point. A request waits
until a slot of the batched GA (`ffsga.Batch`) is free and its shop has no
other event in flight (one shop's events are sequential: event e+1 freezes
the plan event e chose). On admission the shop's instance is rescheduled on
the device (executed plan frozen at the arrival's RS, new jobs appended), the
slot runs `generations` generations alongside every other slot in flight, and
the best elite's decoded plan becomes the shop's executed plan. Instances,
populations and plans stay on the device; the host keeps queues and counts.

`Admission` is the queueing policy alone (slots, memory budget, per-shop
order, deadlines) so that it is tested on the CPU with an injected clock.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Callable, Deque, Dict, List, Optional, Sequence, Tuple

import numpy as np


@dataclass
class Request:
    rid: int
    shop: int
    t_arrive: float
    event: int = -1
    slot: int = -1
    t_admit: float = -1.0
    t_done: float = -1.0
    best_obj: int = -1
    status: str = "queued"     # queued, running, done, late, failed
    error: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class Admission:
    """Request queue and slot assignment.

    The number of usable slots is the smaller of `n_slots` and what
    `memory_budget` bytes hold at `slot_bytes` each. A queued request starts
    when a slot is free and no other request of its shop is in flight; the
    queue is served first come, first served, except that a request blocked
    by its own shop does not hold back requests of other shops. A request
    that finishes after `deadline_s` is marked late (its plan is still the
    exact one).
    """

    def __init__(self, n_slots: int, slot_bytes: int, memory_budget: Optional[int] = None,
                 deadline_s: Optional[float] = None, clock: Callable[[], float] = time.perf_counter):
        if n_slots < 1 or slot_bytes < 1:
            raise ValueError("need at least one slot of positive size")
        self.slot_bytes = int(slot_bytes)
        limit = n_slots if memory_budget is None else min(n_slots, int(memory_budget) // self.slot_bytes)
        if limit < 1:
            raise ValueError(f"a memory budget of {memory_budget} bytes holds no slot of "
                             f"{self.slot_bytes} bytes")
        self.n_slots = int(limit)
        self.free: List[int] = list(range(self.n_slots))[::-1]
        self.queue: Deque[Request] = deque()
        self.in_flight: Dict[int, Request] = {}      # shop -> its running request
        self.deadline_s = deadline_s
        self.clock = clock
        self.next_rid = 0

    def submit(self, shop: int, t_arrive: Optional[float] = None) -> Request:
        r = Request(self.next_rid, int(shop), self.clock() if t_arrive is None else t_arrive)
        self.next_rid += 1
        self.queue.append(r)
        return r

    def admit(self) -> List[Request]:
        """Requests that start now, each with its slot."""
        out: List[Request] = []
        kept: Deque[Request] = deque()
        while self.queue:
            r = self.queue.popleft()
            if self.free and r.shop not in self.in_flight:
                r.slot = self.free.pop()
                r.t_admit = self.clock()
                r.status = "running"
                self.in_flight[r.shop] = r
                out.append(r)
            else:
                kept.append(r)
        self.queue = kept
        return out

    def release(self, r: Request, status: str = "done", error: str = ""):
        r.t_done = self.clock()
        if status == "done" and self.deadline_s is not None and r.latency > self.deadline_s:
            status = "late"
        r.status = status
        r.error = error
        if self.in_flight.get(r.shop) is r:
            del self.in_flight[r.shop]
        if r.slot >= 0:
            self.free.append(r.slot)

    @property
    def busy(self) -> int:
        return self.n_slots - len(self.free)


def percentiles(values: Sequence[float], qs=(50, 99)) -> Dict[str, Optional[float]]:
    if len(values) == 0:
        return {f"p{q}": None for q in qs}
    a = np.asarray(values, dtype=np.float64)
    return {f"p{q}": float(np.percentile(a, q)) for q in qs}


def horizon_room(inst, arrivals) -> int:
    """A bound on every event's horizon for one shop.

    With B_e = RS_e + horizon_e (the horizon bound is the latest of RS,
    ready times, machine-free times and running ends, minus RS, plus the
    longest time of every unfrozen op, plus one), B_0 <= R + S + 1 and
    B_e <= max(RS_e, B_(e-1)) + S + 1, where R is the latest release of the
    first event and S sums the longest time of every op the shop ever holds.
    So every horizon is at most R + RS_last + (events) * (S + 1).
    """
    s = int(np.asarray(inst.proc).max(axis=2).sum()) if inst.n_jobs else 0
    s += sum(int(np.asarray(a.proc).max(axis=2).sum()) for a in arrivals)
    rs_last = max([0] + [int(a.rs) for a in arrivals])
    base = max([0] + [int(x) for x in np.asarray(inst.release)])
    return base + rs_last + (1 + len(arrivals)) * (s + 1)


def poisson_schedule(seed: int, rate_per_s: float, n_events: Sequence[int]) -> List[Tuple[float, int]]:
    """A Poisson request stream: (offset in seconds, shop) pairs, exactly
    n_events[k] requests for shop k, the shops' requests interleaved at random."""
    rng = np.random.default_rng(seed)
    shops = np.repeat(np.arange(len(n_events)), np.asarray(n_events, dtype=np.int64))
    rng.shuffle(shops)
    t = np.cumsum(rng.exponential(1.0 / rate_per_s, size=len(shops)))
    return [(float(a), int(b)) for a, b in zip(t, shops)]


@dataclass
class Shop:
    sid: int
    inst: object                       # ffsga.DeviceInstance of the shop's latest event
    arrivals: list                     # workloads.Arrival not yet applied, in order
    plan_start: object                 # device int32 [jobs the shop will hold, g]
    plan_mach: object
    event: int = 0                     # events planned so far
    history: List[int] = field(default_factory=list)


class Server:
    """The service loop: device-resident shops and one batched GA of `n_slots` slots."""

    def __init__(self, instances, arrivals, ga, generations=100, n_slots=64, gens_per_tick=5,
                 memory_budget=None, deadline_s=None, seed=0, device="cuda", tuning=None,
                 max_horizon=None, clock: Callable[[], float] = time.perf_counter):
        import torch
        from . import ffsga
        self.torch, self.ffsga = torch, ffsga
        self.device = torch.device(device)
        self.generations = int(generations)
        self.gens_per_tick = max(1, int(gens_per_tick))
        self.seed = int(seed)
        self.clock = clock
        if len(instances) != len(arrivals):
            raise ValueError("one arrival list per shop")
        jobs = [int(i.n_jobs) + sum(len(a.release) for a in arr) for i, arr in zip(instances, arrivals)]
        if max_horizon is None:
            max_horizon = max(horizon_room(i, arr) for i, arr in zip(instances, arrivals))
        tuning = tuning or {}
        cfg = ffsga.BatchConfig(
            n_slots=n_slots, max_jobs=max(jobs), max_genes=max(jobs),
            max_stages=max(int(i.n_stages) for i in instances),
            o_max=max(int(i.o_max) for i in instances), max_horizon=int(max_horizon),
            ga=ffsga.GaConfig.of(ga, lds_slots=tuning.get("lds_slots", 0)),
            schedule=tuning.get("schedule", ffsga.FFS_SCHEDULE_CHROMOSOME),
            blocks=tuning.get("blocks", 0), use_graph=tuning.get("use_graph", True),
            profile_classes=tuning.get("profile_classes", 1))
        # the most slots whose workspace fits the memory budget
        fit = int(n_slots)
        if memory_budget is not None:
            while fit >= 1 and _replace(cfg, n_slots=fit).workspace_bytes() > int(memory_budget):
                fit -= 1
            if fit < 1:
                raise ValueError(f"a memory budget of {memory_budget} bytes holds no slot")
        one = _replace(cfg, n_slots=1).workspace_bytes()
        per_slot = _replace(cfg, n_slots=2).workspace_bytes() - one
        self.adm = Admission(fit, per_slot, None, deadline_s, clock)
        self.cfg = _replace(cfg, n_slots=self.adm.n_slots)
        self.batch = ffsga.Batch(self.cfg, device=device)
        self.shops: List[Shop] = []
        for sid, (inst, arr) in enumerate(zip(instances, arrivals)):
            plan = torch.full((jobs[sid], int(inst.n_stages)), -1, dtype=torch.int32, device=self.device)
            self.shops.append(Shop(sid, ffsga.DeviceInstance.from_host(inst, device=device),
                                   list(arr), plan, plan.clone()))
        self.running: Dict[int, Request] = {}          # slot -> request
        self.requests: List[Request] = []
        self.decodes = 0
        self.ticks = 0

    # -- one request ---------------------------------------------------------
    def _begin(self, r: Request):
        """Reschedule the shop for its next event and load it into r's slot."""
        ffsga = self.ffsga
        sh = self.shops[r.shop]
        nxt = sh.inst
        if sh.event > 0:
            if not sh.arrivals:
                raise ffsga.FfsError(ffsga.FFS_E_INVAL, f"shop {r.shop} has no arrival left")
            n = int(sh.inst.s.n_jobs)
            nxt = ffsga.reschedule(sh.inst, sh.plan_start[:n], sh.plan_mach[:n], sh.arrivals[0])
        self.batch.set(r.slot, nxt, self.seed, r.shop, sh.event)
        # the shop moves to its next event only once its slot holds it: a failed
        # rescheduling or load leaves the shop, its plan and its arrivals as they were
        if nxt is not sh.inst:
            sh.arrivals.pop(0)
            sh.inst = nxt
        r.event = sh.event
        self.running[r.slot] = r

    def _finish(self, r: Request):
        """The slot's best elite, decoded, becomes the shop's executed plan."""
        ffsga = self.ffsga
        sh = self.shops[r.shop]
        prio, obj = self.batch.best(r.slot)
        n = int(sh.inst.s.n_jobs)
        # decoded ops land in the executed plan; frozen entries keep their values
        ffsga.ffs_decode(sh.inst, prio.view(1, -1), start_out=sh.plan_start[:n],
                         mach_out=sh.plan_mach[:n])
        r.best_obj = int(obj.item())
        sh.history.append(r.best_obj)
        sh.event += 1
        self.batch.clear(r.slot)
        del self.running[r.slot]
        self.decodes += (1 + self.generations) * self.batch.pop + 1

    # -- the loop ------------------------------------------------------------
    def tick(self):
        """Admit what fits, advance every slot in flight, retire finished ones."""
        ffsga = self.ffsga
        for r in self.adm.admit():
            try:
                self._begin(r)
            except ffsga.FfsError as e:
                self.running.pop(r.slot, None)
                self.adm.release(r, "failed", str(e))
        if not self.running:
            return
        # never step a slot past `generations`: stop at the nearest finish
        left = min(self.generations - self.batch.generation(s) for s in self.running)
        if left > 0:
            self.batch.step(min(self.gens_per_tick, left))
            self.ticks += 1
        for s, r in list(self.running.items()):
            if self.batch.generation(s) >= self.generations:
                self._finish(r)
                self.adm.release(r, "done")

    def prime(self, log: Optional[Callable[[str], None]] = None) -> dict:
        """Plan every shop's first event (its initial instance) through the same
        batched path, so that the requests that follow are arrival events; the
        metrics of this phase are returned and then cleared."""
        m = self.run([(0.0, s.sid) for s in self.shops if s.event == 0], log=log)
        self.reset_metrics()
        return m

    def reset_metrics(self):
        """Forget finished requests and counts (shops, plans and slots stay)."""
        self.requests = []
        self.decodes = 0
        self.ticks = 0

    def run(self, schedule: Sequence[Tuple[float, int]], time_limit_s: Optional[float] = None,
            idle_sleep_s: float = 1e-4, log: Optional[Callable[[str], None]] = None,
            log_every: int = 100) -> dict:
        """Serve a request stream of (offset in seconds, shop). Returns the metrics.
        `log`, if given, receives a progress line every `log_every` finished requests."""
        t0 = self.clock()
        pending = deque(sorted(schedule))
        reported = 0
        while pending or self.adm.queue or self.running:
            if log:
                n_done = sum(r.status in ("done", "late") for r in self.requests)
                if n_done >= reported + log_every:
                    reported = n_done
                    log(f"{n_done} requests served, {len(self.adm.queue)} queued, "
                        f"{len(self.running)} running, {self.clock() - t0:.1f} s")
            now = self.clock() - t0
            while pending and pending[0][0] <= now:
                t, shop = pending.popleft()
                self.requests.append(self.adm.submit(shop, t0 + t))
            if self.adm.queue or self.running:
                self.tick()
            else:
                time.sleep(min(idle_sleep_s, max(0.0, pending[0][0] - now)))
            if time_limit_s is not None and self.clock() - t0 > time_limit_s:
                break
        self.batch.stream.synchronize()
        return self.metrics(self.clock() - t0)

    def metrics(self, wall_s: float) -> dict:
        done = [r for r in self.requests if r.status in ("done", "late")]
        lat = [r.latency for r in done]
        wait = [r.t_admit - r.t_arrive for r in done]
        return {"requests": len(self.requests), "done": len(done),
                "failed": sum(r.status == "failed" for r in self.requests),
                "late": sum(r.status == "late" for r in self.requests),
                "unfinished": sum(r.status in ("queued", "running") for r in self.requests),
                "wall_s": wall_s, "decodes": self.decodes,
                "decodes_per_s": self.decodes / wall_s if wall_s > 0 else 0.0,
                "requests_per_s": len(done) / wall_s if wall_s > 0 else 0.0,
                **{f"latency_{k}_s": v for k, v in percentiles(lat).items()},
                **{f"queue_{k}_s": v for k, v in percentiles(wait).items()},
                "slots": self.adm.n_slots, "ticks": self.ticks}


def _replace(cfg, **kw):
    from dataclasses import replace
    return replace(cfg, **kw)
