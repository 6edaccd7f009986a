"""Autotuner for the batched GA launch.

For a given set of instances and GA shape it times, on the device, the
candidate launch configurations of the batched generation (schedule: one wave
per child or one wave per island; on-chip profile slots; persistent grid
size; graph replay) over a few generations of a scratch batch, and returns
the fastest. Every candidate computes the same results (the tests hold each
schedule to the oracle); only the time differs. Results are cached per shape
signature in a JSON file when a path is given.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import asdict, dataclass
from typing import Dict, List, Optional, Sequence

import torch

from . import ffsga


@dataclass
class Candidate:
    schedule: int
    lds_slots: int
    blocks: int
    use_graph: bool
    profile_classes: int = 1


@dataclass
class TuneResult:
    best: Candidate
    us_per_generation: float
    table: List[dict]


def signature(insts: Sequence, ga) -> str:
    """Shape key: size buckets of the instances and the GA shape."""
    def bucket(x):
        return 1 << max(0, int(x) - 1).bit_length()
    sizes = sorted((bucket(i.n_active), int(i.n_stages), int(i.o_max)) for i in insts)
    return json.dumps({"n": len(insts), "sizes": sizes[:: max(1, len(sizes) // 16)],
                       "ga": [ga.islands, ga.rows, ga.cols, ga.mig_interval, ga.mig_k]})


def default_candidates(n_cu: int, horizon_max: int) -> List[Candidate]:
    """On-chip profile slots from 4096 up to the largest horizon (at most 32768;
    a decode whose schedule outgrows them is redone off chip), persistent grids of
    4, 8 and 16 blocks per CU, both schedules, graph replay; one eager candidate."""
    out = []
    ladder = [x for x in (4096, 8192, 16384, 32768) if x < 2 * horizon_max] or [4096]
    for lds in ladder:
        for blocks in (4 * n_cu, 8 * n_cu, 16 * n_cu):
            out.append(Candidate(ffsga.FFS_SCHEDULE_CHROMOSOME, lds, blocks, True))
        out.append(Candidate(ffsga.FFS_SCHEDULE_ISLAND, lds, 8 * n_cu, True))
        # size classes from 2048 up to lds (at most 4)
        cls = min(ffsga.FFS_BATCH_MAX_CLASSES, max(1, (lds // 2048).bit_length()))
        if cls > 1:
            for blocks in (8 * n_cu, 16 * n_cu):
                out.append(Candidate(ffsga.FFS_SCHEDULE_CHROMOSOME, lds, blocks, True, cls))
    out.append(Candidate(ffsga.FFS_SCHEDULE_CHROMOSOME, ladder[-1], 8 * n_cu, False))
    return out


def batch_config(insts, ga, horizon_max, cand: Candidate, n_slots=None) -> ffsga.BatchConfig:
    return ffsga.BatchConfig(
        n_slots=n_slots or len(insts), max_jobs=max(int(i.n_jobs) for i in insts),
        max_genes=max(i.n_active for i in insts), max_stages=max(int(i.n_stages) for i in insts),
        o_max=max(int(i.o_max) for i in insts), max_horizon=horizon_max,
        ga=ffsga.GaConfig.of(ga, lds_slots=cand.lds_slots), schedule=cand.schedule,
        blocks=cand.blocks, use_graph=cand.use_graph, profile_classes=cand.profile_classes)


def time_candidate(dev_insts, insts, ga, horizon_max, cand: Candidate, generations=3,
                   warmup=1) -> float:
    """Microseconds per generation of a scratch batch holding every instance."""
    b = ffsga.Batch(batch_config(insts, ga, horizon_max, cand))
    try:
        for s, d in enumerate(dev_insts):
            b.set(s, d, seed=1, shop=s, event=0)
        b.step(warmup)
        b.stream.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(b.stream)
        b.step(generations)
        stop.record(b.stream)
        stop.synchronize()
        b.status()
        return start.elapsed_time(stop) * 1e3 / generations
    finally:
        b.destroy()
        del b


def tune(dev_insts, insts, ga, candidates: Optional[List[Candidate]] = None,
         cache_path: Optional[str] = None, generations=3, log=None) -> TuneResult:
    horizon_max = max(d.horizon for d in dev_insts)
    key = signature(insts, ga)
    cache: Dict[str, dict] = {}
    if cache_path and os.path.exists(cache_path):
        cache = json.load(open(cache_path))
        if key in cache:
            c = cache[key]
            return TuneResult(Candidate(**c["best"]), c["us_per_generation"], c["table"])
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cands = candidates or default_candidates(n_cu, horizon_max)
    table = []
    for cand in cands:
        t0 = time.perf_counter()
        us = time_candidate(dev_insts, insts, ga, horizon_max, cand, generations)
        table.append({**asdict(cand), "us_per_generation": us,
                      "tuning_s": time.perf_counter() - t0})
        if log:
            log(f"autotune {asdict(cand)}: {us:.0f} us/generation")
    best = min(table, key=lambda r: r["us_per_generation"])
    res = TuneResult(Candidate(best["schedule"], best["lds_slots"], best["blocks"],
                               best["use_graph"], best["profile_classes"]),
                     best["us_per_generation"], table)
    if cache_path:
        cache[key] = {"best": asdict(res.best), "us_per_generation": res.us_per_generation,
                      "table": table}
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1)
    return res
