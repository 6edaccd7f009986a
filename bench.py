"""Benchmark: exact chromosome decodes per second of the whole EDFFS hot path on one GPU.

Default workload: large-200x10x4-6 (200 jobs, 10 stages, 4-6 unrelated
machines per stage, 10 arrival events of 10-30 jobs; the island GA with 512
islands of 8x16 = 65536 individuals, 200 generations per event, 2 best
migrating every 10 generations). One step = one event: the GA (init + 200
generations of selection, crossover, mutation, decode, replacement,
migration), the decode of the executed plan, and the rescheduling at the next
arrival; consecutive steps go through the 11 events in order and start again
at event 0. Inputs are synthetic and seeded, resident on the GPU before the
timed region starts. The paper-shaped workload (50 jobs, 5 stages, 3
machines, 6 events of 4096 individuals x 500 generations, one step = all 6
events) is measured beside it and reported under "paper_shaped".

Prints one JSON line. `roofline` reports the GA generation kernel (breed +
decode, the dominant kernel) against the chip's int32 VALU issue rate, with
the algorithmic work counted by the decoder itself; `cpu_baseline` times the
CPU oracle on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CUs x 128 int32 lanes per clock (4 SIMDs x 32) x 2.4 GHz: the fp32 vector
# figure, 157.3 TFLOP/s, counts an FMA as two FLOP, i.e. 78.6 T lane-FMAs/s; int32
# adds issue at that rate too (measure_peaks reaches 66 T at 8 waves per SIMD, more
# than 64 lanes per clock per CU allow)
VALU_INT32_PEAK_TOPS = 256 * 128 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def cpu_baseline(wl):
    """The CPU oracle (OpenMP over the population, as the paper's master-slave GA) on one
    full step of the same workload: every event's GA, executed plan and rescheduling."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    out = oracle.run_events(wl.initial, wl.arrivals, wl.ga, wl.generations, wl.seed, wl.shop,
                            n_threads=threads)
    dt = time.perf_counter() - t0
    decodes = len(out) * ((1 + wl.generations) * wl.ga.pop + 1)
    # one thread, on a bounded sample: event 0, generation 0 and 4 generations
    t1 = time.perf_counter()
    oracle.ga_run(wl.initial, wl.ga, wl.seed, wl.shop, 0, 4, n_threads=1)
    dt1 = time.perf_counter() - t1
    model = cpu_model()
    return {"value": decodes / dt, "unit": "decodes/s", "cores": threads, "kind": "oracle",
            "sample": f"one full step: {len(out)} events x (1 + {wl.generations}) generations x "
                      f"{wl.ga.pop} individuals + plan decodes ({decodes} decodes, {dt:.1f} s)",
            "single_thread": {"value": 5 * wl.ga.pop / dt1, "unit": "decodes/s", "cores": 1,
                              "sample": f"event 0 only (50 jobs; later events have up to 100 and "
                                        f"decode slower, so this rate is optimistic): generation "
                                        f"0 + 4 generations ({5 * wl.ga.pop} decodes, "
                                        f"{dt1:.1f} s)"},
            "nproc": os.cpu_count(), "cpu_model": model,
            "best_obj_per_event": [int(e["best_obj"]) for e in out]}


def progress(msg):
    """A progress line on stderr (stdout carries only the JSON result)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def common(args, metric, value, unit, ms_per_step, dtype, config, higher=True, scaling="weak"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": higher,
            "scaling": scaling, "vs_baseline": None, "dtype": dtype,
            "data": "synthetic (seeded generator, paper-shaped)", "config": config}


def bench_batch(args):
    """Uneven shops in one batched launch (512 shops, jobs U{20..200}, stages U{3..10},
    machines U{2..6}, population 1024 each): one step = every shop's generation 0 and
    100 generations, in the launch configuration the autotuner picks."""
    import torch
    from paper_1903_10741_amd import autotune, ffsga
    from paper_1903_10741_amd import workloads as W
    shops = W.shops(args.seed, args.shops)
    ga = W.SERVING_GA
    gens = args.generations or 100
    dev = [ffsga.DeviceInstance.from_host(s) for s in shops]
    horizon = max(d.horizon for d in dev)
    if args.no_autotune:
        n_cu = torch.cuda.get_device_properties(0).multi_processor_count
        tune = autotune.TuneResult(autotune.Candidate(ffsga.FFS_SCHEDULE_CHROMOSOME, 8192, 8 * n_cu,
                                                      True, 3), float("nan"), [])
    else:
        tune = autotune.tune(dev, shops, ga, generations=2, log=progress)
    cfg = autotune.batch_config(shops, ga, horizon, tune.best)
    b = ffsga.Batch(cfg)

    def one_step():
        for s, d in enumerate(dev):
            b.set(s, d, args.seed, s, 0)
        b.step(gens)
    for _ in range(args.warmup):
        one_step()
    b.status()
    progress("batch warm-up done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step()
        b.stream.synchronize()
        progress(f"batch step {k + 1} done")
    b.stream.synchronize()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    b.status()
    decodes = len(shops) * ga.pop * (1 + gens)
    # roofline of the generation kernel: a timed eager run of the same shape
    rcand = autotune.Candidate(tune.best.schedule, tune.best.lds_slots, tune.best.blocks, False,
                               tune.best.profile_classes)
    rb = ffsga.Batch(autotune.batch_config(shops, ga, horizon, rcand))
    for s, d in enumerate(dev):
        rb.set(s, d, args.seed, s, 0)
    rb.stream.synchronize()
    w0 = int(rb.view(0)["work"].item())
    ffsga.timing_enable(True, families=[ffsga.TIMING_BATCH])
    rb.step(min(gens, 10))
    gen_ms, launches = ffsga.timing_read(ffsga.TIMING_BATCH)
    ffsga.timing_enable(False)
    rb.status()
    work = int(rb.view(0)["work"].item()) - w0
    avg = gen_ms / 1e3 / max(launches, 1)
    achieved = work / max(launches, 1) / avg / 1e12
    out = common(args, "exact chromosome decodes/sec", decodes * args.steps / elapsed, "decodes/s",
                 elapsed * 1e3 / args.steps, "int32", {
                     "workload": f"batched uneven shops: {len(shops)} shops, jobs U{{20..200}}, "
                                 f"stages U{{3..10}}, machines U{{2..6}}, pop 1024 each, "
                                 f"{gens} generations",
                     "decodes_per_step": decodes, "autotuned": tune.best.__dict__,
                     "tuning_table": tune.table})
    out["roofline"] = {"bound": "alu", "kernel": "batch_generation_kernel", "achieved": achieved,
                       "peak": VALU_INT32_PEAK_TOPS, "unit": "TOP/s int32",
                       "frac": achieved / VALU_INT32_PEAK_TOPS, "traffic": None,
                       "avg_launch_us": avg * 1e6, "launches": launches,
                       "work_per_decode": work / max(len(shops) * ga.pop * min(gens, 10), 1),
                       "build_id": ffsga.ffs_build_id()}
    return out


def oracle_rate_large(wl, gens=20):
    """The CPU oracle on event 0 of the large workload: init + `gens` generations of
    the whole population (OpenMP over the population, all host threads), and one
    thread on a bounded sample of random priority vectors."""
    import oracle
    from paper_1903_10741_amd import workloads as W
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    oracle.ga_run(wl.initial, wl.ga, wl.seed, wl.shop, 0, gens, n_threads=threads)
    dt = time.perf_counter() - t0
    decodes = (1 + gens) * wl.ga.pop
    sample = W.random_population(wl.seed + 1, 1024, wl.initial.n_active)
    t1 = time.perf_counter()
    oracle.decode_pop(wl.initial, sample, n_threads=1)
    dt1 = time.perf_counter() - t1
    rate = decodes / dt
    full = (1 + len(wl.arrivals)) * ((1 + wl.generations) * wl.ga.pop + 1)
    return {"value": rate, "unit": "decodes/s", "cores": threads, "kind": "oracle",
            "sample": f"event 0 only (200 jobs; later events have up to 385 and decode slower, so "
                      f"this rate is optimistic for the whole run): init + {gens} generations of "
                      f"{wl.ga.pop} individuals ({decodes} decodes, {dt:.1f} s)",
            "extrapolated_full_run_s": full / rate,
            "extrapolated_note": f"{full} decodes of the 11 events at the event-0 rate",
            "single_thread": {"value": len(sample) / dt1, "unit": "decodes/s", "cores": 1,
                              "sample": f"event 0, {len(sample)} random priority vectors "
                                        f"({dt1:.1f} s)"},
            "nproc": os.cpu_count(), "cpu_model": cpu_model()}


def cpu_model():
    try:
        return next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                    if l.startswith("model name"))
    except (OSError, StopIteration):
        return ""


def profile_figures(kname, workload):
    """HBM bytes per decode, VALU issue rate and VALU lane utilisation from the
    rocprofv3 counter runs committed under profiles/, used only when they were
    taken on this very build: (traffic per decode, issue TOP/s, lane utilisation).
    The counter runs launch one wave per decode, so a launch's bytes over its
    waves are the bytes of one decode."""
    from paper_1903_10741_amd import ffsga
    tpath = os.path.join(ROOT, "profiles", f"{kname}_{workload}.traffic.json")
    if not os.path.exists(tpath):
        return None, None, None
    t = json.load(open(tpath))
    if t.get("build_id") != ffsga.ffs_build_id() or not t.get("decodes_per_launch"):
        return None, None, None
    return ((t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]) / t["decodes_per_launch"],
            t.get("valu_issue_tlops"), t.get("valu_lane_utilisation"))


def bench_large(args):
    """The large workload end to end: large-200x10x4-6 (200 jobs, 10 stages, 4-6
    unrelated machines per stage, 10 arrival events of 10-30 jobs; 512 islands x
    8x16 = 65536 individuals, 200 generations per event). One step = one event:
    the GA (init + 200 generations), the executed plan's decode and the
    rescheduling at the next arrival; steps go through the 11 events in order and
    start again at event 0 (whose instance stays resident). The on-chip profile
    of each event is sized from its generation 0 (FFS_LDS_AUTO). Before the timed
    region the autotuner times one wave per chromosome against one wave per
    island on event 0; the GA runs in the faster schedule."""
    import torch
    from paper_1903_10741_amd import autotune, ffsga
    from paper_1903_10741_amd import workloads as W
    from paper_1903_10741_amd.run import EventLoop
    wl = W.config3(args.seed)
    if args.generations is not None:
        wl.generations = args.generations
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    tune = None
    if not args.no_autotune:
        d0 = ffsga.DeviceInstance.from_host(wl.initial)
        cands = [autotune.Candidate(ffsga.FFS_SCHEDULE_CHROMOSOME, 8192, 8 * n_cu, True),
                 autotune.Candidate(ffsga.FFS_SCHEDULE_ISLAND, 8192, 2 * n_cu, True)]
        tune = autotune.tune([d0], [wl.initial], wl.ga, candidates=cands, generations=2,
                             log=progress)
        if tune.best.schedule != ffsga.FFS_SCHEDULE_CHROMOSOME:
            raise SystemExit("the autotuner picked one wave per island for the large workload; "
                             "this benchmark runs the event loop on ga_step (one wave per "
                             "chromosome) and would not measure the tuned schedule")
        del d0
    loop = EventLoop(wl, lds_slots=ffsga.FFS_LDS_AUTO)
    for k in range(args.warmup):
        loop.run_event()
        progress(f"large warm-up step {k + 1} done")
    torch.cuda.synchronize()
    ffsga.timing_enable(True, families=[ffsga.TIMING_GENERATION, ffsga.TIMING_STEP], every=8)
    per_event, events = [], []
    decodes = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ts = time.perf_counter()
        ev = loop.run_event()     # ends synchronised (plan decode status, rescheduling)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        decodes += ev.decodes
        events.append(ev)
        per_event.append({"event": ev.event, "n_active": ev.n_active, "lds_slots": ev.lds_slots,
                          "narrow_lds": ev.narrow_lds, "s": dt, "decodes_per_s": ev.decodes / dt,
                          "decodes_redone_off_chip": ev.overflows})
        progress(f"large step {k + 1}: event {ev.event}, {ev.n_active} jobs, "
                 f"{ev.lds_slots} on-chip slots, {dt:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gen_ms, gen_launches = ffsga.timing_read(ffsga.TIMING_GENERATION)
    step_ms, step_gens = ffsga.timing_read(ffsga.TIMING_STEP)
    ffsga.timing_enable(False)
    work = sum(int(ev.work.item()) for ev in events)
    ga_decodes = sum(ev.decodes - 1 for ev in events)
    work_per_decode = work / max(ga_decodes, 1)
    avg_launch_s = gen_ms / 1e3 / max(gen_launches, 1)
    per_gen_s = step_ms / 1e3 / max(step_gens, 1)
    # as in bench_paper: overlapping island-group launches are set against the
    # time per generation of the whole population
    groups = max(ev.island_groups for ev in events)
    if groups > 1:
        achieved = work_per_decode * wl.ga.pop / per_gen_s / 1e12
    else:
        achieved = work_per_decode * wl.ga.pop / avg_launch_s / 1e12
    traffic, valu_issue, lane_util = profile_figures("ga_generation_kernel", "large-200x10x4-6")
    if traffic is not None:
        traffic *= wl.ga.pop // groups  # HBM bytes per launch
    best = {}
    for ev in events:
        best.setdefault(ev.event, int(ev.best_obj.item()))
    config = {
        "workload": "large-200x10x4-6: 200 jobs, 10 stages, 4-6 unrelated machines per stage, "
                    "10 arrival events of 10-30 jobs; 512 islands x 8x16 = 65536, 200 "
                    "generations per event; one step = one event (GA init + 200 generations + "
                    "executed-plan decode + rescheduling), steps cycling through the 11 events",
        "encoding": "job priority vector",
        "decodes_per_step_mean": decodes / args.steps,
        "events_timed": [ev.event for ev in events],
        "per_event": per_event,
        "best_obj_per_event": [best[e] for e in sorted(best)],
        "on_chip_slots": "sized per event from generation 0's longest schedule (FFS_LDS_AUTO)",
    }
    if tune is not None:
        config["autotuned"] = {"pick": tune.best.__dict__, "table": tune.table}
    out = common(args, "exact chromosome decodes/sec", decodes / elapsed, "decodes/s",
                 elapsed * 1e3 / args.steps, "int32", config)
    out["roofline"] = {
        "bound": "alu",
        "kernel": "ga_generation_kernel (selection, crossover, mutation, decode)",
        "achieved": achieved,
        "peak": VALU_INT32_PEAK_TOPS,
        "unit": "TOP/s int32",
        "frac": achieved / VALU_INT32_PEAK_TOPS,
        "traffic": traffic,
        "valu_issue_frac": (valu_issue / VALU_INT32_PEAK_TOPS) if valu_issue else None,
        "valu_lane_utilisation": lane_util,
        "work_per_decode": work_per_decode,
        "island_groups": groups,
        "decodes_per_launch": wl.ga.pop // groups,
        "avg_launch_us": avg_launch_s * 1e6,
        "generation_us": per_gen_s * 1e6,
        "achieved_from": "generation_us" if groups > 1 else "avg_launch_us",
        "timed_launches": gen_launches,
        "timed_every": 8,
        "build_id": ffsga.ffs_build_id(),
    }
    return out


def bench_serve(args):
    """Rescheduling requests from 512 shops arriving Poisson: each request is one
    arrival event (U{5..10} new jobs) of a shop whose first plan exists, rescheduled
    and then 100 generations of population 1024, continuously batched; latency and
    throughput. The first plans are made beforehand through the same path and not
    counted. With --rates r1,r2,...: a latency-vs-load sweep, the shops split into
    one group per rate (both arrivals of each shop of group k offered at rate k),
    every rate served by the same primed service one after the other."""
    import dataclasses
    import numpy as np
    import torch
    from paper_1903_10741_amd import autotune, ffsga
    from paper_1903_10741_amd import workloads as W
    from paper_1903_10741_amd.serve import Server, poisson_schedule
    n_arrivals = 2
    shops = W.shops(args.seed, args.shops)
    arrs = [W.shop_arrivals(args.seed, k, s, n_arrivals) for k, s in enumerate(shops)]
    gens = args.generations or 100
    dev = [ffsga.DeviceInstance.from_host(s) for s in shops[:64]]
    tune = autotune.tune(dev, shops[:64], W.SERVING_GA, generations=2, log=progress)
    srv = Server(shops, arrs, W.SERVING_GA, generations=gens, n_slots=args.slots,
                 gens_per_tick=args.gens_per_tick, seed=args.seed,
                 tuning={"use_graph": True, "blocks": tune.best.blocks,
                         "lds_slots": tune.best.lds_slots, "schedule": tune.best.schedule,
                         "profile_classes": tune.best.profile_classes})
    progress("first plans")
    first = srv.prime()
    progress(f"first plans done in {first['wall_s']:.1f} s; serving starts")
    rates = [float(x) for x in args.rates.split(",")] if args.rates else [args.rate]
    groups = np.array_split(np.arange(len(shops)), len(rates))
    curve = []
    for k, (rate, grp) in enumerate(zip(rates, groups)):
        n_events = [n_arrivals if s in set(grp.tolist()) else 0 for s in range(len(shops))]
        sched = poisson_schedule(args.seed + k, rate, n_events)
        srv.reset_metrics()
        torch.cuda.synchronize()
        m = srv.run(sched, log=progress)
        progress(f"rate {rate}/s: {m['done']} served, p50 {m['latency_p50_s']:.2f} s, "
                 f"p99 {m['latency_p99_s']:.2f} s, {m['decodes_per_s']:.3g} decodes/s")
        curve.append({"offered_per_s": rate, "shops": len(grp), **m})
    need = 1.03e5 * 200   # decodes per request x the workload's 200 requests/s
    last = curve[-1]
    # roofline of the serving loop's generation kernel: its batch configuration
    # (slots, profile classes, launch shape) run eagerly with HIP events around every
    # batched-generation launch, on the shops' current instances
    rb = ffsga.Batch(dataclasses.replace(srv.cfg, use_graph=False))
    for k in range(rb.cfg.n_slots):
        sh = srv.shops[k % len(srv.shops)]
        rb.set(k, sh.inst, args.seed, sh.sid, sh.event)
    rb.stream.synchronize()
    w0 = int(rb.view(0)["work"].item())   # the batch's work counter (all slots)
    ffsga.timing_enable(True, families=[ffsga.TIMING_BATCH])
    rgens = 10
    rb.step(rgens)
    gen_ms, launches = ffsga.timing_read(ffsga.TIMING_BATCH)
    ffsga.timing_enable(False)
    rb.status()
    work = int(rb.view(0)["work"].item()) - w0
    avg = gen_ms / 1e3 / max(launches, 1)
    achieved = work / max(launches, 1) / avg / 1e12
    out = common(args, "exact chromosome decodes/sec", last["decodes_per_s"], "decodes/s",
                 last["wall_s"] * 1e3, "int32", {
                     "workload": f"serving: {len(shops)} shops, {n_arrivals} arrival requests each "
                                 f"(U{{5..10}} jobs), {gens} generations x pop 1024 per request, "
                                 f"Poisson arrivals at {', '.join(f'{r:g}' for r in rates)}/s" +
                                 (f" (shops split into {len(rates)} groups, one per rate)"
                                  if len(rates) > 1 else ""),
                     "first_plans_s": first["wall_s"],
                     "value_at": f"offered {rates[-1]:g} requests/s",
                     "decodes_per_s_needed_at_200_per_s": need,
                     "capacity_gap": need / max(max(c["decodes_per_s"] for c in curve), 1.0),
                     "autotuned": tune.best.__dict__,
                     "curve": curve})
    out["steps"] = 1
    out["warmup"] = 0
    out["roofline"] = {"bound": "alu", "kernel": f"batch_generation_kernel (serving batch: "
                                                 f"{rb.cfg.n_slots} slots x {rb.pop})",
                       "achieved": achieved, "peak": VALU_INT32_PEAK_TOPS, "unit": "TOP/s int32",
                       "frac": achieved / VALU_INT32_PEAK_TOPS, "traffic": None,
                       "avg_launch_us": avg * 1e6, "launches": launches,
                       "work_per_decode": work / max(rb.cfg.n_slots * rb.pop * rgens, 1),
                       "build_id": ffsga.ffs_build_id()}
    return out


def bench_rs_ratio(args):
    """Section 5.3, Table 10: complete rescheduling (the method) against the
    traditional static approach as the rescheduling point moves through the
    original schedule. For each ratio r and each Table 5-shaped instance (10 jobs,
    3 stages of 2 machines, power peak 4, WT = 100): the GA (64 islands of 8x8 =
    4096, 100 generations) plans event 0, RS = round(r x that plan's makespan)
    and round(r x 10) jobs arrive at RS; event 1 is then planned both ways by
    the same GA (same seed) and the best objectives compared. Improvement ratio
    = mean static objective / mean complete-rescheduling objective."""
    import numpy as np
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    import dataclasses
    gens = args.generations or 100
    xy = args.encoding == "xy"
    ga = dataclasses.replace(W.TABLE5_GA, encoding=1 if xy else 0)
    cfg = ffsga.GaConfig.of(ga)
    paper = {0.2: (2727.61, 1195.29, 2.28), 0.4: (5608.31, 3745.06, 1.50),
             0.6: (5464.86, 4673.57, 1.17), 0.8: (4805.43, 4755.91, 1.01)}
    rows = []
    t0 = time.perf_counter()
    decodes = 0
    for r in (0.2, 0.4, 0.6, 0.8):
        st_obj, dy_obj = [], []
        for sd in range(args.seed, args.seed + args.instances):
            inst = W.table5_instance(sd)
            d0 = ffsga.DeviceInstance.from_host(inst)
            g0 = ffsga.GA(d0, cfg, sd, 0, 0)
            g0.step(gens)
            prio, _ = g0.best()
            plan = ffsga.ffs_decode(d0, prio.view(1, -1), want_schedule=True, xy=xy)
            ps, pm = plan["start"][0], plan["mach"][0]
            p_np = np.asarray(inst.proc)
            s_np, m_np = ps.cpu().numpy(), pm.cpu().numpy()
            span = max(int(s_np[j, s]) + int(p_np[j, s, m_np[j, s]])
                       for j in range(inst.n_jobs) for s in range(inst.n_stages))
            rs = max(1, int(round(r * span)))
            arr = W.table5_arrival(1000 + sd, inst, rs, max(1, int(round(r * inst.n_jobs))))
            out = []
            for static in (True, False):
                d1 = ffsga.reschedule(d0, ps, pm, arr, static=static)
                g1 = ffsga.GA(d1, cfg, sd, 0, 1)
                g1.step(gens)
                out.append(int(g1.best()[1].item()))
            st_obj.append(out[0])
            dy_obj.append(out[1])
            decodes += 3 * (1 + gens) * ga.pop + 1
        ms, md = float(np.mean(st_obj)), float(np.mean(dy_obj))
        row = {"ratio": r, "instances": len(st_obj), "static_mean_obj": ms,
               "rescheduling_mean_obj": md, "improvement_ratio": ms / md,
               "instances_static_worse": int(sum(a > b for a, b in zip(st_obj, dy_obj))),
               "instances_equal": int(sum(a == b for a, b in zip(st_obj, dy_obj))),
               "paper": {"static": paper[r][0], "rescheduling": paper[r][1],
                         "improvement_ratio": paper[r][2], "hardware": "Tesla K40 (their own "
                         "random Table 5 instances, not these)"}}
        progress(f"ratio {r}: static {ms:.1f}, rescheduling {md:.1f}, improvement {ms / md:.2f}")
        rows.append(row)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    out = common(args, "improvement ratio of complete rescheduling over the static approach",
                 float(np.mean([x["improvement_ratio"] for x in rows])),
                 "x (mean static objective / mean rescheduling objective, averaged over ratios)",
                 elapsed * 1e3, "int32", {
                     "workload": f"Table 5-shaped instances {args.seed}-"
                                 f"{args.seed + args.instances - 1} (10 jobs, 3 stages x 2 machines, "
                                 f"Q_max 4, WT 100); GA 64 islands x 8x8, {gens} generations per "
                                 f"event; arrivals of round(r x 10) jobs at RS = r x makespan; "
                                 f"{'X/Y chromosomes' if xy else 'job-priority vectors'}",
                     "encoding": "xy" if xy else "job priority vector",
                     "decodes": decodes, "table": rows})
    out["steps"] = 1
    out["warmup"] = 0
    return out


def bench_schemes(args):
    """Section 5.2, Tables 8-9: the hybrid GA (8x8 islands, ring migration) against
    the classical GA (roulette wheel on eq. (13), random pairing) and the cellular
    GA (neighbourhood parents, replace if better), all on the GPU, at populations
    64x64, 128x128 and 256x256, 100 generations from the same seed, on two
    instance families: Table 5-shaped (10 jobs, 3 stages of 2 machines, power peak
    4, WT = 100: the paper's test 2 size) and paper-50x5x3 event 0 (50 jobs).
    Per scheme: best objective (mean and best over the instances) and wall time
    per 100 generations (init included)."""
    import numpy as np
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    gens = args.generations or 100
    paper_s = {64: (8.77, 8.14, 129.16), 128: (30.71, 31.13, 554.01), 256: (105.73, 108.07, 2651.61)}
    families = (("table5-10x3x2", W.table5_instance), ("paper-50x5x3", lambda sd: W.config2(sd).initial))
    rows = []
    for fam, make in families:
        for side in (64, 128, 256):
            per = {}
            for name, scheme, gp in (("hybrid", ffsga.FFS_GA_HYBRID,
                                      W.GaParams(side * side // 64, 8, 8)),
                                     ("classical", ffsga.FFS_GA_CLASSICAL, W.GaParams(1, side, side)),
                                     ("cellular", ffsga.FFS_GA_CELLULAR, W.GaParams(1, side, side))):
                cfg = ffsga.GaConfig.of(gp, scheme=scheme)
                objs, times = [], []
                for sd in range(args.seed, args.seed + args.instances):
                    d = ffsga.DeviceInstance.from_host(make(sd))
                    if sd == args.seed:   # warm-up of this launch shape
                        ffsga.GA(d, cfg, sd, 0, 0).step(2)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    g = ffsga.GA(d, cfg, sd, 0, 0)
                    g.step(gens)
                    best = int(g.best()[1].item())
                    times.append(time.perf_counter() - t0)
                    objs.append(best)
                per[name] = {"mean_best_obj": float(np.mean(objs)), "best_obj": int(min(objs)),
                             "s_per_100_generations": float(np.mean(times)) * 100 / gens,
                             "decodes_per_s": (1 + gens) * gp.pop / float(np.mean(times))}
                progress(f"{fam} {side}x{side} {name}: mean best {np.mean(objs):.1f}, "
                         f"{np.mean(times) * 1e3:.1f} ms per run")
            rows.append({"instances": fam, "population": f"{side}x{side}", **per,
                         "paper_k40_s_per_100_generations": {
                             "hybrid": paper_s[side][0], "cellular": paper_s[side][1],
                             "classical_1_cpu_core": paper_s[side][2],
                             "note": "the paper's own small instances (10 jobs, 3 stages x 2 "
                                     "machines), K40 and Xeon E5640"}})
    out = common(args, "wall time per 100 generations, hybrid vs classical vs cellular GA",
                 rows[0]["hybrid"]["s_per_100_generations"], "s (hybrid GA, 64x64, Table 5-shaped)",
                 sum(r[k]["s_per_100_generations"] for r in rows
                     for k in ("hybrid", "classical", "cellular")) * 1e3, "int32", {
                     "workload": f"instances {args.seed}-{args.seed + args.instances - 1} of each "
                                 f"family, {gens} generations per run, job-priority vectors",
                     "table": rows})
    out["higher_is_better"] = False
    out["steps"] = 1
    out["warmup"] = 0
    return out


def spearman(a, b):
    import numpy as np
    ra = np.argsort(np.argsort(a))
    rb = np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


def populations(d, ga_cfg, seed, snap_gens):
    """Decoder-labelled chromosomes: the populations of one plain GA run at the given
    generations (0 = the initial population), with their exact objectives."""
    import torch
    from paper_1903_10741_amd import ffsga
    g = ffsga.GA(d, ga_cfg, seed, 0, 0)
    prios, objs, done = [], [], 0
    for k in snap_gens:
        if k > done:
            g.step(k - done)
            done = k
        v = g.view()
        prios.append(v["prio"].clone())
        objs.append(v["obj"].clone())
    return torch.cat(prios), torch.cat(objs)


def sg_train(model, data, gen, batch=4096, epochs=2, lr=1e-3):
    """Adam on decoder-labelled chromosomes: `epochs` passes worth of batches, each
    batch drawn from one instance's pairs (instance and rows from `gen`)."""
    import numpy as np
    import torch
    n_pairs = sum(int(x[1].shape[0]) for x in data)
    steps = epochs * n_pairs // batch
    losses = []
    for _ in range(steps):
        i = int(torch.randint(len(data), (1,), generator=gen))
        feats, prio, tgt = data[i]
        idx = torch.randint(prio.shape[0], (batch,), generator=gen).cuda()
        losses.append(model.train_step(feats, prio[idx], tgt[idx], lr)[0])
    torch.cuda.synchronize()
    losses = [float(x.item()) for x in losses]
    return steps, losses[0], float(np.mean(losses[-50:]))


def sg_race(model, d, cfg, table, seed, screened, gens):
    """One GA run from `seed`, best elite read every 10 generations:
    [(generations, seconds, best objective)]."""
    import torch
    from paper_1903_10741_amd import ffsga
    g = ffsga.GA(d, cfg, seed, 0, 0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    trace, done = [], 0
    while done < gens:
        k = min(10, gens - done)
        if screened:
            g.step_screened(model, table, 4, k)
        else:
            g.step(k)
        done += k
        trace.append((done, time.perf_counter() - t0, int(g.view()["elite_obj"].min().item())))
    g.status()
    return trace


def sg_first(trace, target, offset=0.0):
    """(generations, seconds + offset) at which a trace first reaches target."""
    return next(((gn, t + offset) for gn, t, b in trace if b <= target), (None, None))


def sg_evaluate(model, d, cfg, sd, plain, gens, tag, offset_s=0.0):
    """Race the screened GA against a plain trace on one instance; held-out rank
    correlation of the network's scores on two populations of another run.
    offset_s: time charged to the screened run before it starts (data and training
    of a network made for this very instance)."""
    import numpy as np
    pop = cfg.islands * cfg.rows * cfg.cols
    table = model.score_table(model.features(d), d.n_active)
    hp, ho = populations(d, cfg, 7777 + sd, (0, 20))
    ys = model.score(table, hp).cpu().numpy()
    ho = ho.cpu().numpy()
    rho = [spearman(ys[k * pop:(k + 1) * pop], ho[k * pop:(k + 1) * pop]) for k in (0, 1)]
    scr = sg_race(model, d, cfg, table, sd, True, gens)
    target = plain[-1][2]
    gp, tp = sg_first(plain, target)
    gs, ts = sg_first(scr, target, offset_s)
    progress(f"{tag} instance {sd}: plain {target} at gen {gp}, screened {scr[-1][2]}, "
             f"reached at gen {gs}, rank correlation {rho[0]:.2f}/{rho[1]:.2f}")
    return {"instance_seed": sd, "plain_final": target, "screened_final": scr[-1][2],
            "plain_gens_to_target": gp, "plain_s_to_target": tp,
            "screened_gens_to_target": gs, "screened_s_to_target": ts,
            "speedup": (tp / ts) if ts else None, "heldout_spearman_gen0_20": rho,
            "plain_s_per_gen": plain[-1][1] / plain[-1][0],
            "screened_s_per_gen": scr[-1][1] / scr[-1][0]}


def sg_summary(rows):
    import numpy as np
    sp = [r["speedup"] if r["speedup"] is not None else 0.0 for r in rows]
    rho = np.array([r["heldout_spearman_gen0_20"] for r in rows])
    return {"median_speedup": float(np.median(sp)), "runs": len(rows),
            "reached": sum(r["screened_s_to_target"] is not None for r in rows),
            "screened_better_final": sum(r["screened_final"] < r["plain_final"] for r in rows),
            "heldout_spearman_median_gen0": float(np.median(rho[:, 0])),
            "heldout_spearman_median_gen20": float(np.median(rho[:, 1])),
            "per_instance": rows}


def surrogate_cross(args, n_train, race_seeds, gens):
    """Time to equal fitness by the cross-instance protocol: one network trained on
    the populations (generations 0, 10, 20, 40, 80 of one plain run each) of
    paper-shaped event-0 instances of seeds 100..100+n_train-1, then raced on the
    unseen instances of seeds args.seed..: plain GA and screened GA (4 candidates
    per cell) from the same GA seed; speedup = plain's time to its own final
    objective / screened's time to reach it (0 if never). Data and training are
    made once for every instance to come, so they are reported apart (amortised)."""
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    cfg = ffsga.GaConfig.of(W.config2(0).ga)
    pop = cfg.islands * cfg.rows * cfg.cols
    model = ffsga.Surrogate(W.surrogate_init(args.seed))
    gen = torch.Generator(device="cpu").manual_seed(args.seed)
    t0 = time.perf_counter()
    data = []
    for sd in range(100, 100 + n_train):
        d = ffsga.DeviceInstance.from_host(W.config2(sd).initial)
        prio, obj = populations(d, cfg, sd, (0, 10, 20, 40, 80))
        data.append((model.features(d), prio, model.targets(obj, pop)))
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    pairs = sum(int(x[1].shape[0]) for x in data)
    t1 = time.perf_counter()
    fit = sg_train(model, data, gen)
    t_train = time.perf_counter() - t1
    del data
    progress(f"cross-instance network: {pairs} pairs, {fit[0]} steps, loss {fit[1]:.3f} -> "
             f"{fit[2]:.3f}, data {t_data:.1f} s, training {t_train:.1f} s")
    rows = []
    for k, sd in enumerate(range(args.seed, args.seed + race_seeds)):
        d = ffsga.DeviceInstance.from_host(W.config2(sd).initial)
        if k == 0:   # warm-up of both paths
            table = model.score_table(model.features(d), d.n_active)
            sg_race(model, d, cfg, None, sd, False, 20)
            sg_race(model, d, cfg, table, sd, True, 20)
        plain = sg_race(model, d, cfg, None, sd, False, gens)
        rows.append(sg_evaluate(model, d, cfg, sd, plain, gens, "cross-instance network"))
    out = sg_summary(rows)
    out.update({"protocol": f"one network trained on instances {100}-{99 + n_train} "
                            f"(generations 0, 10, 20, 40, 80 of one plain run each), raced on "
                            f"unseen instances {args.seed}-{args.seed + race_seeds - 1}; data and "
                            f"training amortised over every instance to come, reported apart",
                "train_pairs": pairs, "train_steps": fit[0], "loss_first": fit[1],
                "loss_last50": fit[2], "data_s": t_data, "train_s": t_train})
    return out


def bench_surrogate(args):
    """Time to reach the plain GA's final fitness, screened GA (4 candidates per cell,
    the lowest surrogate score kept) against the plain GA, on paper-shaped event-0
    instances of seeds 0..race_seeds-1, same GA seed, 500 generations each.

    The value is the median speedup of one network trained across instances
    (seeds 100-199) and raced on the unseen ones (surrogate_cross). Beside it,
    per instance, --train-seeds networks trained on that instance itself (the
    populations of 16 seeded plain-GA runs at generations 0-30, or 0, 10, ...,
    300 with --train-snapshots spread; 2.03 M pairs, 2 epochs of Adam; network k
    from initial weights of seed k and its own batch-order generator): such a
    network serves one instance only, so its data generation and training count
    in its time to the target."""
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    gens = args.generations or W.config2(0).generations
    cross = surrogate_cross(args, args.train_instances, args.race_seeds, gens)
    cfg = ffsga.GaConfig.of(W.config2(0).ga)
    pop = cfg.islands * cfg.rows * cfg.cols
    own_rows, prep = [], []
    for sd in range(args.seed, args.seed + (args.race_seeds if args.train_seeds > 0 else 0)):
        d = ffsga.DeviceInstance.from_host(W.config2(sd).initial)
        plain = sg_race(None, d, cfg, None, sd, False, gens)
        for k in range(args.train_seeds):
            t0 = time.perf_counter()
            model = ffsga.Surrogate(W.surrogate_init(k))
            feats = model.features(d)
            data = []
            snaps = tuple(range(31)) if args.train_snapshots == "early" else tuple(range(0, 301, 10))
            for rs in range(1000, 1016):
                prio, obj = populations(d, cfg, rs, snaps)
                data.append((feats, prio, model.targets(obj, pop)))
            torch.cuda.synchronize()
            t_data = time.perf_counter() - t0
            t1 = time.perf_counter()
            fit = sg_train(model, data, torch.Generator(device="cpu").manual_seed(1_000_003 * sd + k))
            t_train = time.perf_counter() - t1
            del data
            prep.append({"instance_seed": sd, "train_seed": k, "data_s": t_data,
                         "train_s": t_train, "steps": fit[0], "loss_first": fit[1],
                         "loss_last50": fit[2]})
            row = sg_evaluate(model, d, cfg, sd, plain, gens, f"own-instance network {k}",
                              offset_s=t_data + t_train)
            row["train_seed"] = k
            own_rows.append(row)
    out = common(args, "time-to-equal-fitness, surrogate vs plain GA", cross["median_speedup"],
                 "x (plain GA time / screened GA time to the plain GA's final objective)",
                 sum(r["screened_s_per_gen"] for r in cross["per_instance"]) * gens * 1e3
                 / max(len(cross["per_instance"]), 1),
                 "bf16/fp32 surrogate, int32 decode", {
                     "workload": "paper-shaped event 0 (50 jobs, 5 stages, 3 machines), 32 islands "
                                 f"x 8x16, {gens} generations, screened: 4 candidates per cell; "
                                 f"raced on instances {args.seed}-{args.seed + args.race_seeds - 1}; "
                                 "value: median over them of the speedup of the cross-instance "
                                 "network (0 where the screened run never reaches the target)",
                     "cross_instance": cross})
    if own_rows:
        out["config"]["own_instance"] = {**sg_summary(own_rows), "training": prep,
                                         "train_snapshots": args.train_snapshots,
                                         "note": "data generation and training of each network "
                                                 "are inside its time to the target"}
    out["steps"] = 1
    out["warmup"] = 1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large",
                    choices=["large", "paper", "batch", "serve", "surrogate", "rs-ratio",
                             "schemes", "peaks"],
                    help="large (default): the large-200x10x4-6 event loop, one event per step, "
                         "with the paper-shaped workload measured beside it")
    ap.add_argument("--lds-slots", type=int, default=0)
    ap.add_argument("--rules", type=int, default=0, choices=[0, 1, 2, 3],
                    help="paper workload: job-vector decode variants, bit 0 FIFO stage order, "
                         "bit 1 power-aware machine choice")
    ap.add_argument("--encoding", default="job", choices=["job", "xy"],
                    help="paper workload: one priority per job (default) or the paper's X/Y "
                         "machine and priority matrices")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-paper", action="store_true",
                    help="large workload: skip the paper-shaped measurement beside it")
    ap.add_argument("--paper-steps", type=int, default=2)
    ap.add_argument("--no-surrogate", action="store_true",
                    help="large workload: skip the surrogate's time-to-equal-fitness beside it")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--generations", type=int, default=None,
                    help="override generations per event (profiling runs only)")
    ap.add_argument("--shops", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--rates", default=None,
                    help="serve: comma-separated offered request rates for a latency-vs-load sweep")
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--gens-per-tick", type=int, default=10)
    ap.add_argument("--race-seeds", type=int, default=10)
    ap.add_argument("--instances", type=int, default=20,
                    help="rs-ratio, schemes: Table 5-shaped instances per point")
    ap.add_argument("--train-instances", type=int, default=100)
    ap.add_argument("--train-seeds", type=int, default=3,
                    help="surrogate: own-instance networks per instance (initial weights and "
                         "batch order from seed k)")
    ap.add_argument("--train-snapshots", default="early", choices=["early", "spread"],
                    help="surrogate: train on generations 0-30 (early) or 0, 10, ..., 300 (spread) "
                         "of each seeded run")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch: the usual tuned configuration (8192 profile slots in 3 classes, "
                         "8 blocks per CU, one wave per child, graph) without tuning; large: "
                         "skip the schedule comparison")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 256 MiB device copy, the reference for HBM byte counters")
    ap.add_argument("--island-groups", type=int, default=0,
                    help="island groups ga_step runs on streams of their own (0: the library's "
                         "default of 4; 1: one stream)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the hot path is built and "
              f"measured on one GPU; sharding it across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    from paper_1903_10741_amd import ffsga
    ffsga.set_island_groups(args.island_groups)
    copy_calibration(args)
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(bench_surrogate(args)), flush=True)
        return
    if args.workload == "rs-ratio":
        print(json.dumps(bench_rs_ratio(args)), flush=True)
        return
    if args.workload == "schemes":
        print(json.dumps(bench_schemes(args)), flush=True)
        return
    if args.workload == "peaks":
        pk = measure_peaks()
        print(json.dumps(common(args, "measured int32 VALU rate", pk["valu_int32_tops"],
                                "T lane-ops/s", None, "int32",
                                {"workload": "device peaks: int32 vector adds, bf16 matrix-core "
                                             "products, device-to-device copy", **pk})), flush=True)
        return
    if args.workload == "paper":
        out = bench_paper(args, args.steps, args.warmup)
        if not args.no_cpu_baseline:
            from paper_1903_10741_amd import workloads as W
            out["cpu_baseline"] = cpu_baseline(W.config2(args.seed))
        print(json.dumps(out), flush=True)
        return
    out = bench_large(args)
    if not args.no_paper:
        progress("paper-shaped workload")
        paper = bench_paper(args, args.paper_steps, 1)
        if not args.no_cpu_baseline:
            from paper_1903_10741_amd import workloads as W
            paper["cpu_baseline"] = cpu_baseline(W.config2(args.seed))
        out["paper_shaped"] = {k: paper[k] for k in ("value", "unit", "steps", "warmup",
                                                     "ms_per_step", "config", "roofline",
                                                     "cpu_baseline") if k in paper}
    if not args.no_surrogate:
        progress("surrogate: time to equal fitness (cross-instance network)")
        sg = surrogate_cross(args, args.train_instances, args.race_seeds, 500)
        out["surrogate_time_to_equal_fitness"] = {
            "metric": "time-to-equal-fitness, surrogate vs plain GA",
            "value": sg["median_speedup"],
            "unit": "x (plain GA time / screened GA time to the plain GA's final objective; "
                    "0 where never reached)",
            **{k: v for k, v in sg.items() if k != "per_instance"},
            "per_instance": [{k: r[k] for k in ("instance_seed", "speedup",
                                                  "plain_gens_to_target",
                                                  "screened_gens_to_target",
                                                  "heldout_spearman_gen0_20")}
                             for r in sg["per_instance"]]}
    if not args.no_cpu_baseline:
        from paper_1903_10741_amd import workloads as W
        progress("CPU oracle (large workload, event 0)")
        out["cpu_baseline"] = oracle_rate_large(W.config3(args.seed))
        progress("device peaks")
        out["measured_peaks"] = measure_peaks()
    print(json.dumps(out), flush=True)


def measure_peaks():
    """The rates the rooflines divide by, measured on this GPU: int32 vector adds
    (8 independent chains per lane, 1-32 blocks of 4 waves per CU), bf16
    matrix-core products (v_mfma_f32_32x32x16_bf16, 4 independent accumulators per
    wave, 1-16 blocks per CU) and a 2 GiB device-to-device copy (read + write
    bytes). The best rate of each sweep is reported beside the sweep."""
    import torch
    from paper_1903_10741_amd import peaks
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    peaks.ffs_peak_valu_int32(8 * n_cu, 64)
    valu = [(k, peaks.ffs_peak_valu_int32(k * n_cu, 1000)[1] / 1e12) for k in (1, 2, 4, 8, 16, 32)]
    peaks.ffs_peak_mfma_bf16(4 * n_cu, 8)
    mfma = [(k, peaks.ffs_peak_mfma_bf16(k * n_cu, 200)[1] / 1e12) for k in (1, 2, 4, 8, 16)]
    n = 1 << 29
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    copy_s = e0.elapsed_time(e1) / 1e3 / 5
    del src, dst
    hbm = 2 * n * 4 / copy_s / 1e9
    v_best, m_best = max(r for _, r in valu), max(r for _, r in mfma)
    return {"valu_int32_tops": v_best, "valu_frac_of_peak": v_best / VALU_INT32_PEAK_TOPS,
            "valu_by_blocks_per_cu": {str(k): r for k, r in valu},
            "mfma_bf16_tflops": m_best, "mfma_frac_of_2500": m_best / 2500.0,
            "mfma_by_blocks_per_cu": {str(k): r for k, r in mfma},
            "hbm_copy_gbs": hbm, "hbm_frac_of_8000": hbm / HBM_PEAK_GBS,
            "compute_units": n_cu}


def copy_calibration(args):
    """A 256 MiB device-to-device copy: the reference the HBM byte counters of a
    profiling run are scaled by."""
    if not args.copy_calibration:
        return
    import torch
    src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def bench_paper(args, steps, warmup):
    """The paper-shaped workload end to end: one step = every event of paper-50x5x3
    (the GA's init + 500 generations, the executed plan's decode and the
    rescheduling, for each of the 6 events)."""
    import dataclasses
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    from paper_1903_10741_amd.run import run_workload

    wl = W.config2(args.seed)
    if args.generations is not None:
        wl.generations = args.generations
    xy = args.encoding == "xy"
    if xy:
        wl.ga = dataclasses.replace(wl.ga, encoding=1)
    if args.rules:
        wl.initial = dataclasses.replace(wl.initial, decode_rules=args.rules)

    for _ in range(warmup):
        run_workload(wl, lds_slots=args.lds_slots)
    torch.cuda.synchronize()

    # events on the generation kernel only, one launch in 8 (spread evenly over
    # the timed steps): the other launches carry no markers; and on the caller's
    # stream around each ga_step call (the time per generation of the whole
    # population, which island groups' overlapping launches do not show)
    ffsga.timing_enable(True, families=[ffsga.TIMING_GENERATION, ffsga.TIMING_STEP], every=8)
    decodes = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        res = run_workload(wl, lds_slots=args.lds_slots, sync_results=False)
        decodes += res.decodes
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gen_ms, gen_launches = ffsga.timing_read(ffsga.TIMING_GENERATION)
    step_ms, step_gens = ffsga.timing_read(ffsga.TIMING_STEP)
    ffsga.timing_enable(False)
    groups = max(e.island_groups for e in res.events)
    best = [int(e.best_obj.item()) for e in res.events]
    # algorithmic work of the generation kernel, counted by the decoder (the last
    # timed step's own counters: every step computes the same)
    work_per_decode = sum(int(e.work.item()) for e in res.events) / max(res.ga_decodes, 1)

    kname = "ga_generation_xy_kernel" if xy else "ga_generation_kernel"
    traffic, valu_issue, lane_util = profile_figures(kname, "paper-50x5x3")
    if traffic is not None:
        traffic *= wl.ga.pop // groups  # HBM bytes per launch
    avg_launch_s = gen_ms / 1e3 / max(gen_launches, 1)
    per_gen_s = step_ms / 1e3 / max(step_gens, 1)
    # One launch decodes pop / groups chromosomes. With one group the launch's
    # own duration is the time of its work; with several, the groups' launches
    # run side by side, so the population's work is set against the time per
    # generation of the whole ga_step (replacement and migration included: a
    # lower bound on the kernels' own rate).
    if groups > 1:
        achieved = work_per_decode * wl.ga.pop / per_gen_s / 1e12
    else:
        achieved = work_per_decode * wl.ga.pop / avg_launch_s / 1e12
    out = common(args, "exact chromosome decodes/sec", decodes / elapsed, "decodes/s",
                 elapsed * 1e3 / steps, "int32", {
                     "workload": "paper-shaped plain GA: 50 jobs, 5 stages, 3 unrelated machines, "
                                 "5 arrival events, 32 islands x 8x16 = 4096, 500 "
                                 "generations/event; one step = all 6 events" +
                                 (", X/Y chromosome (machine and priority per operation)"
                                  if xy else ""),
                     "encoding": "xy" if xy else "job priority vector",
                     "decode_rules": args.rules,
                     "decodes_per_step": decodes // steps,
                     "events": 1 + len(wl.arrivals),
                     "best_obj_per_event": best})
    out["steps"], out["warmup"] = steps, warmup
    out["roofline"] = {
        "bound": "alu",
        "kernel": f"{kname} (selection, crossover, mutation, decode)",
        "achieved": achieved,
        "peak": VALU_INT32_PEAK_TOPS,
        "unit": "TOP/s int32",
        "frac": achieved / VALU_INT32_PEAK_TOPS,
        "traffic": traffic,
        "valu_issue_frac": (valu_issue / VALU_INT32_PEAK_TOPS) if valu_issue else None,
        "valu_lane_utilisation": lane_util,
        "work_per_decode": work_per_decode,
        "island_groups": groups,
        "decodes_per_launch": wl.ga.pop // groups,
        "avg_launch_us": avg_launch_s * 1e6,
        "generation_us": per_gen_s * 1e6,
        "achieved_from": "generation_us" if groups > 1 else "avg_launch_us",
        "timed_launches": gen_launches,
        "timed_every": 8,
        "build_id": ffsga.ffs_build_id(),
    }
    return out


if __name__ == "__main__":
    main()
