"""Benchmark: exact chromosome decodes per second of the whole EDFFS hot path on one GPU.

One step = one complete predictive-reactive run of the paper-shaped workload
(50 jobs, 5 stages, 3 unrelated machines per stage, 5 arrival events; the
island GA with 32 islands of 8x16 = 4096 individuals, 500 generations per
event, 2 best migrating every 10 generations): for each of the 6 events the
GA (init + 500 generations of selection, crossover, mutation, decode,
replacement, migration), the decode of the executed plan, and the
rescheduling at the next arrival. Inputs are synthetic and seeded, resident
on the GPU before the timed region starts.

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

# 256 CUs x 64 int32 lanes per clock x 2.4 GHz
VALU_INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
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
    model = ""
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo")
                     if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": decodes / dt, "unit": "decodes/s", "cores": threads, "kind": "oracle",
            "sample": f"one full step: {len(out)} events x (1 + {wl.generations}) generations x "
                      f"{wl.ga.pop} individuals + plan decodes ({decodes} decodes, {dt:.1f} s)",
            "single_thread": {"value": 5 * wl.ga.pop / dt1, "unit": "decodes/s", "cores": 1,
                              "sample": f"event 0, generation 0 + 4 generations ({5 * wl.ga.pop} "
                                        f"decodes, {dt1:.1f} s)"},
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


def bench_large(args):
    """Large decode throughput: event 0 of large-200x10x4-6 (200 jobs, 10 stages, 4-6
    unrelated machines, population 65536 = 512 islands x 8x16) for 200 generations in
    the batched launch, one slot; the autotuner times one wave per child against one
    wave per island (and the on-chip profile sizes) and the step runs the faster."""
    import torch
    from paper_1903_10741_amd import autotune, ffsga
    from paper_1903_10741_amd import workloads as W
    wl = W.config3(args.seed)
    gens = args.generations or wl.generations
    inst = wl.initial
    dev = [ffsga.DeviceInstance.from_host(inst)]
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    cands = []
    for lds in (8192, 16384):
        for sched, blocks in ((ffsga.FFS_SCHEDULE_CHROMOSOME, 8 * n_cu),
                              (ffsga.FFS_SCHEDULE_CHROMOSOME, 16 * n_cu),
                              (ffsga.FFS_SCHEDULE_ISLAND, 2 * n_cu),
                              (ffsga.FFS_SCHEDULE_ISLAND, 4 * n_cu)):
            cands.append(autotune.Candidate(sched, lds, blocks, True))
    tune = autotune.tune(dev, [inst], wl.ga, candidates=cands, generations=2, log=progress)
    b = ffsga.Batch(autotune.batch_config([inst], wl.ga, dev[0].horizon, tune.best))

    def one_step():
        b.set(0, dev[0], args.seed, 0, 0)
        b.step(gens)
    for _ in range(args.warmup):
        one_step()
    b.status()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step()
        b.stream.synchronize()
        progress(f"large step {k + 1} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    b.status()
    decodes = wl.ga.pop * (1 + gens)
    best = {s: min(r["us_per_generation"] for r in tune.table if r["schedule"] == s)
            for s in (ffsga.FFS_SCHEDULE_CHROMOSOME, ffsga.FFS_SCHEDULE_ISLAND)}
    out = common(args, "exact chromosome decodes/sec", decodes * args.steps / elapsed, "decodes/s",
                 elapsed * 1e3 / args.steps, "int32", {
                     "workload": f"large-200x10x4-6 event 0: 200 jobs, 10 stages, 4-6 unrelated "
                                 f"machines, 512 islands x 8x16 = 65536, {gens} generations",
                     "decodes_per_step": decodes, "autotuned": tune.best.__dict__,
                     "us_per_generation_wave_per_child": best[ffsga.FFS_SCHEDULE_CHROMOSOME],
                     "us_per_generation_wave_per_island": best[ffsga.FFS_SCHEDULE_ISLAND],
                     "tuning_table": tune.table})
    return out


def bench_serve(args):
    """Rescheduling requests from 512 shops arriving Poisson at 200/s: each request
    is one arrival event (U{5..10} new jobs) of a shop whose first plan exists,
    rescheduled and then 100 generations of population 1024, continuously
    batched; latency and throughput. The first plans are made beforehand through
    the same path and not counted."""
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
    sched = poisson_schedule(args.seed, args.rate, [n_arrivals] * len(shops))
    torch.cuda.synchronize()
    m = srv.run(sched, log=progress)
    out = common(args, "exact chromosome decodes/sec", m["decodes_per_s"], "decodes/s",
                 m["wall_s"] * 1e3, "int32", {
                     "workload": f"serving: {len(shops)} shops, {n_arrivals} arrival requests each "
                                 f"(U{{5..10}} jobs), Poisson {args.rate}/s, {gens} generations x "
                                 f"pop 1024 per request",
                     "first_plans_s": first["wall_s"],
                     **{k: v for k, v in m.items()}})
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


def bench_surrogate(args):
    """Time to reach the plain GA's final fitness, screened GA (4 candidates per cell,
    the lowest surrogate score kept) against the plain GA, on paper-shaped event-0
    instances of seeds 0..race_seeds-1, same GA seed, 500 generations each; per
    instance the speedup is the plain GA's time to reach its own final objective
    over the screened GA's time to reach it, and the value is the median.

    Per instance (the value): --train-seeds networks are trained on 2.03 M
    decoder-labelled chromosomes of that instance (the populations of 16 seeded
    plain-GA runs at generations 0-30, or 0, 10, ..., 300 with --train-snapshots
    spread), 2 epochs of Adam, network k from initial weights of seed k and its own
    batch-order generator (seeded by instance and k, so no run depends on another);
    each races the plain GA and the value is the median speedup over every
    (instance, network) pair. Data and training time are reported apart. Across
    instances (reported beside it): one network trained on instances of seeds
    100-199 (generations 0, 10, 20, 40, 80 of one run each, 2.05 M chromosomes) and
    raced on the same unseen instances."""
    import numpy as np
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    base = W.config2(0)
    gens = args.generations or base.generations
    cfg = ffsga.GaConfig.of(base.ga)
    pop = base.ga.pop
    B = 4096

    def train(model, data, gen):
        n_pairs = sum(int(x[1].shape[0]) for x in data)
        steps = 2 * n_pairs // B
        losses = []
        for _ in range(steps):
            i = int(torch.randint(len(data), (1,), generator=gen))
            feats, prio, tgt = data[i]
            idx = torch.randint(prio.shape[0], (B,), generator=gen).cuda()
            losses.append(model.train_step(feats, prio[idx], tgt[idx], 1e-3)[0])
        torch.cuda.synchronize()
        losses = [float(x.item()) for x in losses]
        return steps, losses[0], float(np.mean(losses[-50:]))

    def race(model, d, table, seed, screened):
        g = ffsga.GA(d, cfg, seed, 0, 0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        trace = []
        done = 0
        while done < gens:
            k = min(10, gens - done)
            if screened:
                g.step_screened(model, table, 4, k)
            else:
                g.step(k)
            done += k
            best = int(g.view()["elite_obj"].min().item())
            trace.append((done, time.perf_counter() - t0, best))
        g.status()
        return trace

    def first(trace, target):
        return next(((gn, t) for gn, t, b in trace if b <= target), (None, None))

    def evaluate(model, d, sd, plain, tag):
        table = model.score_table(model.features(d), d.n_active)
        hp, ho = populations(d, cfg, 7777 + sd, (0, 20))
        ys = model.score(table, hp).cpu().numpy()
        ho = ho.cpu().numpy()
        rho = [spearman(ys[k * pop:(k + 1) * pop], ho[k * pop:(k + 1) * pop]) for k in (0, 1)]
        scr = race(model, d, table, sd, True)
        target = plain[-1][2]
        gp, tp = first(plain, target)
        gs, ts = first(scr, target)
        progress(f"{tag} instance {sd}: plain {target} at gen {gp}, screened {scr[-1][2]}, "
                 f"reached at gen {gs}, rank correlation {rho[0]:.2f}/{rho[1]:.2f}")
        return {"instance_seed": sd, "plain_final": target, "screened_final": scr[-1][2],
                "plain_gens_to_target": gp, "plain_s_to_target": tp,
                "screened_gens_to_target": gs, "screened_s_to_target": ts,
                "speedup": (tp / ts) if ts else None, "heldout_spearman_gen0_20": rho,
                "plain_s_per_gen": plain[-1][1] / plain[-1][0],
                "screened_s_per_gen": scr[-1][1] / scr[-1][0]}

    def summary(rows):
        sp = [r["speedup"] if r["speedup"] is not None else 0.0 for r in rows]
        return {"median_speedup": float(np.median(sp)), "runs": len(rows),
                "reached": sum(r["screened_s_to_target"] is not None for r in rows),
                "screened_better_final": sum(r["screened_final"] < r["plain_final"] for r in rows),
                "per_instance": rows}

    # the cross-instance network: trained once on instances 100..
    t0 = time.perf_counter()
    cross = ffsga.Surrogate(W.surrogate_init(args.seed))
    cross_gen = torch.Generator(device="cpu").manual_seed(args.seed)
    data = []
    for sd in range(100, 100 + args.train_instances):
        d = ffsga.DeviceInstance.from_host(W.config2(sd).initial)
        prio, obj = populations(d, cfg, sd, (0, 10, 20, 40, 80))
        data.append((cross.features(d), prio, cross.targets(obj, pop)))
    cross_pairs = sum(int(x[1].shape[0]) for x in data)
    cross_fit = train(cross, data, cross_gen)
    del data
    t_cross = time.perf_counter() - t0
    progress(f"cross-instance network: {cross_pairs} pairs, {cross_fit[0]} steps, "
             f"loss {cross_fit[1]:.3f} -> {cross_fit[2]:.3f}, {t_cross:.1f} s")
    own_rows, cross_rows, prep = [], [], []
    for sd in range(args.seed, args.seed + args.race_seeds):
        d = ffsga.DeviceInstance.from_host(W.config2(sd).initial)
        t0 = time.perf_counter()
        feats = cross.features(d)
        data = []
        snaps = tuple(range(31)) if args.train_snapshots == "early" else tuple(range(0, 301, 10))
        for rs in range(1000, 1016):
            prio, obj = populations(d, cfg, rs, snaps)
            data.append((feats, prio, cross.targets(obj, pop)))
        torch.cuda.synchronize()
        t_data = time.perf_counter() - t0
        plain = None
        for k in range(args.train_seeds):
            t1 = time.perf_counter()
            model = ffsga.Surrogate(W.surrogate_init(k))
            fit = train(model, data, torch.Generator(device="cpu").manual_seed(1_000_003 * sd + k))
            prep.append({"instance_seed": sd, "train_seed": k, "data_s": t_data,
                         "train_s": time.perf_counter() - t1, "steps": fit[0], "loss_first": fit[1],
                         "loss_last50": fit[2]})
            if plain is None:
                if sd == args.seed:   # warm-up of both paths
                    race(model, d, None, sd, False)
                    race(model, d, model.score_table(feats, d.n_active), sd, True)
                plain = race(model, d, None, sd, False)
            row = evaluate(model, d, sd, plain, f"own-instance network {k}")
            row["train_seed"] = k
            own_rows.append(row)
        del data
        cross_rows.append(evaluate(cross, d, sd, plain, "cross-instance network"))
    own, crs = summary(own_rows), summary(cross_rows)
    out = common(args, "time-to-equal-fitness, surrogate vs plain GA", own["median_speedup"],
                 "x (plain GA time / screened GA time to the plain GA's final objective)",
                 (sum(r["screened_s_per_gen"] for r in own_rows)
                  + sum(r["plain_s_per_gen"] for r in own_rows if r["train_seed"] == 0)) * gens * 1e3,
                 "bf16/fp32 surrogate, int32 decode", {
                     "workload": "paper-shaped event 0 (50 jobs, 5 stages, 3 machines), 32 islands "
                                 f"x 8x16, {gens} generations, screened: 4 candidates per cell; "
                                 f"instances {args.seed}-{args.seed + args.race_seeds - 1}, "
                                 f"{args.train_seeds} own-instance networks each; value: median over "
                                 "(instance, network) pairs of the speedup (0 where the screened "
                                 "run never reaches the target)",
                     "own_instance": {**own, "training": prep,
                                      "train_snapshots": args.train_snapshots},
                     "cross_instance": {**crs, "train_pairs": cross_pairs, "train_steps": cross_fit[0],
                                        "loss_first": cross_fit[1], "loss_last50": cross_fit[2],
                                        "data_and_train_s": t_cross}})
    out["steps"] = 1
    out["warmup"] = 1
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="paper",
                    choices=["paper", "batch", "serve", "surrogate", "large"])
    ap.add_argument("--lds-slots", type=int, default=0)
    ap.add_argument("--rules", type=int, default=0, choices=[0, 1, 2, 3],
                    help="paper workload: job-vector decode variants, bit 0 FIFO stage order, "
                         "bit 1 power-aware machine choice")
    ap.add_argument("--encoding", default="job", choices=["job", "xy"],
                    help="paper workload: one priority per job (default) or the paper's X/Y "
                         "machine and priority matrices")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--generations", type=int, default=None,
                    help="override generations per event (profiling runs only)")
    ap.add_argument("--shops", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--gens-per-tick", type=int, default=10)
    ap.add_argument("--race-seeds", type=int, default=10)
    ap.add_argument("--train-instances", type=int, default=100)
    ap.add_argument("--train-seeds", type=int, default=3,
                    help="surrogate: own-instance networks per instance (initial weights and "
                         "batch order from seed k)")
    ap.add_argument("--train-snapshots", default="early", choices=["early", "spread"],
                    help="surrogate: train on generations 0-30 (early) or 0, 10, ..., 300 (spread) "
                         "of each seeded run")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch: the usual tuned configuration (8192 profile slots in 3 classes, "
                         "8 blocks per CU, one wave per child, graph) without tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 256 MiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the hot path is built and "
              f"measured on one GPU; sharding it across GPUs is not built.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "batch":
        print(json.dumps(bench_batch(args)), flush=True)
        return
    if args.workload == "serve":
        print(json.dumps(bench_serve(args)), flush=True)
        return
    if args.workload == "surrogate":
        print(json.dumps(bench_surrogate(args)), flush=True)
        return
    if args.workload == "large":
        print(json.dumps(bench_large(args)), flush=True)
        return
    bench_paper(args)


def bench_paper(args):
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    from paper_1903_10741_amd.run import run_workload

    wl = W.config2(args.seed)
    if args.generations is not None:
        wl.generations = args.generations
    xy = args.encoding == "xy"
    import dataclasses
    if xy:
        wl.ga = dataclasses.replace(wl.ga, encoding=1)
    if args.rules:
        wl.initial = dataclasses.replace(wl.initial, decode_rules=args.rules)
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        run_workload(wl, lds_slots=args.lds_slots)
    torch.cuda.synchronize()

    # events on the generation kernel only, one launch in 8 (spread evenly over
    # the timed steps): the other launches carry no markers
    ffsga.timing_enable(True, families=[ffsga.TIMING_GENERATION], every=8)
    work = 0
    decodes = 0
    best = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = run_workload(wl, lds_slots=args.lds_slots, sync_results=False)
        decodes += res.decodes
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    gen_ms, gen_launches = ffsga.timing_read(ffsga.TIMING_GENERATION)
    ffsga.timing_enable(False)
    best = [int(e.best_obj.item()) for e in res.events]

    # algorithmic work of the generation kernel, counted by the decoder
    work_res = run_workload(wl, lds_slots=args.lds_slots, sync_results=True, keep_work=True)
    work_per_decode = work_res.work / max(work_res.ga_decodes, 1)

    value = decodes / elapsed
    traffic = None
    valu_issue = None
    kname = "ga_generation_xy_kernel" if xy else "ga_generation_kernel"
    tpath = os.path.join(ROOT, "profiles", f"{kname}_paper-50x5x3.traffic.json")
    if os.path.exists(tpath):
        t = json.load(open(tpath))
        if t.get("build_id") == ffsga.ffs_build_id():  # counters of this very build only
            traffic = t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
            valu_issue = t.get("valu_issue_tlops")
    avg_launch_s = gen_ms / 1e3 / max(gen_launches, 1)
    decodes_per_launch = wl.ga.pop
    achieved = work_per_decode * decodes_per_launch / avg_launch_s / 1e12
    out = {
        "metric": "exact chromosome decodes/sec",
        "value": value,
        "unit": "decodes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded generator, paper-shaped)",
        "config": {
            "workload": "paper-shaped plain GA: 50 jobs, 5 stages, 3 unrelated machines, "
                        "5 arrival events, 32 islands x 8x16 = 4096, 500 generations/event" +
                        (", X/Y chromosome (machine and priority per operation)" if xy else ""),
            "encoding": "xy" if xy else "job priority vector",
            "decode_rules": args.rules,
            "decodes_per_step": decodes // args.steps,
            "events": 1 + len(wl.arrivals),
            "best_obj_per_event": best,
        },
        "roofline": {
            "bound": "alu",
            "kernel": f"{kname} (selection, crossover, mutation, decode)",
            "achieved": achieved,
            "peak": VALU_INT32_PEAK_TOPS,
            "unit": "TOP/s int32",
            "frac": achieved / VALU_INT32_PEAK_TOPS,
            "traffic": traffic,
            "valu_issue_frac": (valu_issue / VALU_INT32_PEAK_TOPS) if valu_issue else None,
            "work_per_decode": work_per_decode,
            "avg_launch_us": avg_launch_s * 1e6,
            "timed_launches": gen_launches,
            "timed_every": 8,
            "build_id": ffsga.ffs_build_id(),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
