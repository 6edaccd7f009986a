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
    return {"value": decodes / dt, "unit": "decodes/s", "cores": threads, "kind": "oracle",
            "sample": f"one full step: {len(out)} events x (1 + {wl.generations}) generations x "
                      f"{wl.ga.pop} individuals + plan decodes ({decodes} decodes, {dt:.1f} s)",
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
    ffsga.timing_enable(True)
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
    """Rescheduling requests from 512 shops arriving Poisson at 200/s, each 100
    generations of population 1024, continuously batched; latency and throughput."""
    import torch
    from paper_1903_10741_amd import autotune, ffsga
    from paper_1903_10741_amd import workloads as W
    from paper_1903_10741_amd.serve import Server, poisson_schedule
    n_events = 2
    shops = W.shops(args.seed, args.shops)
    arrs = [W.shop_arrivals(args.seed, k, s, n_events - 1) for k, s in enumerate(shops)]
    gens = args.generations or 100
    dev = [ffsga.DeviceInstance.from_host(s) for s in shops[:64]]
    tune = autotune.tune(dev, shops[:64], W.SERVING_GA, generations=2, log=progress)
    srv = Server(shops, arrs, W.SERVING_GA, generations=gens, n_slots=args.slots,
                 gens_per_tick=args.gens_per_tick, seed=args.seed,
                 tuning={"use_graph": True, "blocks": tune.best.blocks,
                         "lds_slots": tune.best.lds_slots, "schedule": tune.best.schedule,
                         "profile_classes": tune.best.profile_classes})
    progress("serving starts")
    sched = poisson_schedule(args.seed, args.rate, [n_events] * len(shops))
    torch.cuda.synchronize()
    m = srv.run(sched, log=progress)
    out = common(args, "exact chromosome decodes/sec", m["decodes_per_s"], "decodes/s",
                 m["wall_s"] * 1e3, "int32", {
                     "workload": f"serving: {len(shops)} shops, {n_events} events each, Poisson "
                                 f"{args.rate}/s, {gens} generations x pop 1024 per request",
                     **{k: v for k, v in m.items()}})
    out["steps"] = 1
    out["warmup"] = 0
    return out


def surrogate_dataset(d, ga_cfg, seeds, gens):
    """Decoder-labelled chromosomes: every population of `gens` plain generations
    (and generation 0) of GA runs with the given seeds, with their exact objectives."""
    import torch
    from paper_1903_10741_amd import ffsga
    prios, objs = [], []
    for sd in seeds:
        g = ffsga.GA(d, ga_cfg, sd, 0, 0)
        for k in range(gens + 1):
            if k:
                g.step(1)
            v = g.view()
            prios.append(v["prio"].clone())
            objs.append(v["obj"].clone())
    return torch.cat(prios), torch.cat(objs)


def spearman(a, b):
    import numpy as np
    ra = np.argsort(np.argsort(a))
    rb = np.argsort(np.argsort(b))
    return float(np.corrcoef(ra, rb)[0, 1])


def bench_surrogate(args):
    """Time to reach the plain GA's final fitness (500 generations, event 0 of the
    paper-shaped workload), screened GA (4 candidates per cell, lowest surrogate
    score kept) against the plain GA, same seed, same GPU."""
    import numpy as np
    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    wl = W.config2(args.seed)
    inst = wl.initial
    gens = args.generations or wl.generations
    cfg = ffsga.GaConfig.of(wl.ga)
    d = ffsga.DeviceInstance.from_host(inst)
    # 1. data: 16 seeded runs x 31 populations x 4096 = 2.03M decoder-labelled chromosomes
    t0 = time.perf_counter()
    prio, obj = surrogate_dataset(d, cfg, range(1000, 1016), 30)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    # 2. training: Adam, batches of 4096, 2 epochs, constant rate; targets standardised
    #    within each population
    model = ffsga.Surrogate(W.surrogate_init(args.seed))
    feats = model.features(d)
    tgt = model.targets(obj, wl.ga.pop)
    gen = torch.Generator(device="cpu").manual_seed(args.seed)
    N = prio.shape[0]
    B = 4096
    t0 = time.perf_counter()
    losses = []
    for ep in range(2):
        perm = torch.randperm(N, generator=gen).cuda()
        for i in range(0, N - B + 1, B):
            idx = perm[i:i + B]
            loss, _ = model.train_step(feats, prio[idx], tgt[idx], 1e-3)
            losses.append(loss)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    losses = [float(x.item()) for x in losses]
    table = model.score_table(feats, inst.n_active)
    # held-out quality: rank correlation inside populations of an unseen seed
    ho_p, ho_o = surrogate_dataset(d, cfg, [7777], 20)
    ys = model.score(table, ho_p).cpu().numpy()
    ho = ho_o.cpu().numpy()
    rho = [spearman(ys[k * wl.ga.pop:(k + 1) * wl.ga.pop], ho[k * wl.ga.pop:(k + 1) * wl.ga.pop])
           for k in (0, 10, 20)]

    # 3. the race, per seed: plain and screened GA for the same generations, best
    #    elite read every 10 generations; the time each first reaches the plain
    #    GA's final objective
    def race(seed, screened):
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
    race(0, False)    # warm-up of both paths
    race(0, True)
    per_seed = []
    for sd in range(args.seed, args.seed + args.race_seeds):
        plain, scr = race(sd, False), race(sd, True)
        target = plain[-1][2]
        gp, tp = first(plain, target)
        gs, ts = first(scr, target)
        per_seed.append({"seed": sd, "plain_final": target, "screened_final": scr[-1][2],
                         "plain_gens_to_target": gp, "plain_s_to_target": tp,
                         "screened_gens_to_target": gs, "screened_s_to_target": ts,
                         "speedup": (tp / ts) if ts else None,
                         "plain_s_per_gen": plain[-1][1] / plain[-1][0],
                         "screened_s_per_gen": scr[-1][1] / scr[-1][0]})
        print(f"[bench] race seed {sd}: plain {target} at gen {gp}, screened {scr[-1][2]}, "
              f"reached at gen {gs}", file=sys.stderr, flush=True)
    sp = [r["speedup"] if r["speedup"] is not None else 0.0 for r in per_seed]
    value = float(np.median(sp))
    out = common(args, "time-to-equal-fitness, surrogate vs plain GA", value,
                 "x (plain GA time / screened GA time to the plain GA's final objective)",
                 sum(r["plain_s_per_gen"] + r["screened_s_per_gen"] for r in per_seed) * gens * 1e3,
                 "bf16/fp32 surrogate, int32 decode", {
                     "workload": "paper-shaped event 0 (50 jobs, 5 stages, 3 machines), "
                                 f"32 islands x 8x16, {gens} generations, screened: 4 candidates "
                                 f"per cell, {args.race_seeds} seeds (median speedup; a seed whose "
                                 "screened run never reaches the target counts 0)",
                     "seeds_reached": sum(r["screened_s_to_target"] is not None for r in per_seed),
                     "screened_better_final": sum(r["screened_final"] < r["plain_final"]
                                                  for r in per_seed),
                     "per_seed": per_seed,
                     "train_pairs": int(N), "train_steps": len(losses), "train_s": t_train,
                     "data_s": t_data, "loss_first": losses[0], "loss_last": losses[-1],
                     "heldout_spearman_gen0_10_20": rho})
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
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--generations", type=int, default=None,
                    help="override generations per event (profiling runs only)")
    ap.add_argument("--shops", type=int, default=512)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--slots", type=int, default=64)
    ap.add_argument("--gens-per-tick", type=int, default=10)
    ap.add_argument("--race-seeds", type=int, default=8)
    ap.add_argument("--no-autotune", action="store_true",
                    help="batch: the usual tuned configuration (8192 profile slots in 3 classes, "
                         "8 blocks per CU, one wave per child, graph) without tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 256 MiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              f"described in DESIGN.md and not built.", file=sys.stderr)
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
    if args.copy_calibration:
        src = torch.ones(64 << 20, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        run_workload(wl, lds_slots=args.lds_slots)
    torch.cuda.synchronize()

    ffsga.timing_enable(True)
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
    tpath = os.path.join(ROOT, "profiles", "ga_generation_kernel_paper-50x5x3.traffic.json")
    if os.path.exists(tpath):
        t = json.load(open(tpath))
        if t.get("build_id") == ffsga.ffs_build_id():  # counters of this very build only
            traffic = t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"]
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
                        "5 arrival events, 32 islands x 8x16 = 4096, 500 generations/event",
            "decodes_per_step": decodes // args.steps,
            "events": 1 + len(wl.arrivals),
            "best_obj_per_event": best,
        },
        "roofline": {
            "bound": "alu",
            "kernel": "ga_generation_kernel (selection, crossover, mutation, decode)",
            "achieved": achieved,
            "peak": VALU_INT32_PEAK_TOPS,
            "unit": "TOP/s int32",
            "frac": achieved / VALU_INT32_PEAK_TOPS,
            "traffic": traffic,
            "work_per_decode": work_per_decode,
            "avg_launch_us": avg_launch_s * 1e6,
            "launches": gen_launches,
            "build_id": ffsga.ffs_build_id(),
        },
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
