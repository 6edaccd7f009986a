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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--lds-slots", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--generations", type=int, default=None,
                    help="override generations per event (profiling runs only)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 256 MiB device copy, the reference for HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              f"described in DESIGN.md and not built.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1903_10741_amd import ffsga
    from paper_1903_10741_amd import workloads as W
    from paper_1903_10741_amd.run import run_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
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
