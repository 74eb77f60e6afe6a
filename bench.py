"""Benchmark of the MapReduce hot path on one MI355X.

Prints ONE JSON line. The headline workload is the RGB histogram over 1 GiB
of interleaved pixels (floor(2^30 / 3) pixels, three-Gaussian mixture, seed
2): `value` is input GB/s over the timed steps (wall clock, inputs resident
in HBM). `per_app` adds the other workloads' input GB/s and fraction of HBM
peak; `roofline` describes the headline's dominant kernel; `cpu_baseline`
times the CPU oracle on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--apps rgb,words,...]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "input GB/s and % of HBM peak per app; batched+learned-select vs plain jobs/s"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3 / steps, outs


def bench_rgb(torch, steps, warmup):
    import numpy as np

    import gen
    from paper_1309_0215_amd import Job
    buf = gen.rgb(2)
    n = len(buf)
    d = torch.from_numpy(buf).to("cuda:0")
    job = Job(device=0, timing=1)
    ms, outs = time_steps(lambda: job.rgb_hist(d)[1], steps, warmup, torch)
    map_ms = sum(o["map_ms"] for o in outs) / len(outs)
    gpu_ms = sum(o["gpu_ms"] for o in outs) / len(outs)
    gbs = n / (ms * 1e-3) / 1e9
    res = {"bytes": n, "ms_per_step": ms, "gpu_ms": gpu_ms, "map_ms": map_ms, "GBps": gbs,
           "hbm_frac": gbs / HBM_PEAK_GBS, "kernel_GBps": n / (map_ms * 1e-3) / 1e9}
    return res, buf


def bench_words(torch, size, steps, warmup, seed=1):
    import gen
    from paper_1309_0215_amd import Job
    buf = gen.text(seed, size)
    d = torch.from_numpy(buf).to("cuda:0")
    job = Job(device=0, timing=1)
    first = job.words(d)  # sizes the output buffers
    o, keep = job._word_out(len(first) + 16, int(first.key_bytes.numel()) + 64)
    from paper_1309_0215_amd import _lib as L

    def step():
        st = job.words_raw(d, o)
        L.check(st, "words")
        return o.stats.gpu_ms, o.stats.map_ms

    ms, outs = time_steps(step, steps, warmup, torch)
    gpu_ms = sum(x[0] for x in outs) / len(outs)
    map_ms = sum(x[1] for x in outs) / len(outs)
    gbs = size / (ms * 1e-3) / 1e9
    return {"bytes": size, "distinct": len(first), "ms_per_step": ms, "gpu_ms": gpu_ms, "map_ms": map_ms, "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "map_kernel_GBps": size / (map_ms * 1e-3) / 1e9}


def cpu_baseline_rgb(buf):
    import oracle
    oracle.rgb(buf[:3 * 1024])  # load
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.rgb(buf)
        reps += 1
        if time.perf_counter() - t0 > 5.0 or reps >= 8:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": len(buf) / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"full 1 GiB input, {reps} pass(es) of the sequential C++ oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--apps", default="rgb,words8,words512")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    apps = set(args.apps.split(","))

    log("rgb: generating 1 GiB")
    rgb, rgb_buf = bench_rgb(torch, args.steps, args.warmup)
    log(f"rgb: {rgb['GBps']:.1f} GB/s (kernel {rgb['kernel_GBps']:.1f} GB/s)")
    per_app = {"rgb_histogram_1GiB": rgb}
    if "words8" in apps:
        w = bench_words(torch, 8 << 20, args.steps, args.warmup)
        per_app["word_count_8MiB"] = w
        log(f"words 8 MiB: {w['GBps']:.1f} GB/s, map {w['map_kernel_GBps']:.1f} GB/s")
    if "words512" in apps:
        w = bench_words(torch, 512 << 20, max(3, args.steps // 4), 2)
        per_app["word_count_512MiB"] = w
        log(f"words 512 MiB: {w['GBps']:.1f} GB/s, map {w['map_kernel_GBps']:.1f} GB/s")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline_rgb(rgb_buf)

    n = rgb["bytes"]
    roof = {"kernel": "k_rgb_partial", "bound": "hbm", "achieved": rgb["kernel_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": rgb["kernel_GBps"] / HBM_PEAK_GBS, "traffic": None,
            "algorithmic_bytes_per_launch": n}
    line = {
        "metric": METRIC,
        "value": rgb["GBps"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": rgb["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "rgb_histogram_1GiB", "pixels": n // 3, "bytes": n,
                   "distribution": "3 clipped Gaussians, means 40/128/210, sd 25, seed 2",
                   "output": "3x256 uint64 bins"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "per_app": per_app,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
