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
    out = torch.empty(768, dtype=torch.int64, device="cuda:0")  # one output buffer: repeated calls replay a graph
    ms, outs = time_steps(lambda: job.rgb_hist(d, out=out)[1], steps, warmup, torch)
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
    from paper_1309_0215_amd import _lib as L
    first = Job(device=0).words(d)  # sizes the output buffers

    def run(job, steps_, warmup_):
        o, keep = job._word_out(len(first) + 16, int(first.key_bytes.numel()) + 64)

        def step():
            L.check(job.words_raw(d, o), "words")
            return o.stats.gpu_ms, o.stats.map_ms

        return time_steps(step, steps_, warmup_, torch)

    # whole job, as a caller repeating it sees it (the repeat replays a captured graph)
    ms, outs = run(Job(device=0), steps, warmup)
    gpu_ms = sum(x[0] for x in outs) / len(outs)
    # the map kernel alone (timed launches between events)
    _, touts = run(Job(device=0, timing=1), steps, 2)
    map_ms = sum(x[1] for x in touts) / len(touts)
    gbs = size / (ms * 1e-3) / 1e9
    return {"bytes": size, "distinct": len(first), "ms_per_step": ms, "gpu_ms": gpu_ms, "map_ms": map_ms, "GBps": gbs,
            "hbm_frac": gbs / HBM_PEAK_GBS, "map_kernel_GBps": size / (map_ms * 1e-3) / 1e9}


def bench_kmeans(torch, steps, warmup):
    import gen
    from paper_1309_0215_amd import Job
    X, C0 = gen.kmeans(3)  # 16,777,216 x 32 float32, k = 64
    Xd = torch.from_numpy(X).to("cuda:0")
    job = Job(device=0, km_centroids=torch.from_numpy(C0).to("cuda:0"), timing=1)
    ms, outs = time_steps(lambda: job.kmeans(Xd)[4], steps, warmup, torch)
    map_ms = sum(o["map_ms"] for o in outs) / len(outs)
    n, d, k = X.shape[0], X.shape[1], C0.shape[0]
    flops = 2.0 * n * k * d
    res = {"bytes": X.nbytes, "points": n, "ms_per_step": ms, "map_ms": map_ms, "GBps": X.nbytes / (ms * 1e-3) / 1e9,
           "hbm_frac": X.nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "assign_kernel_TFLOPs": flops / (map_ms * 1e-3) / 1e12,
           "fp32_frac": flops / (map_ms * 1e-3) / 1e12 / 157.3, "rechecked": outs[-1]["km_rechecked"]}
    del Xd
    return res


def bench_batched(torch, reps=3):
    """256 word-count jobs: one graph-replayed mr_batch_run vs 256 separate mr_run calls."""
    import gen
    from paper_1309_0215_amd import Job, _lib as L
    specs = gen.batched_specs()
    bufs = gen.job_inputs(specs)
    dev = [torch.from_numpy(b).to("cuda:0") for b in bufs]
    total = sum(len(b) for b in bufs)
    plain = Job(device=0)
    first = [plain.words(d) for d in dev]
    outs = [plain._word_out(len(r) + 16, int(r.key_bytes.numel()) + 64) for r in first]

    def run_plain():
        for d, (o, _) in zip(dev, outs):
            L.check(plain.words_raw(d, o), "words")

    batch = Job(device=0)
    prep = batch.batch_prepare(dev, cap_keys=[len(r) + 16 for r in first],
                               cap_bytes=[int(r.key_bytes.numel()) + 64 for r in first])
    res_b = batch.words_batch(dev, prepared=prep)
    same = all(torch.equal(a.key_bytes, b.key_bytes) and torch.equal(a.values, b.values)
               for a, b in zip(first, res_b))
    # the same batch with the autotuned launch parameters (tile share, LDS cache, load limit)
    tuned = Job(device=0)
    tuned.load_tuning()
    prep_t = tuned.batch_prepare(dev, cap_keys=[len(r) + 16 for r in first],
                                 cap_bytes=[int(r.key_bytes.numel()) + 64 for r in first])
    res_t = tuned.words_batch(dev, prepared=prep_t)
    same = same and all(torch.equal(a.key_bytes, b.key_bytes) and torch.equal(a.values, b.values)
                        for a, b in zip(first, res_t))
    ms_p, _ = time_steps(run_plain, reps, 1, torch)
    ms_b, _ = time_steps(lambda: batch.words_batch(dev, prepared=prep), reps, 1, torch)
    ms_t, _ = time_steps(lambda: tuned.words_batch(dev, prepared=prep_t), reps, 1, torch)
    return {"jobs": len(dev), "bytes": total, "plain_ms": ms_p, "batched_ms": ms_b, "batched_tuned_ms": ms_t,
            "plain_jobs_per_s": len(dev) / (ms_p * 1e-3), "batched_jobs_per_s": len(dev) / (ms_b * 1e-3),
            "batched_tuned_jobs_per_s": len(dev) / (ms_t * 1e-3), "batched_GBps": total / (ms_b * 1e-3) / 1e9,
            "batched_tuned_GBps": total / (ms_t * 1e-3) / 1e9, "speedup": ms_p / ms_b, "speedup_tuned": ms_p / ms_t,
            "outputs_identical": bool(same)}


def bench_selector(torch, n_jobs=200):
    """Held-out selector jobs: plain per-job rule vs learned vs batched word jobs + learned."""
    import gen
    from paper_1309_0215_amd import Job, _lib as L, selector as S
    specs_all = S._specs(2000, 16)
    _, test = S.split(specs_all, 1500)
    specs = [specs_all[i] for i in test[:n_jobs]]
    bufs = gen.job_inputs(specs)
    dev = []
    for s, b in zip(specs, bufs):
        d = torch.from_numpy(b).to("cuda:0")
        dev.append(d.view(torch.int32) if s.kind == "u32" else d)
    runner = S.Runner(torch)
    model = S.load_model(runner.learned)
    outs = [runner.outputs(s, d) for s, d in zip(specs, dev)]
    words = [i for i, s in enumerate(specs) if s.kind == "words"]
    ints = [i for i, s in enumerate(specs) if s.kind == "u32"]

    def plain():
        for s, d, (o, _) in zip(specs, dev, outs):
            L.check(runner.run(runner.rule, s, d, o)[0], "rule")

    def learned():
        for s, d, (o, _) in zip(specs, dev, outs):
            L.check(runner.run(runner.learned if s.kind == "u32" else runner.rule, s, d, o)[0], "learned")

    bjob = Job(device=0)
    prep = bjob.batch_prepare([dev[i] for i in words])

    def batched_learned():
        bjob.words_batch([dev[i] for i in words], prepared=prep)
        for i in ints:
            L.check(runner.run(runner.learned, specs[i], dev[i], outs[i][0])[0], "learned")

    ms_plain, _ = time_steps(plain, 2, 1, torch)
    ms_learn, _ = time_steps(learned, 2, 1, torch)
    ms_bl, _ = time_steps(batched_learned, 2, 1, torch)
    rep = model.get("meta", {}).get("report", {})
    return {"jobs": len(specs), "word_jobs": len(words), "int_jobs": len(ints),
            "bytes": int(sum(len(b) for b in bufs)),
            "plain_rule_jobs_per_s": len(specs) / (ms_plain * 1e-3),
            "learned_jobs_per_s": len(specs) / (ms_learn * 1e-3),
            "batched_learned_jobs_per_s": len(specs) / (ms_bl * 1e-3),
            "speedup_batched_learned_vs_plain": ms_plain / ms_bl,
            "heldout_regret_learned_mean": rep.get("regret_learned_mean"),
            "heldout_regret_rule_mean": rep.get("regret_rule_mean"),
            "heldout_regret_learned_p95": rep.get("regret_learned_p95"),
            "heldout_regret_rule_p95": rep.get("regret_rule_p95"),
            "trained_on": "1,500 of 2,000 seeded jobs, sizes 1-16 MiB (measured by the runtime on this GPU model)"}


def bench_hist16m(torch, steps=5):
    """The paper's Histogram: 2^28 uint32 keys over 2^24 possible keys, COUNT.

    The rule picks the global array (one array, atomics); the hash table and
    the sort are timed on the same input for comparison."""
    import gen
    from paper_1309_0215_amd import Job
    n, R = 1 << 28, 1 << 24
    keys = gen.uniform_keys(20, n, R)
    kt = torch.from_numpy(keys.view("int32")).to("cuda:0")
    del keys
    res = {"elements": n, "key_range": R, "bytes": 4 * n}
    for name, strat in (("rule", 0), ("hash", 4), ("sort", 5)):
        job = Job(device=0, strategy=strat, timing=1)
        ms, outs = time_steps(lambda: job.u32(kt, key_range=R).stats, steps, 1, torch)
        map_ms = sum(o["map_ms"] for o in outs) / len(outs)
        res[name] = {"strategy_used": int(outs[-1]["strategy_used"]), "ms_per_step": ms,
                     "GBps": 4 * n / (ms * 1e-3) / 1e9, "elements_per_s": n / (ms * 1e-3),
                     "map_ms": map_ms, "map_kernel_GBps": 4 * n / (map_ms * 1e-3) / 1e9}
        del job
    del kt
    return res


def bench_bloom(torch, steps=10):
    """The paper's Bloom Filter build: 30 million k-mers (k = 20) of synthetic
    DNA, 7 hash positions each, into one array of 300 million bits."""
    import gen
    from paper_1309_0215_amd import Job
    n, m, k, h = 30_000_019, 300_000_000, 20, 7
    d = torch.from_numpy(gen.dna(20, n)).to("cuda:0")
    job = Job(device=0, bloom_k=k, bloom_hashes=h)
    ms, outs = time_steps(lambda: job.bloom(d, m)[1], steps, 2, torch)
    kmers = int(outs[-1]["n_items"])
    algo = n + m // 8  # input read once, filter written once
    del d, job
    return {"bytes": n, "bits": m, "k": k, "hashes": h, "kmers": kmers, "ms_per_step": ms,
            "kmers_per_s": kmers / (ms * 1e-3), "input_GBps": n / (ms * 1e-3) / 1e9,
            "algorithmic_GBps": algo / (ms * 1e-3) / 1e9}


def bench_links(torch, steps=5):
    """The paper's Reverse Index: 78,355 synthetic HTML files, 307,921 links, 1 GiB."""
    import gen
    from paper_1309_0215_amd import Job
    h = gen.html(3)
    n = len(h.buf)
    d = torch.from_numpy(h.buf).to("cuda:0")
    r = torch.from_numpy(h.rec.view("int64")).to("cuda:0")
    job = Job(device=0)
    first = job.links(d, r)  # sizes the outputs
    caps = dict(cap_keys=len(first), cap_bytes=int(first.key_bytes.numel()), cap_ids=int(first.list_ids.numel()))
    ms, outs = time_steps(lambda: job.links(d, r, **caps).stats, steps, 1, torch)
    del d, r, job
    return {"bytes": n, "files": len(h.rec) - 1, "links": int(outs[-1]["n_items"]), "urls": len(first),
            "list_entries": int(first.list_ids.numel()), "ms_per_step": ms, "GBps": n / (ms * 1e-3) / 1e9,
            "links_per_s": int(outs[-1]["n_items"]) / (ms * 1e-3)}


def bench_copy(torch, steps=5):
    """A plain 1 GiB device-to-device copy: the reference whose HBM counters scale the kernels' counters."""
    n = 1 << 30
    x = torch.empty(n, dtype=torch.uint8, device="cuda:0").fill_(1)
    y = torch.empty_like(x)
    ms, _ = time_steps(lambda: y.copy_(x), steps, 1, torch)
    del x, y
    return {"bytes_read": n, "bytes_written": n, "ms_per_copy": ms, "GBps_read_plus_write": 2 * n / (ms * 1e-3) / 1e9}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_rgb_partial_rgb1GiB_hbm_counters.txt")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1309_0215_amd", "csrc", "hist.hip")


def measured_traffic():
    """HBM bytes per launch of k_rgb_partial from the committed counter summary.

    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are each scaled by what the
    same counter reads for a plain 1 GiB copy. None when the summary is
    missing or was taken on another version of the kernel source."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            line = line.strip()
            if line and not line.startswith("#") and "=" in line:
                k, v = (t.strip() for t in line.split("=", 1))
                kv[k] = v
        sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
        if kv.get("source_sha256") != sha:
            return None
        copy_kib = float(kv["copy_bytes"]) / 1024.0
        fetch = float(kv["kernel_fetch_kib"]) * copy_kib / float(kv["copy_fetch_kib"])
        write = float(kv["kernel_write_kib"]) * copy_kib / float(kv["copy_write_kib"])
        return (fetch + write) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline_rgb(buf):
    import oracle
    oracle.rgb(buf[:3 * 1024])  # load
    reps = 0
    t0 = time.perf_counter()
    while True:
        oracle.rgb(buf)
        reps += 1
        if time.perf_counter() - t0 > 12.0 or reps >= 16:
            break
    dt = (time.perf_counter() - t0) / reps
    return {"value": len(buf) / dt / 1e9, "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"full 1 GiB input, {reps} pass(es) of the sequential C++ oracle"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--apps", default="rgb,words8,words512,kmeans,hist16m,bloom,links,batched,selector")
    ap.add_argument("--no-cpu", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)", file=sys.stderr)
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

    if "kmeans" in apps:
        km = bench_kmeans(torch, max(3, args.steps // 2), 2)
        per_app["kmeans_step_16M_d32_k64"] = km
        log(f"kmeans: {km['GBps']:.1f} GB/s, assign {km['assign_kernel_TFLOPs']:.1f} TFLOP/s")
    if "batched" in apps:
        bt = bench_batched(torch)
        per_app["batched_word_count_256_jobs"] = bt
        log(f"batched: {bt['batched_jobs_per_s']:.0f} jobs/s, tuned {bt['batched_tuned_jobs_per_s']:.0f} jobs/s, "
            f"vs plain {bt['plain_jobs_per_s']:.0f} jobs/s")
    if "selector" in apps:
        sl = bench_selector(torch)
        per_app["selector_heldout_jobs"] = sl
        log(f"selector: batched+learned {sl['batched_learned_jobs_per_s']:.0f} jobs/s vs plain rule "
            f"{sl['plain_rule_jobs_per_s']:.0f} jobs/s")

    if "hist16m" in apps:
        h = bench_hist16m(torch)
        per_app["histogram_2p24_keys_2p28_elements"] = h
        log(f"histogram 2^24 keys: rule {h['rule']['GBps']:.1f} GB/s, hash {h['hash']['GBps']:.1f} GB/s, "
            f"sort {h['sort']['GBps']:.1f} GB/s")
    if "bloom" in apps:
        bl = bench_bloom(torch)
        per_app["bloom_filter_30M_kmers_300M_bits"] = bl
        log(f"bloom: {bl['ms_per_step']:.3f} ms, {bl['kmers_per_s'] / 1e9:.2f} G k-mers/s")
    if "links" in apps:
        li = bench_links(torch)
        per_app["reverse_index_78355_files_1GiB"] = li
        log(f"reverse index: {li['ms_per_step']:.3f} ms, {li['GBps']:.1f} GB/s")
    if "copy" in apps:
        cp = bench_copy(torch)
        per_app["copy_1GiB"] = cp
        log(f"copy: {cp['GBps_read_plus_write']:.1f} GB/s read+write")

    cpu = None
    if not args.no_cpu:
        log("cpu baseline")
        cpu = cpu_baseline_rgb(rgb_buf)

    n = rgb["bytes"]
    roof = {"kernel": "k_rgb_partial", "bound": "hbm", "achieved": rgb["kernel_GBps"], "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": rgb["kernel_GBps"] / HBM_PEAK_GBS, "traffic": measured_traffic(),
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
