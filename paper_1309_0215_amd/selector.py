"""Training and evaluation of the learned reduce-strategy selector.

The runtime generates its own training data: every job of a seeded synthetic
set is run with each feasible reduce container (LDS array, global array, hash
table, sort), the device time of each is measured, and all containers must
produce identical outputs. Job features come from the library's feature
kernel. The 12-64-64-4 network is trained on the GPU with the library's own
forward, backward and Adam kernels (this module only marshals tensors), and
is compared with the paper-style rule by regret on held-out jobs.

Readings of the selector set-up (not in the paper): ReLU; the four outputs
predict standardised log device times (one mean and scale over all
containers, so outputs compare directly); masked mean squared error over the
feasible containers; Adam (lr 1e-3, betas 0.9 / 0.999, eps 1e-8), batch 64,
He-uniform initialisation with a fixed seed; split stratified by key type.
"""
from __future__ import annotations

import ctypes as C
import json
import os
import time

import numpy as np

from . import _lib as L

STRATS = [L.STRAT_LDS_ARRAY, L.STRAT_GLOBAL_ARRAY, L.STRAT_HASH, L.STRAT_SORT]
STRAT_NAMES = ["lds_array", "global_array", "hash", "sort"]
LDS_BUDGET = 64 * 1024
GLOBAL_MAX = 1 << 27
WEIGHTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "selector_weights.json")


def feasible(spec) -> np.ndarray:
    """Which of the four containers can run this job (same test as the library)."""
    if spec.kind == "words":
        return np.array([False, False, True, False])
    R = spec.card if spec.declare_range else 0
    lds = R > 0 and (4 * R + (8 * R + 8 if spec.op == "sum" else 0)) <= LDS_BUDGET
    return np.array([lds, R > 0 and R <= GLOBAL_MAX, True, True])


def rule_choice(spec) -> int:
    f = feasible(spec)
    if spec.kind == "words":
        return 2
    if f[0]:
        return 0
    if f[1]:
        return 1
    return 2


def _nbytes(d) -> int:
    return int(d.numel()) * int(d.element_size())


class Runner:
    """One library job per container (strategy fixed at creation), on torch's current stream."""

    def __init__(self, torch, device=0):
        from . import Job
        self.torch = torch
        self.jobs = {s: Job(device=device, strategy=s) for s in STRATS}
        self.rule = Job(device=device, strategy=L.STRAT_RULE)
        self.learned = Job(device=device, strategy=L.STRAT_LEARNED)
        self.lib = self.rule.lib

    def features(self, spec, d) -> np.ndarray:
        f = np.zeros(12, np.float32)
        kind = L.MAP_WORDS if spec.kind == "words" else (L.MAP_U32_KV if spec.op == "sum" else L.MAP_U32_KEYS)
        op = L.REDUCE_SUM if spec.op == "sum" else L.REDUCE_COUNT
        R = spec.card if (spec.kind == "u32" and spec.declare_range) else 0
        L.check(self.lib.mr_job_features(self.rule.h, kind, op, d.data_ptr(), _nbytes(d), R,
                                         f.ctypes.data_as(C.c_void_p)), "mr_job_features")
        return f

    def run(self, job, spec, d, out):
        """One mr_run; returns (status, device ms)."""
        if spec.kind == "words":
            st = job.words_raw(d, out)
        else:
            kind = L.MAP_U32_KV if spec.op == "sum" else L.MAP_U32_KEYS
            op = L.REDUCE_SUM if spec.op == "sum" else L.REDUCE_COUNT
            R = spec.card if spec.declare_range else 0
            st = self.lib.mr_run(job.h, kind, op, d.data_ptr(), _nbytes(d), None, 0, R, C.byref(out))
        return st, out.stats.gpu_ms

    def outputs(self, spec, d):
        """Output buffers sized for the job."""
        torch = self.torch
        n = _nbytes(d)
        o = L.Output()
        if spec.kind == "words":
            cap = min(n // 2 + 1, spec.card + 16)
            kb = torch.empty(max(n, 1), dtype=torch.uint8, device=d.device)
            ko = torch.empty(cap + 1, dtype=torch.int64, device=d.device)
            v = torch.empty(max(cap, 1), dtype=torch.int32, device=d.device)
            o.key_bytes, o.key_offsets, o.values = kb.data_ptr(), ko.data_ptr(), v.data_ptr()
            o.cap_keys, o.cap_key_bytes = cap, n
            return o, (kb, ko, v)
        esz = 8 if spec.op == "sum" else 4
        cap = max(1, min(n // esz, spec.card))
        k = torch.empty(cap, dtype=torch.int32, device=d.device)
        v = torch.empty(cap, dtype=torch.int64 if spec.op == "sum" else torch.int32, device=d.device)
        o.keys, o.values, o.cap_keys = k.data_ptr(), v.data_ptr(), cap
        return o, (k, v)


def measure(runner: Runner, specs, inputs, reps: int = 2, check_agreement: bool = True, log=None):
    """Features and per-container device times (ms; inf when infeasible) of each job."""
    torch = runner.torch
    X = np.zeros((len(specs), 12), np.float32)
    T = np.full((len(specs), 4), np.inf)
    for i, (spec, buf) in enumerate(zip(specs, inputs)):
        d = torch.from_numpy(buf).to("cuda:0")
        if spec.kind == "u32":
            d = d.view(torch.int32)
        X[i] = runner.features(spec, d)
        feas = feasible(spec)
        ref = None
        for s in range(4):
            if not feas[s]:
                continue
            out, keep = runner.outputs(spec, d)
            st, _ = runner.run(runner.jobs[STRATS[s]], spec, d, out)  # warm-up (sizes workspaces)
            L.check(st, f"job {i} {STRAT_NAMES[s]}")
            ms = []
            for _ in range(reps):
                st, t = runner.run(runner.jobs[STRATS[s]], spec, d, out)
                L.check(st, f"job {i} {STRAT_NAMES[s]}")
                ms.append(t)
            T[i, s] = float(np.median(ms))
            if check_agreement and spec.kind == "u32":
                n = int(out.n_keys)
                got = (keep[0][:n].clone(), keep[1][:n].clone())
                if ref is None:
                    ref = got
                elif not (torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])):
                    raise AssertionError(f"job {i}: containers disagree ({STRAT_NAMES[s]})")
        if log and i % 100 == 0:
            log(f"measured {i + 1}/{len(specs)}")
    return X, T


def split(specs, n_train: int, seed: int = 0):
    """Stratified split by key type."""
    rng = np.random.default_rng(seed)
    idx = np.arange(len(specs))
    kinds = np.array([s.kind for s in specs])
    train = []
    for k in ("u32", "words"):
        ids = idx[kinds == k]
        rng.shuffle(ids)
        take = int(round(n_train * len(ids) / len(specs)))
        train.extend(ids[:take].tolist())
    train = np.array(sorted(train))
    test = np.setdiff1d(idx, train)
    return train, test


def train(torch, X, T, feas, epochs: int = 500, batch: int = 64, lr: float = 1e-3, seed: int = 0, log=None):
    """Train on the GPU with mr_selector_train (the library runs the whole
    loop with its forward, backward and Adam kernels). Returns (model dict,
    mean loss per epoch)."""
    import tempfile

    from . import Job
    job = Job(device=0)
    cfg = L.TrainConfig(epochs=epochs, batch=batch, lr=lr, beta1=0.9, beta2=0.999, eps=1e-8, seed=seed)
    Xc = np.ascontiguousarray(X, np.float32)
    Tc = np.ascontiguousarray(np.where(feas, T, 1.0), np.float32)
    Fc = np.ascontiguousarray(feas, np.uint8)
    hist = np.zeros(epochs, np.float32)
    p = lambda a: a.ctypes.data_as(C.c_void_p)  # noqa: E731
    with tempfile.TemporaryDirectory() as d:
        path = os.path.join(d, "selector_weights.json")
        L.check(job.lib.mr_selector_train(job.h, p(Xc), p(Tc), p(Fc), len(Xc), C.byref(cfg), p(hist), path.encode()),
                "mr_selector_train")
        with open(path) as f:
            model = json.load(f)
    if log:
        for ep in list(range(0, epochs, 100)) + [epochs - 1]:
            log(f"epoch {ep}: loss {hist[ep]:.4f}")
    return model, hist.tolist()


def predict(torch, model, X) -> np.ndarray:
    """Network outputs for features X, on the GPU with the library's forward kernel."""
    from . import Job
    job = Job(device=0)
    Xn = ((X - np.array(model["feat_mean"], np.float32)) / np.array(model["feat_scale"], np.float32)).astype(np.float32)
    P = torch.tensor(model["params"], dtype=torch.float32, device="cuda:0")
    Xd = torch.from_numpy(Xn).to("cuda:0")
    Y = torch.empty(len(Xn), 4, device="cuda:0")
    L.check(job.lib.mr_mlp_forward(job.h, P.data_ptr(), Xd.data_ptr(), len(Xn), None, None, Y.data_ptr()), "forward")
    return Y.cpu().numpy()


def choose(pred: np.ndarray, feas: np.ndarray) -> np.ndarray:
    return np.argmin(np.where(feas, pred, np.inf), axis=1)


def regret(T: np.ndarray, feas: np.ndarray, chosen: np.ndarray) -> np.ndarray:
    best = np.where(feas, T, np.inf).min(1)
    return T[np.arange(len(T)), chosen] / best - 1.0


def load_model(job, path: str = WEIGHTS_PATH):
    """Load trained weights into a library job (mr_selector_set)."""
    with open(path) as f:
        m = json.load(f)
    arrs = [np.ascontiguousarray(np.array(m[k], np.float32)) for k in
            ("params", "feat_mean", "feat_scale", "feat_lo", "feat_hi")]
    L.check(job.lib.mr_selector_set(job.h, *[a.ctypes.data_as(C.c_void_p) for a in arrs]), "mr_selector_set")
    return m


def save_model(model: dict, path: str = WEIGHTS_PATH, meta: dict | None = None):
    m = dict(model)
    if meta:
        m["meta"] = meta
    with open(path, "w") as f:
        json.dump(m, f)


def timed_jobs_per_second(runner: Runner, job, specs, inputs) -> tuple[float, float]:
    """Wall-clock jobs/s of running every job once with `job` (inputs already resident), and total ms."""
    torch = runner.torch
    devs = []
    outs = []
    for spec, buf in zip(specs, inputs):
        d = buf
        devs.append(d)
        outs.append(runner.outputs(spec, d))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for spec, d, (o, _) in zip(specs, devs, outs):
        st, _ = runner.run(job, spec, d, o)
        L.check(st, "timed run")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return len(specs) / dt, dt * 1e3


# ----------------------------------------------------------------------------
# command line: build the timing set on the GPU, train, evaluate, save
# ----------------------------------------------------------------------------

def _specs(n_jobs: int, size_hi_mib: int, seed: int = 5):
    import gen
    specs = gen.selector_specs(seed=seed, n_jobs=n_jobs, size_hi=size_hi_mib << 20)
    for sp in specs:
        if sp.kind == "words":
            sp.card = min(sp.card, 1 << 20)  # vocabulary generation cost on the host
    return specs


def main(argv=None):
    import argparse
    import sys

    import torch

    import gen
    ap = argparse.ArgumentParser(description="train the reduce-strategy selector on measured timings")
    ap.add_argument("--n-jobs", type=int, default=2000)
    ap.add_argument("--n-train", type=int, default=1500)
    ap.add_argument("--size-hi-mib", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=500)
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--out", default="selector_out")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)
    log = lambda *a: print(*a, file=sys.stderr, flush=True)  # noqa: E731
    pool = gen.job_pool()  # before any GPU use: no process is started after that
    specs = _specs(args.n_jobs, args.size_hi_mib)
    train_idx, test_idx = split(specs, args.n_train)
    feas = np.array([feasible(s) for s in specs])
    runner = Runner(torch)
    X = np.zeros((len(specs), 12), np.float32)
    T = np.full((len(specs), 4), np.inf)
    test_dev = {}
    chunk = 64
    t0 = time.time()
    test_set = set(test_idx.tolist())
    for c0 in range(0, len(specs), chunk):
        ids = list(range(c0, min(len(specs), c0 + chunk)))
        bufs = gen.job_inputs([specs[i] for i in ids], pool=pool)
        Xi, Ti = measure(runner, [specs[i] for i in ids], bufs, reps=args.reps)
        X[ids], T[ids] = Xi, Ti
        for j, i in enumerate(ids):
            if i in test_set:
                d = torch.from_numpy(bufs[j]).to("cuda:0")
                test_dev[i] = d.view(torch.int32) if specs[i].kind == "u32" else d
        log(f"jobs {ids[-1] + 1}/{len(specs)} measured, {time.time() - t0:.0f} s")
    pool.shutdown()
    np.savez(os.path.join(args.out, "timings.npz"), X=X, T=T, feas=feas, train=train_idx, test=test_idx)
    model, hist = train(torch, X[train_idx], T[train_idx], feas[train_idx], epochs=args.epochs, log=log)
    pred = predict(torch, model, X[test_idx])
    ch_learned = choose(pred, feas[test_idx])
    ch_rule = np.array([rule_choice(specs[i]) for i in test_idx])
    r_l = regret(T[test_idx], feas[test_idx], ch_learned)
    r_r = regret(T[test_idx], feas[test_idx], ch_rule)
    save_model(model, os.path.join(args.out, "selector_weights.json"),
               meta={"n_jobs": len(specs), "n_train": int(len(train_idx)), "size_hi_mib": args.size_hi_mib,
                     "epochs": args.epochs, "final_loss": hist[-1],
                     "command": "python -m paper_1309_0215_amd.selector " + " ".join(argv or sys.argv[1:])})
    # held-out jobs/s: rule-selected vs learned-selected, one mr_run per job, inputs resident
    load_model(runner.learned, os.path.join(args.out, "selector_weights.json"))
    tspecs = [specs[i] for i in test_idx]
    tdev = [test_dev[i] for i in test_idx]
    timed_jobs_per_second(runner, runner.rule, tspecs[:8], tdev[:8])  # warm-up
    timed_jobs_per_second(runner, runner.learned, tspecs[:8], tdev[:8])
    jps_rule, ms_rule = timed_jobs_per_second(runner, runner.rule, tspecs, tdev)
    jps_learn, ms_learn = timed_jobs_per_second(runner, runner.learned, tspecs, tdev)
    u32_test = np.array([specs[i].kind == "u32" for i in test_idx])
    report = {
        "n_jobs": len(specs), "n_train": int(len(train_idx)), "n_test": int(len(test_idx)),
        "size_range_mib": [1, args.size_hi_mib], "loss_first": hist[0], "loss_last": hist[-1],
        "regret_learned_mean": float(r_l.mean()), "regret_learned_p95": float(np.quantile(r_l, 0.95)),
        "regret_rule_mean": float(r_r.mean()), "regret_rule_p95": float(np.quantile(r_r, 0.95)),
        "regret_learned_u32_mean": float(r_l[u32_test].mean()), "regret_rule_u32_mean": float(r_r[u32_test].mean()),
        "oracle_best_device_ms": float(np.where(feas[test_idx], T[test_idx], np.inf).min(1).sum()),
        "learned_device_ms": float(T[test_idx][np.arange(len(test_idx)), ch_learned].sum()),
        "rule_device_ms": float(T[test_idx][np.arange(len(test_idx)), ch_rule].sum()),
        "jobs_per_s_rule": jps_rule, "jobs_per_s_learned": jps_learn,
        "wall_ms_rule": ms_rule, "wall_ms_learned": ms_learn,
        "choices_learned": np.bincount(ch_learned, minlength=4).tolist(),
        "choices_rule": np.bincount(ch_rule, minlength=4).tolist(),
    }
    with open(os.path.join(args.out, "report.json"), "w") as f:
        json.dump(report, f, indent=1)
    # the held-out jobs' features and measured container times: the table the
    # regret test replays (learned choices from the device, rule choices as run)
    heldout = {"features": np.round(X[test_idx], 6).tolist(), "times_ms": np.where(np.isfinite(T[test_idx]),
                                                                                    T[test_idx], -1.0).round(6).tolist(),
               "feasible": feas[test_idx].astype(int).tolist(), "rule_choice": ch_rule.tolist(),
               "kind": [specs[i].kind for i in test_idx], "size_range_mib": [1, args.size_hi_mib]}
    with open(os.path.join(args.out, "selector_heldout.json"), "w") as f:
        json.dump(heldout, f)
    print(json.dumps(report))


if __name__ == "__main__":
    main()
