"""GPU parity of integer-key jobs (all four containers x all reduce ops) against the CPU oracle, bit-exact."""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

STRATS = {"lds_array": 2, "global_array": 3, "hash": 4, "sort": 5}
OPS = {"count": 0, "sum": 1, "min": 2, "max": 3}


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


_jobs = {}


def _job(strategy, **kw):
    from paper_1309_0215_amd import Job
    key = (strategy, tuple(sorted(kw.items())))
    if key not in _jobs:
        _jobs[key] = Job(device=0, strategy=strategy, **kw)
    return _jobs[key]


def _run(torch, job, keys, vals, op, R):
    kt = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
    vt = None if vals is None else torch.from_numpy(vals.view(np.int32)).to("cuda:0")
    return job.u32(kt, vt, op=OPS[op], key_range=R)


def _check(res, keys, vals, op):
    ek, ev = oracle.u32(keys, vals, op)
    gk = res.keys.cpu().numpy().view(np.uint32)
    gv = res.values.cpu().numpy()
    gv = gv.view(np.uint64) if op == "sum" else gv.view(np.uint32).astype(np.uint64)
    assert np.array_equal(gk, ek), (len(gk), len(ek))
    assert np.array_equal(gv, ev)


@pytest.mark.parametrize("strat", list(STRATS))
@pytest.mark.parametrize("op", list(OPS))
def test_strategies_ops(torch, strat, op):
    R = 3000
    n = 200_001
    keys, vals = gen.u32_keys(11, n, R, 1.1, with_values=True)
    if op == "count":
        vals = None
    res = _run(torch, _job(STRATS[strat]), keys, vals, op, R)
    _check(res, keys, vals, op)
    assert res.stats["strategy_used"] == STRATS[strat]


@pytest.mark.parametrize("strat", ["hash", "sort"])
def test_no_range_high_cardinality(torch, strat):
    rng = np.random.default_rng(5)
    keys = rng.integers(0, 2**32, size=300_000, dtype=np.uint64).astype(np.uint32)
    keys[:100] = 0xFFFFFFFF
    keys[100:200] = 0
    vals = rng.integers(0, 2**32, size=len(keys), dtype=np.uint64).astype(np.uint32)
    for op in OPS:
        v = None if op == "count" else vals
        _check(_run(torch, _job(STRATS[strat]), keys, v, op, 0), keys, v, op)


def test_rule_picks_by_range(torch):
    j = _job(0)
    keys, _ = gen.u32_keys(3, 100_000, 1000, 1.0)
    r = _run(torch, j, keys, None, "count", 1000)
    assert r.stats["strategy_used"] == STRATS["lds_array"]
    _check(r, keys, None, "count")
    keys2, _ = gen.u32_keys(4, 100_000, 1 << 20, 1.0)
    r = _run(torch, j, keys2, None, "count", 1 << 20)
    assert r.stats["strategy_used"] == STRATS["global_array"]
    _check(r, keys2, None, "count")
    r = _run(torch, j, keys2, None, "count", 0)
    assert r.stats["strategy_used"] == STRATS["hash"]
    _check(r, keys2, None, "count")


def test_empty_input(torch):
    for s in STRATS.values():
        j = _job(s)
        e = np.zeros(0, np.uint32)
        r = _run(torch, j, e, None, "count", 100)
        assert len(r.keys) == 0


def test_key_outside_range_is_rejected(torch):
    from paper_1309_0215_amd import MRError
    keys = np.arange(1000, dtype=np.uint32)
    for s in STRATS.values():
        with pytest.raises(MRError) as e:
            _run(torch, _job(s), keys, None, "count", 500)
        assert e.value.status == -1
    # the containers stay clean after the rejected runs
    for s in STRATS.values():
        k2 = (np.arange(5000) % 400).astype(np.uint32)
        _check(_run(torch, _job(s), k2, None, "count", 500), k2, None, "count")


def test_sum_wide_values(torch):
    keys = np.repeat(np.arange(50, dtype=np.uint32), 40_000)
    vals = np.full(len(keys), 0xFFFFFFFF, np.uint32)
    for s in STRATS.values():
        _check(_run(torch, _job(s), keys, vals, "sum", 50), keys, vals, "sum")


def test_hash_forced_collisions_and_regrowth(torch):
    keys, _ = gen.u32_keys(8, 60_000, 5000, 0.5)
    _check(_run(torch, _job(4, debug_hash=1), keys, None, "count", 0), keys, None, "count")
    keys2, _ = gen.u32_keys(9, 400_000, 200_000, 0.3)
    r = _run(torch, _job(4, table_slots=4096), keys2, None, "count", 0)
    _check(r, keys2, None, "count")
    assert r.stats["retries"] >= 1


def test_capacity_error(torch):
    import ctypes as C
    from paper_1309_0215_amd import _lib as L
    j = _job(4)
    keys = np.arange(1000, dtype=np.uint32)
    kt = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
    ko = torch.empty(10, dtype=torch.int32, device="cuda:0")
    vo = torch.empty(10, dtype=torch.int32, device="cuda:0")
    o = L.Output()
    o.keys, o.values, o.cap_keys = ko.data_ptr(), vo.data_ptr(), 10
    st = j.lib.mr_run(j.h, L.MAP_U32_KEYS, L.REDUCE_COUNT, kt.data_ptr(), 4000, None, 0, 0, C.byref(o))
    assert st == L.MR_ERR_CAPACITY and o.n_keys == 1000


@pytest.mark.parametrize("strat", list(STRATS))
def test_large_zipf(torch, strat):
    R = 1 << 16 if strat != "lds_array" else 4096
    keys, vals = gen.u32_keys(21, 4_000_000, R, 1.0, with_values=True)
    _check(_run(torch, _job(STRATS[strat]), keys, vals, "sum", R), keys, vals, "sum")


def test_mixed_kinds_on_one_job(torch):
    # One job alternating integer keys, word count, histogram and k-means:
    # every kind keeps its own buffers valid across the others' runs.
    from paper_1309_0215_amd import Job
    j = Job(device=0, strategy=4, km_centroids=torch.from_numpy(gen.kmeans(3, n=64)[1]).cuda())
    keys, vals = gen.u32_keys(12, 100_000, 5000, 1.0, with_values=True)
    txt = gen.text(13, 200_000, V=3000)
    rgb = gen.rgb(14, 3 * 10_000)
    X, _ = gen.kmeans(3, n=5000)
    for rep in range(3):
        _check(_run(torch, j, keys, vals, "sum", 0), keys, vals, "sum")
        w = j.words(torch.from_numpy(txt).cuda())
        assert w.items() == oracle.words(txt).items()
        _check(_run(torch, j, keys, None, "count", 0), keys, None, "count")
        h, _ = j.rgb_hist(torch.from_numpy(rgb).cuda())
        assert np.array_equal(h.cpu().numpy().astype(np.uint64), oracle.rgb(rgb))
        a, s, c, cent, st = j.kmeans(torch.from_numpy(X).cuda())
        assert int(c.sum()) == len(X)


@pytest.mark.parametrize("n", [524_288, 524_289])
def test_sort_at_the_one_workgroup_scan_limit(torch, n):
    """The sort's digit histograms (256 digits x 2048-element tiles) are
    scanned by one workgroup up to 65,536 entries: 524,288 pairs fill that
    exactly (64 steps of 64 entries per wave), one more pair takes the
    three-kernel scan."""
    keys, vals = gen.u32_keys(31, n, 1 << 20, 1.0, with_values=True)
    res = _run(torch, _job(STRATS["sort"]), keys, vals, "sum", 1 << 20)
    assert res.stats["strategy_used"] == STRATS["sort"]
    _check(res, keys, vals, "sum")
