"""Caller workspace (mr_job_config.workspace) and mr_workspace_bytes: each map
kind runs inside a workspace of exactly the queried size, with no device
allocation by the library (stats.device_allocs == 0), and gives results
identical to a job whose memory the library allocates (and to the oracle).
Also: a workspace one byte too small fails with MR_ERR_CAPACITY and reports
the bytes needed; calls of different kinds share one workspace; the
selector weights load from their JSON file."""
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _ws(torch, nbytes):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device="cuda:0")


def _words_equal(a, b):
    return (np.array_equal(a.key_bytes.cpu().numpy(), b.key_bytes.cpu().numpy())
            and np.array_equal(a.key_offsets.cpu().numpy(), b.key_offsets.cpu().numpy())
            and np.array_equal(a.values.cpu().numpy(), b.values.cpu().numpy()))


def test_words_in_exact_workspace(torch):
    from paper_1309_0215_amd import Job, workspace_bytes, _lib as L
    buf = gen.text(1, 8 << 20)
    d = torch.from_numpy(buf).to("cuda:0")
    need = workspace_bytes(L.MAP_WORDS, len(buf))
    job = Job(device=0, workspace=_ws(torch, need))
    ref = Job(device=0).words(d)
    exp = oracle.words(buf)
    for rep in range(3):  # the repeats keep the clean table and replay the graph
        r = job.words(d)
        assert r.stats["device_allocs"] == 0, rep
        assert _words_equal(r, ref), rep
    assert np.array_equal(r.values.cpu().numpy().astype(np.uint64), exp.values)


def test_rgb_u32_kmeans_bloom_in_exact_workspaces(torch):
    from paper_1309_0215_amd import Job, workspace_bytes, _lib as L
    # RGB
    buf = gen.rgb(2, 3 * 1_000_003)
    d = torch.from_numpy(buf).to("cuda:0")
    job = Job(device=0, workspace=_ws(torch, workspace_bytes(L.MAP_RGB_HIST, len(buf))))
    bins, st = job.rgb_hist(d)
    assert st["device_allocs"] == 0
    assert np.array_equal(bins.cpu().numpy().astype(np.uint64), oracle.rgb(buf))
    # integer keys: each container the rule or a forced strategy picks
    for strat, R, n in ((L.STRAT_RULE, 5000, 1 << 20), (L.STRAT_RULE, 1 << 22, 1 << 21), (L.STRAT_RULE, 0, 1 << 20),
                        (L.STRAT_SORT, 0, 300_001), (L.STRAT_LEARNED, 1 << 16, 1 << 20)):
        keys, _ = gen.u32_keys(7, n, R or 100_000, 0.8)
        kt = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
        need = workspace_bytes(L.MAP_U32_KEYS, 4 * n, key_range=R, strategy=strat)
        job = Job(device=0, strategy=strat, workspace=_ws(torch, need))
        if strat == L.STRAT_LEARNED:
            from paper_1309_0215_amd import selector as S
            S.load_model(job)
        for rep in range(2):
            res = job.u32(kt, key_range=R)
            assert res.stats["device_allocs"] == 0, (strat, R, rep)
            ek, ev = oracle.u32(keys)
            assert np.array_equal(res.keys.cpu().numpy().view(np.uint32), ek), (strat, R)
            assert np.array_equal(res.values.cpu().numpy().view(np.uint32).astype(np.uint64), ev), (strat, R)
    # k-means
    X, Cn = gen.kmeans(3, n=100_000, d=32, k=64)
    Xd = torch.from_numpy(X).to("cuda:0")
    Cd = torch.from_numpy(Cn).to("cuda:0")
    need = workspace_bytes(L.MAP_KMEANS, X.nbytes, km_k=64, km_d=32)
    job = Job(device=0, km_centroids=Cd, workspace=_ws(torch, need))
    ref = Job(device=0, km_centroids=Cd).kmeans(Xd)
    for rep in range(2):
        got = job.kmeans(Xd)
        assert got[4]["device_allocs"] == 0
        for a, b in zip(got[:4], ref[:4]):
            assert torch.equal(a, b), rep
    # Bloom filter
    dna = gen.dna(20, 1_000_003)
    dd = torch.from_numpy(dna).to("cuda:0")
    m = 10_000_019
    job = Job(device=0, workspace=_ws(torch, workspace_bytes(L.MAP_BLOOM, len(dna), key_range=m)))
    words, st = job.bloom(dd, m)
    assert st["device_allocs"] == 0
    exp, _ = oracle.bloom(dna, m)
    assert np.array_equal(words.cpu().numpy().view(np.uint32), exp)


def test_workspace_too_small_reports_need(torch):
    """A call in too small a workspace fails with MR_ERR_CAPACITY and reports
    the bytes it needs, at most the planned figure; a workspace of exactly
    that size then runs it."""
    from paper_1309_0215_amd import Job, workspace_bytes, _lib as L
    buf = gen.text(2, 1 << 20)
    d = torch.from_numpy(buf).to("cuda:0")
    planned = workspace_bytes(L.MAP_WORDS, len(buf))
    small = Job(device=0, workspace=_ws(torch, 4096))
    o, keep = small._word_out(1 << 16, 1 << 20)
    assert small.words_raw(d, o) == L.MR_ERR_CAPACITY
    need = int(o.stats.workspace_needed)
    assert 4096 < need <= planned
    job = Job(device=0, workspace=_ws(torch, need))
    r = job.words(d)
    assert r.stats["device_allocs"] == 0
    assert np.array_equal(r.values.cpu().numpy().astype(np.uint64), oracle.words(buf).values)


def test_kinds_share_one_workspace_and_library_allocations_are_counted(torch):
    from paper_1309_0215_amd import Job, workspace_bytes, _lib as L
    text = gen.text(3, 2 << 20)
    rgb = gen.rgb(4, 3 * 400_000)
    keys, _ = gen.u32_keys(5, 1 << 20, 1 << 18, 1.0)
    dt, dr = torch.from_numpy(text).to("cuda:0"), torch.from_numpy(rgb).to("cuda:0")
    dk = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
    need = max(workspace_bytes(L.MAP_WORDS, len(text)), workspace_bytes(L.MAP_RGB_HIST, len(rgb)),
               workspace_bytes(L.MAP_U32_KEYS, 4 * len(keys)))
    job = Job(device=0, workspace=_ws(torch, need))
    lib_job = Job(device=0)
    exp_w = oracle.words(text)
    exp_k = oracle.u32(keys)
    first = lib_job.words(dt)
    assert first.stats["device_allocs"] > 0
    assert lib_job.words(dt).stats["device_allocs"] == 0  # kept between calls
    for _ in range(2):
        w = job.words(dt)
        assert np.array_equal(w.values.cpu().numpy().astype(np.uint64), exp_w.values)
        assert np.array_equal(w.key_bytes.cpu().numpy(), exp_w.key_bytes)
        b, _ = job.rgb_hist(dr)
        assert np.array_equal(b.cpu().numpy().astype(np.uint64), oracle.rgb(rgb))
        u = job.u32(dk)
        assert np.array_equal(u.keys.cpu().numpy().view(np.uint32), exp_k[0])
        assert np.array_equal(u.values.cpu().numpy().view(np.uint32).astype(np.uint64), exp_k[1])
        for r in (w.stats, u.stats):
            assert r["device_allocs"] == 0


def test_selector_load_from_json(torch):
    import ctypes as C
    from paper_1309_0215_amd import Job, MRError, _lib as L, selector as S
    a, b = Job(device=0), Job(device=0)
    S.load_model(a)
    L.check(b.lib.mr_selector_load(b.h, S.WEIGHTS_PATH.encode()), "mr_selector_load")
    f = np.random.default_rng(0).standard_normal(12).astype(np.float32)
    pa, pb = np.zeros(4, np.float32), np.zeros(4, np.float32)
    for job, p in ((a, pa), (b, pb)):
        L.check(job.lib.mr_selector_predict(job.h, f.ctypes.data_as(C.c_void_p), p.ctypes.data_as(C.c_void_p)), "predict")
    assert np.array_equal(pa, pb)
    assert b.lib.mr_selector_load(b.h, b"/nonexistent/weights.json") == L.MR_ERR_INVALID_ARG
