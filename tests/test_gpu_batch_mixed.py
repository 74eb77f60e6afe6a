"""mr_batch_run over a mixed set of word-count and integer-key jobs (the
selector workload's mix of key types, value types, declared and undeclared
ranges): every item equals the oracle and the same job run alone with
mr_run, under the rule and under the learned selector (whose choices for all
integer items come from one captured graph, replayed on the repeat)."""
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


def _set(seed=50, n=48):
    specs = gen.selector_specs(seed=seed, n_jobs=n, size_lo=64 << 10, size_hi=2 << 20, c_hi=1 << 18)
    for sp in specs:
        if sp.kind == "words":
            sp.card = min(sp.card, 1 << 16)
    return specs, [gen.job_input(sp) for sp in specs]


def _entries(torch, specs, bufs):
    ents = []
    for sp, b in zip(specs, bufs):
        d = torch.from_numpy(b).to("cuda:0")
        if sp.kind == "words":
            ents.append({"kind": "words", "data": d, "cap_keys": min(len(b) // 2 + 1, sp.card + 16),
                         "cap_bytes": max(len(b), 1)})
        else:
            from paper_1309_0215_amd import _lib as L
            sumop = sp.op == "sum"
            n = len(b) // (8 if sumop else 4)
            ents.append({"kind": "u32_kv" if sumop else "u32", "data": d.view(torch.int32),
                         "op": L.REDUCE_SUM if sumop else L.REDUCE_COUNT,
                         "key_range": sp.card if sp.declare_range else 0, "cap_keys": max(1, min(n, sp.card))})
    return ents


def _expected(sp, b):
    if sp.kind == "words":
        e = oracle.words(b)
        return e.key_bytes, e.key_offsets, e.values
    w = b.view(np.uint32)
    if sp.op == "sum":
        k, v = oracle.u32(w[0::2], w[1::2], "sum")
    else:
        k, v = oracle.u32(w)
    return k, v


def _check(job_cls, res, sp, exp):
    if sp.kind == "words":
        kb, ko, v = exp
        assert np.array_equal(res.key_bytes.cpu().numpy(), kb)
        assert np.array_equal(res.key_offsets.cpu().numpy().astype(np.uint64), ko)
        assert np.array_equal(res.values.cpu().numpy().astype(np.uint32).astype(np.uint64), v)
    else:
        k, v = exp
        assert np.array_equal(res.keys.cpu().numpy().view(np.uint32), k)
        got = res.values.cpu().numpy()
        got = got.view(np.uint64) if got.dtype == np.int64 else got.view(np.uint32).astype(np.uint64)
        assert np.array_equal(got, v)


@pytest.mark.parametrize("learned", [False, True])
def test_mixed_batch_matches_oracle_and_single_runs(torch, learned):
    from paper_1309_0215_amd import Job, _lib as L, selector as S
    specs, bufs = _set()
    assert {sp.kind for sp in specs} == {"words", "u32"}
    exp = [_expected(sp, b) for sp, b in zip(specs, bufs)]
    strat = L.STRAT_LEARNED if learned else L.STRAT_RULE
    job = Job(device=0, strategy=strat)
    alone = Job(device=0, strategy=strat)
    if learned:
        S.load_model(job)
        S.load_model(alone)
    prep = job.batch_prepare_mixed(_entries(torch, specs, bufs))
    for rep in range(2):  # the repeat replays the selection graph and the word graph
        job.batch_run(prep)
        for i, sp in enumerate(specs):
            r = Job.batch_result(prep, i)
            _check(Job, r, sp, exp[i])
            if sp.kind == "u32" and learned:
                assert r.stats["selector_used"] in (0, 1)
    # each integer item's container equals the one mr_run picks for the job alone
    runner = S.Runner(torch)
    for i, sp in enumerate(specs):
        if sp.kind != "u32":
            continue
        d = prep[2][i]  # output tensors; compare the container used
        r = Job.batch_result(prep, i)
        out, keep = runner.outputs(sp, torch.from_numpy(bufs[i]).to("cuda:0").view(torch.int32))
        st, _ = runner.run(alone, sp, torch.from_numpy(bufs[i]).to("cuda:0").view(torch.int32), out)
        L.check(st, "alone")
        assert out.stats.strategy_used == r.stats["strategy_used"], i
        assert out.stats.selector_used == r.stats["selector_used"], i
    if learned:
        assert any(Job.batch_result(prep, i).stats["selector_used"] for i, sp in enumerate(specs) if sp.kind == "u32")
