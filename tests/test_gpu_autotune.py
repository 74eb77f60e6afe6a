"""GPU checks of tuned launch parameters (mr_tune_set).

* With the committed tuning loaded, word jobs in several size buckets, a
  batch, and uint32 jobs (hash table and declared ranges) give outputs
  identical to an untuned job's.
* A tuned load limit sets the planned table size (1 MiB of text: 65,536
  slots at 35%, 32,768 at 70%), and the job's own setting wins over it.
* Malformed entries are rejected and change nothing.
"""
import numpy as np
import pytest

import gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _same(a, b, torch):
    return (torch.equal(a.key_bytes, b.key_bytes) and torch.equal(a.key_offsets, b.key_offsets) and
            torch.equal(a.values, b.values))


def test_tuned_words_and_batch_match_untuned(torch):
    from paper_1309_0215_amd import Job
    tuned, plain = Job(device=0), Job(device=0)
    tuned.load_tuning()
    for seed, size in ((1, 100_000), (2, 1 << 20), (3, 8 << 20), (4, 40 << 20)):
        d = torch.from_numpy(gen.text(seed, size, V=20_000)).to("cuda:0")
        assert _same(tuned.words(d), plain.words(d), torch), size
    specs = gen.batched_specs(seed=9, n_jobs=40)
    dev = [torch.from_numpy(b).to("cuda:0") for b in gen.job_inputs(specs)]
    for a, b in zip(tuned.words_batch(dev), plain.words_batch(dev)):
        assert _same(a, b, torch)


def test_tuned_u32_matches_untuned(torch):
    from paper_1309_0215_amd import Job
    tuned, plain = Job(device=0), Job(device=0)
    tuned.set_tuning([dict(kind="u32", bytes_lo=0, bytes_hi=1 << 62, max_load_pct=35, lds_array_bytes=16384)])
    for card, R in ((100_000, 0), (6_000, 6_000), (12_000, 12_000)):
        keys, _ = gen.u32_keys(31 + card, 1 << 20, card, 1.0)
        k = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
        a, b = tuned.u32(k, key_range=R), plain.u32(k, key_range=R)
        assert torch.equal(a.keys, b.keys) and torch.equal(a.values, b.values)
        if R:  # the tuned LDS budget (16 KiB) sends these ranges to the global array
            assert a.stats["strategy_used"] == 3 and b.stats["strategy_used"] == 2


def test_load_limit_sets_the_table_and_config_wins(torch):
    from paper_1309_0215_amd import Job
    d = torch.from_numpy(gen.text(5, 1 << 20, V=2000)).to("cuda:0")
    slots = {}
    for pct in (35, 70):
        job = Job(device=0)
        job.set_tuning([dict(kind="words", bytes_lo=0, bytes_hi=1 << 62, max_load_pct=pct)])
        slots[pct] = job.words(d).stats["table_slots"]
    assert slots == {35: 65536, 70: 32768}
    job = Job(device=0, max_load_pct=70)
    job.set_tuning([dict(kind="words", bytes_lo=0, bytes_hi=1 << 62, max_load_pct=35)])
    assert job.words(d).stats["table_slots"] == 32768


def test_malformed_entries_are_rejected(torch):
    from paper_1309_0215_amd import Job, MRError
    job = Job(device=0)
    good = dict(kind="words", bytes_lo=0, bytes_hi=1 << 62)
    for bad in (dict(lds_slots=512), dict(max_load_pct=99), dict(map_grid_pct=101), dict(lds_array_bytes=1 << 17),
                dict(bytes_lo=5, bytes_hi=5)):
        with pytest.raises(MRError) as e:
            job.set_tuning([{**good, **bad}])
        assert e.value.status == -1
    job.set_tuning([])
