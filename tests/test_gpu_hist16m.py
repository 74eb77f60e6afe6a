"""GPU parity of the large-range histogram (the paper's Histogram workload:
2^24 possible keys, 2^28 uint32 input elements, reduced into one global array
with atomics instead of per-worker local arrays, Section III-E).

* 2^22 elements over 2^24 keys: every output (key, count) against the CPU
  oracle, with the rule's container (global array) and with the hash table
  and the sort forced.
* The full 2^28 elements: every one of the 2^24 bins against np.bincount.
* Skewed inputs through the key-range partitions: most elements on one key
  (one range's segment holds nearly all of them), keys on the range
  boundaries, and an input of a single key.
* Inputs off the fast tile path: a partial last tile, keys 4 bytes past a
  16-byte boundary, and (key, value) pairs.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

R = 1 << 24
GLOBAL_ARRAY, HASH, SORT = 3, 4, 5


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _run(torch, strategy, keys):
    from paper_1309_0215_amd import Job
    kt = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
    res = Job(device=0, strategy=strategy).u32(kt, key_range=R)
    del kt
    return res


@pytest.mark.parametrize("strategy", [0, HASH, SORT])
def test_2p22_elements_every_key(torch, strategy):
    keys = gen.uniform_keys(21, 1 << 22, R)
    res = _run(torch, strategy, keys)
    assert res.stats["strategy_used"] == (GLOBAL_ARRAY if strategy == 0 else strategy)
    ek, ev = oracle.u32(keys)
    assert np.array_equal(res.keys.cpu().numpy().view(np.uint32), ek)
    assert np.array_equal(res.values.cpu().numpy().view(np.uint32).astype(np.uint64), ev)


def test_full_2p28_elements():
    """Every one of the 2^24 bins against np.bincount of the 2^28 keys."""
    import torch
    n = 1 << 28
    keys = gen.uniform_keys(22, n, R)
    res = _run(torch, 0, keys)
    assert res.stats["strategy_used"] == GLOBAL_ARRAY
    gk = res.keys.cpu().numpy().view(np.uint32)
    gv = res.values.cpu().numpy().view(np.uint32).astype(np.uint64)
    counts = np.bincount(keys, minlength=R).astype(np.uint64)
    ek = np.flatnonzero(counts).astype(np.uint32)
    assert np.array_equal(gk, ek)
    assert np.array_equal(gv, counts[ek])
    assert int(gv.sum()) == n


def test_key_outside_the_range_is_rejected(torch):
    from paper_1309_0215_amd import Job, MRError
    keys = gen.uniform_keys(24, 1 << 21, R)
    keys[123457] = R  # one key at the declared range
    kt = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
    with pytest.raises(MRError) as e:
        Job(device=0).u32(kt, key_range=R)
    assert e.value.status == -1


def test_pairs_count_and_ragged_range(torch):
    """(key, value) pairs with COUNT, and a range that is not a multiple of 2^14."""
    from paper_1309_0215_amd import Job
    Rr = (1 << 20) + 12345
    keys = gen.uniform_keys(25, (1 << 20) + 77, Rr)
    vals = np.arange(len(keys), dtype=np.uint32)
    d = lambda a: torch.from_numpy(a.view(np.int32)).to("cuda:0")  # noqa: E731
    res = Job(device=0).u32(d(keys), d(vals), op=0, key_range=Rr)
    assert res.stats["strategy_used"] == GLOBAL_ARRAY
    ek, ev = oracle.u32(keys)
    assert np.array_equal(res.keys.cpu().numpy().view(np.uint32), ek)
    assert np.array_equal(res.values.cpu().numpy().view(np.uint32).astype(np.uint64), ev)


@pytest.mark.parametrize("share", [0.9, 1.0])
def test_skewed_keys_through_the_partitions(torch, share):
    """A share of the 2^22 elements on one key of the last 2^15-key range,
    keys on both sides of every range boundary, the rest uniform."""
    n = 1 << 22
    rng = np.random.default_rng(26)
    keys = gen.uniform_keys(26, n, R)
    hot = rng.random(n) < share
    keys[hot] = R - 5
    if share < 1.0:
        edges = np.arange(1, R >> 15, dtype=np.uint32) << 15
        keys[:len(edges)] = edges
        keys[len(edges):2 * len(edges)] = edges - 1
    res = _run(torch, 0, keys)
    assert res.stats["strategy_used"] == GLOBAL_ARRAY
    ek, ev = oracle.u32(keys)
    assert np.array_equal(res.keys.cpu().numpy().view(np.uint32), ek)
    assert np.array_equal(res.values.cpu().numpy().view(np.uint32).astype(np.uint64), ev)


@pytest.mark.parametrize("offset", [0, 1])
def test_ragged_and_unaligned_inputs(torch, offset):
    """Plain keys whose last 16K-element tile is partial (offset 0: the whole
    tiles are held in registers, the last one is read twice), and the same
    keys starting 4 bytes past a 16-byte boundary (offset 1: every tile takes
    the path that reads it twice, one key at a time)."""
    from paper_1309_0215_amd import Job
    n = (1 << 22) + 77
    keys = gen.uniform_keys(27, n + 1, R)
    kt = torch.from_numpy(keys.view(np.int32)).to("cuda:0")
    view = kt[offset:offset + n]
    assert (view.data_ptr() % 16 == 0) == (offset == 0)
    res = Job(device=0).u32(view, key_range=R)
    assert res.stats["strategy_used"] == GLOBAL_ARRAY
    ek, ev = oracle.u32(keys[offset:offset + n])
    assert np.array_equal(res.keys.cpu().numpy().view(np.uint32), ek)
    assert np.array_equal(res.values.cpu().numpy().view(np.uint32).astype(np.uint64), ev)
