"""GPU parity of the Bloom filter build (benchmark application "Bloom
Filter": 30 million k-mers into 300 million bits, one large global array
instead of per-worker local arrays, Section III-E).

Every filter word is compared with the CPU oracle's, bit for bit:
* small inputs over several tiles and a ragged tail, with runs of N, for
  k-mer lengths 1..32, hash counts 1..8 and filter sizes that are not
  multiples of 32 bits or of the 2^18-bit position ranges;
* inputs with no k-mer (shorter than k, or only N), and a single k-mer;
* the full workload: 30,000,019 bytes of synthetic DNA, k = 20, h = 7,
  m = 300,000,000 bits;
and the argument checks of the entry point.
"""
import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _gpu(torch, s, m, k=20, h=7):
    from paper_1309_0215_amd import Job
    d = torch.from_numpy(np.ascontiguousarray(s, np.uint8)).to("cuda:0")
    words, stats = Job(device=0, bloom_k=k, bloom_hashes=h).bloom(d, m)
    return words.cpu().numpy().view(np.uint32), stats


def _check(torch, s, m, k=20, h=7):
    gw, st = _gpu(torch, s, m, k, h)
    ew, n = oracle.bloom(s, m, k, h)
    assert len(gw) == len(ew)
    bad = np.flatnonzero(gw != ew)
    assert len(bad) == 0, f"{len(bad)} words differ, first at {bad[:4]}"
    assert st["n_items"] == max(len(s) - k + 1, 0)
    return n


@pytest.mark.parametrize("n,m,k,h,seed", [
    (100_000, 1_000_003, 20, 7, 1),
    (2048 + 19, 4096, 20, 7, 2),          # exactly one tile of k-mers plus the k - 1 bytes
    (2048 + 20, 4096, 20, 7, 3),          # one k-mer into a second tile
    (333_333, (1 << 19) * 3 + 17, 31, 8, 4),
    (333_333, 300_001, 32, 3, 5),
    (50_001, 77, 1, 1, 6),
    (250_000, 5_000_000, 12, 5, 7),
    (1_000_000, 1 << 29, 20, 7, 8),      # the largest filter
])
def test_small_inputs_every_word(torch, n, m, k, h, seed):
    s = gen.dna(seed, n, n_rate=1e-3)
    _check(torch, s, m, k, h)


def test_no_kmer_and_single_kmer(torch):
    m = 100_003
    s = gen.dna(9, 40, n_rate=0)
    assert _check(torch, s[:19], m) == 0                      # shorter than k: filter all clear
    assert _check(torch, np.full(5000, ord("N"), np.uint8), m) == 0
    assert _check(torch, s[:20], m) == 1
    assert _check(torch, np.frombuffer(b"A" * 64, np.uint8), 300_000_000) == 45  # fmix64(0) = 0: only bit 0


def test_lowercase_and_other_bytes_emit_nothing(torch):
    s = np.frombuffer(b"acgtACGTNacgtRYACGTACGTACGTACGTACGTACGTAC" * 100, np.uint8)
    _check(torch, s, 65_537, k=8, h=4)


def test_full_workload_30m_kmers_300m_bits(torch):
    s = gen.dna(20, 30_000_019)
    n = _check(torch, s, 300_000_000, 20, 7)
    assert n > 29_900_000


def test_arguments_are_checked(torch):
    from paper_1309_0215_amd import Job, MRError
    d = torch.from_numpy(gen.dna(10, 1000)).to("cuda:0")
    with pytest.raises(MRError) as e:
        Job(device=0).bloom(d, 0)
    assert e.value.status == -1
    with pytest.raises(MRError) as e:
        Job(device=0).bloom(d, (1 << 29) + 1)
    assert e.value.status == -5
    with pytest.raises(MRError) as e:
        Job(device=0, bloom_k=33).bloom(d, 1000)
    assert e.value.status == -1
    with pytest.raises(MRError) as e:
        Job(device=0, bloom_hashes=9).bloom(d, 1000)
    assert e.value.status == -1


def test_capacity_is_reported(torch):
    import ctypes as C
    from paper_1309_0215_amd import Job, _lib as L
    d = torch.from_numpy(gen.dna(11, 1000)).to("cuda:0")
    job = Job(device=0)
    w = torch.empty(10, dtype=torch.int32, device="cuda:0")
    o = L.Output()
    o.values, o.cap_keys = w.data_ptr(), 10
    st = job.lib.mr_run(job.h, L.MAP_BLOOM, L.REDUCE_COUNT, d.data_ptr(), 1000, None, 0, 1000, C.byref(o))
    assert st == L.MR_ERR_CAPACITY and o.n_keys == 32
