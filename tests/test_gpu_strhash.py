"""Word hashing one character per lane per step (mr_hash_words): FNV-1a 64 of
every word against the oracle, and the lanes' schedules against the oracle's
SIMDH-Padding and SIMDH-Stream schedules, starting from the paper's worked
two-unit example."""
import json
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def job():
    from paper_1309_0215_amd import Job
    return Job(device=0)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _blocks(lens, units, block, stream):
    out = []
    for b0 in range(0, len(lens), block):
        f = oracle.stream_schedule if stream else oracle.padding_schedule
        out.extend(f(lens[b0:b0 + block], units))
    return out


def test_worked_example_two_units(job):
    g = json.load(open(os.path.join(GOLDEN, "stream_hash_example.json")))
    buf = np.frombuffer(" ".join(g["strings"]).encode(), np.uint8)
    h, sched, _ = job.hash_words(_dev(buf), stream=True, units=g["units"], schedule=True)
    assert sched.cpu().numpy().tolist() == g["stream"]
    assert h.cpu().numpy().view(np.uint64).tolist() == [oracle.fnv1a64(w.encode()) for w in g["strings"]]
    _, sched_p, _ = job.hash_words(_dev(buf), stream=False, units=g["units"], schedule=True)
    assert sched_p.cpu().numpy().tolist() == oracle.padding_schedule([len(w) for w in g["strings"]], g["units"])


@pytest.mark.parametrize("stream", [False, True])
@pytest.mark.parametrize("units,block", [(64, 4096), (7, 100), (1, 37)])
def test_hashes_and_schedules(job, stream, units, block):
    rng = np.random.default_rng(units)
    text = gen.text(31, 300_000, V=3000, s=1.0, lmin=1, lmax=24)
    raw = rng.integers(0, 256, 20_000, dtype=np.uint8)  # every separator, NUL and high bytes
    buf = np.concatenate([text, raw, text[:777]])
    h, sched, _ = job.hash_words(_dev(buf), stream=stream, units=units, block=block, schedule=True)
    assert np.array_equal(h.cpu().numpy().view(np.uint64), oracle.word_hashes(buf))
    _, lens = oracle.word_spans(buf)
    assert sched.cpu().numpy().tolist() == _blocks(lens.tolist(), units, block, stream)


def test_empty_and_all_separators(job):
    import torch
    for buf in (np.zeros(0, np.uint8), np.frombuffer(b" \n\t  \r", np.uint8)):
        d = _dev(buf) if len(buf) else torch.empty(0, dtype=torch.uint8, device="cuda:0")
        h, sched, _ = job.hash_words(d, schedule=True)
        assert h.numel() == 0 and sched.numel() == 0
