"""Pins of the word-hashing oracle (Section III-C): FNV-1a 64 against its
published test vectors, the SIMDH-Stream schedule against the paper's worked
example, and schedule invariants."""
import json
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_fnv1a64_published_vectors():
    # the FNV reference test vectors for FNV-1a 64
    assert oracle.fnv1a64(b"") == 0xCBF29CE484222325
    assert oracle.fnv1a64(b"a") == 0xAF63DC4C8601EC8C
    assert oracle.fnv1a64(b"foobar") == 0x85944171F73967E8


def test_stream_schedule_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "stream_hash_example.json")))
    lens = [len(w) for w in g["strings"]]
    assert oracle.stream_schedule(lens, g["units"]) == g["stream"]


def test_word_spans_and_hashes():
    buf = np.frombuffer(b"  This is\tXeon\n\nPhi  a", np.uint8)
    offs, lens = oracle.word_spans(buf)
    assert offs.tolist() == [2, 7, 10, 16, 21] and lens.tolist() == [4, 2, 4, 3, 1]
    h = oracle.word_hashes(buf)
    assert h[4] == 0xAF63DC4C8601EC8C
    # the words agree with the word count
    wc = dict(oracle.words(buf).items())
    assert sorted(wc) == sorted({buf.tobytes()[o:o + l] for o, l in zip(offs.tolist(), lens.tolist())})


def test_schedule_invariants():
    rng = np.random.default_rng(3)
    for units in (1, 2, 7, 64):
        lens = rng.integers(0, 20, 500).tolist()
        for sched in (oracle.stream_schedule(lens, units), oracle.padding_schedule(lens, units)):
            per_unit = {}
            for (u, a, b), l in zip(sched, lens):
                assert 0 <= u < units and b - a == l  # len characters, then the terminator
                per_unit.setdefault(u, []).append((a, b))
            for iv in per_unit.values():  # a unit holds one string at a time
                iv.sort()
                assert all(iv[k][1] < iv[k + 1][0] for k in range(len(iv) - 1))
        st = oracle.stream_schedule(lens, units)
        # stream keeps every unit busy until the strings run out: the last
        # iteration is at most the padded schedule's
        assert max(b for _, _, b in st) <= max(b for _, _, b in oracle.padding_schedule(lens, units))
    # one unit: strictly one string after another
    assert oracle.stream_schedule([3, 0, 2], 1) == [[0, 1, 4], [0, 5, 5], [0, 6, 8]]
