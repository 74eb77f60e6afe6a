"""Pins of the Reverse Index oracle (benchmark application "Reverse Index":
URL -> files that link to it, hash table container).

A link is the nine bytes <a href=" then 1 to 4095 bytes other than a double
quote, then a double quote, all inside one record (file); the URL is the
bytes between the quotes. The pins do not come from the oracle's code:
* hand-worked cases in tests/golden/links_hand.json (near misses, empty URL,
  missing quote, duplicates in one file, record boundaries, byte order);
* a regular expression over each record (Python's re engine) as brute force
  on random inputs built from markers, near misses, quotes and URL bytes;
* the synthetic HTML generator's planted links: the index built from the
  planted (file, URL) pairs, at an eighth of the workload's size;
* URL length limits 4095 / 4096 and malformed record offsets.
"""
import json
import os
import re
from collections import defaultdict

import numpy as np
import pytest

import gen
import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
# every start position is tried (a zero-width lookahead), as links may overlap:
# the last quote of one marker can close the URL of an earlier one
LINK = re.compile(rb'(?=<a href="([^"]{1,4095})")')


def _records(strs):
    bs = [s.encode("latin-1") for s in strs]
    buf = np.frombuffer(b"".join(bs), np.uint8) if any(bs) else np.zeros(0, np.uint8)
    rec = np.cumsum([0] + [len(b) for b in bs]).astype(np.uint64)
    return buf, rec


def _brute(buf, rec):
    idx = defaultdict(lambda: [0, []])
    raw = buf.tobytes()
    for f in range(len(rec) - 1):
        for m in LINK.finditer(raw[int(rec[f]):int(rec[f + 1])]):
            e = idx[m.group(1)]
            e[0] += 1
            if not e[1] or e[1][-1] != f:
                e[1].append(f)
    return [(k, v[0], v[1]) for k, v in sorted(idx.items())]


def test_hand_cases():
    cases = json.load(open(os.path.join(HERE, "golden", "links_hand.json")))["cases"]
    for c in cases:
        buf, rec = _records(c["records"])
        got = oracle.links(buf, rec).items()
        want = [(u.encode("latin-1"), n, ids) for u, n, ids in c["expect"]]
        assert got == want, c["name"]


def test_regex_brute_force_on_random_inputs():
    rng = np.random.default_rng(7)
    frags = [b'<a href="', b'"', b'<A HREF="', b"<a href='", b"<a href=", b"x", b"ab", b"/", b" ", b"\xff", b"\x00",
             b"<", b'<a href="u', b'">']
    for trial in range(200):
        parts = [frags[i] for i in rng.integers(0, len(frags), size=int(rng.integers(0, 80)))]
        raw = b"".join(parts)
        buf = np.frombuffer(raw, np.uint8) if raw else np.zeros(0, np.uint8)
        cuts = np.sort(rng.integers(0, len(raw) + 1, size=int(rng.integers(0, 4))))
        rec = np.concatenate([[0], cuts, [len(raw)]]).astype(np.uint64)
        assert oracle.links(buf, rec).items() == _brute(buf, rec), trial
        assert oracle.links(buf).items() == _brute(buf, np.array([0, len(raw)], np.uint64))


def test_url_length_limit():
    for L, ok in ((4095, True), (4096, False), (1, True)):
        raw = b'<a href="' + b"u" * L + b'">'
        r = oracle.links(np.frombuffer(raw, np.uint8)).items()
        assert (r == [(b"u" * L, 1, [0])]) if ok else (r == [])


def test_malformed_offsets_rejected():
    buf = np.frombuffer(b'<a href="x">', np.uint8)
    with pytest.raises(ValueError):
        oracle.links(buf, np.array([0, 9, 5], np.uint64))
    with pytest.raises(ValueError):
        oracle.links(buf, np.array([0, 99], np.uint64))


def test_planted_links_of_generated_html():
    """The generated files hold exactly the planted links; the index built
    from the planted pairs must equal the oracle's."""
    h = gen.html(2, n_files=78_355 // 8, n_links=307_921 // 8, size=(1 << 30) // 8)
    r = oracle.links(h.buf, h.rec)
    idx = defaultdict(lambda: [0, set()])
    for f, u in zip(h.link_file.tolist(), h.link_url.tolist()):
        e = idx[h.urls[u]]
        e[0] += 1
        e[1].add(f)
    want = [(k, v[0], sorted(v[1])) for k, v in sorted(idx.items())]
    assert r.items() == want
    assert int(r.counts.sum()) == len(h.link_file)
