"""GPU parity of the Reverse Index (benchmark application "Reverse Index":
URL -> files that link to it; 78,355 files, 307,921 links, 1 GB).

Every output is compared with the CPU oracle: the URL bytes and offsets, the
link count of each URL and each URL's ascending list of distinct files.
* the hand-worked cases of tests/golden/links_hand.json;
* random inputs built from markers, near misses, quotes and URL bytes, cut
  into random records (overlapping links, links across record boundaries);
* URL lengths 16 / 17 (inline and global keys), 4095 / 4096 (the limit);
* an input that starts off a 16-byte boundary, no records, no links, empty;
* every key forced onto one hash (collision handling);
* generated HTML at an eighth of the workload, and the full workload;
* capacity reporting, and malformed record offsets.
"""
import json
import os

import numpy as np
import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    return t


def _dev(torch, a):
    return torch.from_numpy(np.array(a)).to("cuda:0")


def _gpu(torch, buf, rec=None, **kw):
    from paper_1309_0215_amd import Job
    d = _dev(torch, np.ascontiguousarray(buf, np.uint8))
    r = _dev(torch, np.asarray(rec, np.uint64).view(np.int64)) if rec is not None else None
    return Job(device=0, **{k: v for k, v in kw.items() if k in ("debug_hash", "table_slots")}).links(d, r)


def _check(torch, buf, rec=None, **kw):
    res = _gpu(torch, buf, rec, **kw)
    want = oracle.links(buf, rec)
    got = res.items()
    assert got == want.items()
    assert res.stats["n_items"] == int(want.counts.sum())
    return want


def _records(strs):
    bs = [s.encode("latin-1") for s in strs]
    buf = np.frombuffer(b"".join(bs), np.uint8).copy() if any(bs) else np.zeros(0, np.uint8)
    return buf, np.cumsum([0] + [len(b) for b in bs]).astype(np.uint64)


def test_hand_cases(torch):
    for c in json.load(open(os.path.join(HERE, "golden", "links_hand.json")))["cases"]:
        buf, rec = _records(c["records"])
        if len(buf) == 0:
            continue
        _check(torch, buf, rec)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_fragments(torch, seed):
    rng = np.random.default_rng(seed)
    frags = [b'<a href="', b'"', b'<A HREF="', b"<a href='", b"<a href=", b"x", b"ab", b"/", b" ", b"\xff", b"\x00",
             b"<", b'<a href="u', b'">', b"0123456789abcdef", b"http://example.com/"]
    parts = [frags[i] for i in rng.integers(0, len(frags), size=40_000)]
    buf = np.frombuffer(b"".join(parts), np.uint8).copy()
    cuts = np.sort(rng.integers(0, len(buf) + 1, size=300))
    rec = np.concatenate([[0], cuts, [len(buf)]]).astype(np.uint64)
    _check(torch, buf, rec)
    _check(torch, buf)


def test_url_lengths(torch):
    parts = []
    for L in (1, 15, 16, 17, 31, 32, 33, 4095, 4096, 5000):
        parts.append(b'<a href="' + bytes([97 + L % 26]) * L + b'"> ')
    buf = np.frombuffer(b"".join(parts) * 3, np.uint8).copy()
    w = _check(torch, buf)
    assert sorted(len(k) for k, _, _ in w.items()) == [1, 15, 16, 17, 31, 32, 33, 4095]


def test_unaligned_start_no_records_no_links(torch):
    from paper_1309_0215_amd import Job
    h = gen.html(5, n_files=200, n_links=900, size=1 << 20, V=500)
    full = _dev(torch, h.buf)
    for start in (1, 7, 15):  # device pointers off a 16-byte boundary
        res = Job(device=0).links(full[start:])
        assert res.items() == oracle.links(h.buf[start:]).items()
    _check(torch, np.frombuffer(b"no links here <a href=x> " * 1000, np.uint8).copy())
    res = Job(device=0).links(torch.empty(0, dtype=torch.uint8, device="cuda:0"))
    assert res.items() == []


def test_all_keys_collide(torch):
    h = gen.html(6, n_files=100, n_links=600, size=1 << 19, V=200)
    _check(torch, h.buf, h.rec, debug_hash=1)


def test_generated_eighth(torch):
    h = gen.html(2, n_files=78_355 // 8, n_links=307_921 // 8, size=(1 << 30) // 8)
    _check(torch, h.buf, h.rec)


def test_full_workload(torch):
    h = gen.html(3)
    w = _check(torch, h.buf, h.rec)
    assert int(w.counts.sum()) == 307_921 and len(h.rec) == 78_356


def test_capacity_and_bad_offsets(torch):
    import ctypes as C
    from paper_1309_0215_amd import Job, MRError, _lib as L
    h = gen.html(7, n_files=50, n_links=400, size=1 << 18, V=100)
    want = oracle.links(h.buf, h.rec)
    d = _dev(torch, h.buf)
    r = _dev(torch, h.rec.view(np.int64))
    job = Job(device=0)
    kb = torch.empty(1 << 16, dtype=torch.uint8, device="cuda:0")
    ko = torch.empty(1024, dtype=torch.int64, device="cuda:0")
    v = torch.empty(1024, dtype=torch.int32, device="cuda:0")
    lo = torch.empty(1024, dtype=torch.int64, device="cuda:0")
    ids = torch.empty(4, dtype=torch.int32, device="cuda:0")
    o = L.Output()
    o.key_bytes, o.key_offsets, o.values, o.cap_keys, o.cap_key_bytes = kb.data_ptr(), ko.data_ptr(), v.data_ptr(), 1023, 1 << 16
    o.list_offsets, o.list_ids, o.cap_list_ids = lo.data_ptr(), ids.data_ptr(), 4
    st = job.lib.mr_run(job.h, L.MAP_LINKS, L.REDUCE_COUNT, d.data_ptr(), len(h.buf), r.data_ptr(), len(h.rec) - 1, 0,
                        C.byref(o))
    assert st == L.MR_ERR_CAPACITY and o.n_list_ids == len(want.ids) and o.n_keys == len(want)
    bad = h.rec.copy()
    bad[10] = h.rec[-1]  # a file that starts after the next one
    with pytest.raises(MRError) as e:
        job.links(d, _dev(torch, bad.view(np.int64)))
    assert e.value.status == -1
