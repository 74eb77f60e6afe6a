"""MI355X (gfx950) MapReduce hot path: thin Python binding over libmr.so.

Every step of the path runs in the library's HIP kernels. This module only
marshals arguments: torch CUDA tensors provide device memory and the stream.
There is no CPU fallback; without the built library every call raises.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

from . import _lib as L
from ._lib import MRError  # noqa: F401

__all__ = ["Job", "WordsResult", "U32Result", "MRError", "load", "workspace_bytes"]


def load():
    return L.load(required=True)


def _ptr(t) -> int | None:
    if t is None:
        return None
    return t.data_ptr()


def _stream_handle(torch, device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


@dataclass
class WordsResult:
    key_bytes: "object"     # torch.uint8 [key_bytes_used]
    key_offsets: "object"   # torch.int64 [n + 1] (uint64 bit pattern)
    values: "object"        # torch.int32 [n] (uint32 bit pattern)
    stats: dict

    def __len__(self):
        return int(self.values.numel())

    def items(self):
        kb = self.key_bytes.cpu().numpy().tobytes()
        o = self.key_offsets.cpu().numpy().astype("uint64")
        v = self.values.cpu().numpy().astype("uint32")
        return [(kb[o[i]:o[i + 1]], int(v[i])) for i in range(len(v))]


@dataclass
class U32Result:
    keys: "object"
    values: "object"
    stats: dict


def _stats(o: L.Output) -> dict:
    s = o.stats
    return {"strategy_used": s.strategy_used, "retries": s.retries, "table_slots": s.table_slots,
            "n_items": s.n_items, "gpu_ms": s.gpu_ms, "map_ms": s.map_ms, "km_rechecked": s.km_rechecked,
            "selector_used": s.selector_used, "device_allocs": s.device_allocs, "sort_spills": s.sort_spills,
            "workspace_needed": s.workspace_needed}


TUNE_KINDS = {"words": L.MAP_WORDS, "u32": L.MAP_U32_KEYS, "u32_kv": L.MAP_U32_KV}
TUNE_FIELDS = ("lds_slots", "max_load_pct", "map_grid_pct", "lds_array_bytes")


def tune_entries(entries):
    """mr_tune_entry array from dicts with keys kind ("words", "u32" or
    "u32_kv"), bytes_lo, bytes_hi and any of TUNE_FIELDS (missing = 0, the
    default)."""
    arr = (L.TuneEntry * max(1, len(entries)))()
    for i, e in enumerate(entries):
        arr[i].kind = TUNE_KINDS[e["kind"]]
        arr[i].bytes_lo, arr[i].bytes_hi = int(e["bytes_lo"]), int(e["bytes_hi"])
        for f in TUNE_FIELDS:
            setattr(arr[i], f, int(e.get(f, 0)))
    return arr


@dataclass
class LinksResult:
    """Reverse index on the device: URLs (key_bytes, key_offsets), link counts,
    and the file lists (list_ids[list_offsets[i]:list_offsets[i + 1]])."""
    key_bytes: object
    key_offsets: object
    counts: object
    list_offsets: object
    list_ids: object
    stats: dict

    def __len__(self):
        return int(self.counts.numel())

    def items(self):
        kb = self.key_bytes.cpu().numpy().tobytes()
        o = self.key_offsets.cpu().numpy()
        c = self.counts.cpu().numpy().view("uint32")
        lo = self.list_offsets.cpu().numpy()
        ids = self.list_ids.cpu().numpy().view("uint32")
        return [(kb[o[i]:o[i + 1]], int(c[i]), ids[lo[i]:lo[i + 1]].tolist()) for i in range(len(c))]


def workspace_bytes(kind: int, input_bytes: int, key_range: int = 0, device: int = 0, strategy: int = L.STRAT_RULE,
                    km_k: int = 0, km_d: int = 0, bloom_k: int = 0, bloom_hashes: int = 0) -> int:
    """mr_workspace_bytes: device bytes an mr_run of `kind` needs for inputs of up to input_bytes."""
    lib = load()
    cfg = L.JobConfig()
    cfg.device, cfg.strategy, cfg.km_k, cfg.km_d = device, strategy, km_k, km_d
    cfg.bloom_k, cfg.bloom_hashes = bloom_k, bloom_hashes
    out = C.c_uint64(0)
    L.check(lib.mr_workspace_bytes(C.byref(cfg), kind, input_bytes, key_range, C.byref(out)), "mr_workspace_bytes")
    return int(out.value)


class Job:
    """One mr_job bound to a device and to that device's current torch stream."""

    def __init__(self, device: int = 0, strategy: int = L.STRAT_RULE, lds_slots: int = 0, max_load_pct: int = 0,
                 debug_hash: int = 0, table_slots: int = 0, km_centroids=None, stream=None, timing: int = 0,
                 bloom_k: int = 0, bloom_hashes: int = 0, wave_combine: int = 0, workspace=None):
        import torch
        self.torch = torch
        self.lib = load()
        self.device = device
        cfg = L.JobConfig()
        cfg.device = device
        cfg.stream = stream if stream is not None else _stream_handle(torch, device)
        cfg.strategy = strategy
        cfg.lds_slots = lds_slots
        cfg.max_load_pct = max_load_pct
        cfg.debug_hash = debug_hash
        cfg.table_slots = table_slots
        cfg.timing = timing
        cfg.bloom_k = bloom_k
        cfg.bloom_hashes = bloom_hashes
        cfg.wave_combine = wave_combine
        # a caller workspace (uint8 CUDA tensor): the library then allocates no device memory
        self._ws = workspace
        if workspace is not None:
            cfg.workspace = workspace.data_ptr()
            cfg.workspace_bytes = int(workspace.numel()) * int(workspace.element_size())
        self._km = None
        if km_centroids is not None:
            c = km_centroids.to(device=f"cuda:{device}", dtype=torch.float32).contiguous()
            cfg.km_k, cfg.km_d = int(c.shape[0]), int(c.shape[1])
            cfg.km_centroids = c.data_ptr()
            self._km = c
        self.cfg = cfg
        h = C.c_void_p()
        L.check(self.lib.mr_job_create(C.byref(cfg), C.byref(h)), "mr_job_create")
        self.h = h

    def set_tuning(self, entries):
        """Tuned launch parameters (see tune_entries); an empty list clears them."""
        L.check(self.lib.mr_tune_set(self.h, tune_entries(entries), len(entries)), "mr_tune_set")

    def load_tuning(self, path: str | None = None):
        """Apply the entries of a tuning file written by paper_1309_0215_amd.autotune."""
        import json
        from .autotune import TUNING_PATH
        with open(path or TUNING_PATH) as f:
            self.set_tuning(json.load(f)["entries"])

    def close(self):
        if getattr(self, "h", None):
            self.lib.mr_job_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ words
    def _word_out(self, cap_keys: int, cap_bytes: int):
        torch = self.torch
        dev = f"cuda:{self.device}"
        kb = torch.empty(max(cap_bytes, 1), dtype=torch.uint8, device=dev)
        ko = torch.empty(cap_keys + 1, dtype=torch.int64, device=dev)
        vals = torch.empty(max(cap_keys, 1), dtype=torch.int32, device=dev)
        o = L.Output()
        o.key_bytes, o.key_offsets, o.values = kb.data_ptr(), ko.data_ptr(), vals.data_ptr()
        o.cap_keys, o.cap_key_bytes = cap_keys, cap_bytes
        return o, (kb, ko, vals)

    def words(self, data, record_offsets=None, cap_keys: int | None = None, cap_bytes: int | None = None) -> WordsResult:
        """Word count of a uint8 CUDA tensor; record_offsets is an int64 CUDA tensor [n + 1] or None."""
        n = int(data.numel())
        if cap_keys is None:
            cap_keys = max(1024, min(n // 2 + 1, 1 << 20))
        if cap_bytes is None:
            cap_bytes = max(4096, min(n, 1 << 24))
        for _ in range(2):
            o, keep = self._word_out(cap_keys, cap_bytes)
            ro = None if record_offsets is None else record_offsets
            st = self.lib.mr_run(self.h, L.MAP_WORDS, L.REDUCE_COUNT, _ptr(data), n, _ptr(ro),
                                 0 if ro is None else int(ro.numel()) - 1, 0, C.byref(o))
            if st == L.MR_ERR_CAPACITY and (o.n_keys > cap_keys or o.key_bytes_used > cap_bytes):
                cap_keys, cap_bytes = int(o.n_keys), int(o.key_bytes_used)
                continue
            L.check(st, "mr_run(words)")
            kb, ko, vals = keep
            nk = int(o.n_keys)
            return WordsResult(kb[:o.key_bytes_used], ko[:nk + 1], vals[:nk], _stats(o))
        raise MRError(L.MR_ERR_CAPACITY, "output capacity retry failed")

    def words_raw(self, data, out: L.Output, record_offsets=None) -> int:
        """mr_run with caller-prepared output buffers; returns the status (for timing loops)."""
        ro = record_offsets
        return self.lib.mr_run(self.h, L.MAP_WORDS, L.REDUCE_COUNT, _ptr(data), int(data.numel()), _ptr(ro),
                               0 if ro is None else int(ro.numel()) - 1, 0, C.byref(out))

    def words_batch(self, inputs, cap_keys: list[int] | None = None, cap_bytes: list[int] | None = None,
                    record_offsets: list | None = None, prepared=None):
        """One mr_batch_run over a list of uint8 CUDA tensors; returns a list of WordsResult.

        `prepared` (from batch_prepare) reuses item and output arrays, so that
        repeated calls keep the same launch layout and replay the captured graph."""
        if prepared is not None:
            items, outs, keep = prepared
            n = len(keep)
            L.check(self.lib.mr_batch_run(self.h, items, n, outs), "mr_batch_run")
            return [WordsResult(keep[i][0][:outs[i].key_bytes_used], keep[i][1][:int(outs[i].n_keys) + 1],
                                keep[i][2][:int(outs[i].n_keys)], _stats(outs[i])) for i in range(n)]
        items, outs, keep = self.batch_prepare(inputs, cap_keys, cap_bytes, record_offsets)
        return self.words_batch(inputs, prepared=(items, outs, keep))

    def batch_prepare(self, inputs, cap_keys=None, cap_bytes=None, record_offsets=None):
        n = len(inputs)
        items = (L.BatchItem * n)()
        outs = (L.Output * n)()
        keep = []
        for i, d in enumerate(inputs):
            items[i].kind, items[i].op = L.MAP_WORDS, L.REDUCE_COUNT
            items[i].d_input, items[i].input_bytes = d.data_ptr(), int(d.numel())
            if record_offsets is not None and record_offsets[i] is not None:
                items[i].d_record_offsets = record_offsets[i].data_ptr()
                items[i].n_records = int(record_offsets[i].numel()) - 1
            ck = cap_keys[i] if cap_keys else max(1024, min(int(d.numel()) // 2 + 1, 1 << 20))
            cb = cap_bytes[i] if cap_bytes else max(4096, min(int(d.numel()), 1 << 24))
            o, k = self._word_out(ck, cb)
            outs[i] = o
            keep.append(k)
        return items, outs, keep

    def batch_prepare_mixed(self, entries):
        """Item and output arrays of a batch of word-count and integer-key jobs.

        Each entry is a dict: {"kind": "words", "data": uint8 tensor, "cap_keys",
        "cap_bytes"} or {"kind": "u32" | "u32_kv", "data": int32 tensor (keys,
        or interleaved (key, value) pairs), "op", "key_range", "cap_keys"}."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        n = len(entries)
        items = (L.BatchItem * n)()
        outs = (L.Output * n)()
        keep = []
        for i, e in enumerate(entries):
            d = e["data"]
            items[i].d_input, items[i].input_bytes = d.data_ptr(), int(d.numel()) * int(d.element_size())
            if e["kind"] == "words":
                items[i].kind, items[i].op = L.MAP_WORDS, L.REDUCE_COUNT
                ck = e.get("cap_keys") or max(1024, min(int(d.numel()) // 2 + 1, 1 << 20))
                cb = e.get("cap_bytes") or max(4096, min(int(d.numel()), 1 << 24))
                o, k = self._word_out(ck, cb)
            else:
                items[i].kind = L.MAP_U32_KV if e["kind"] == "u32_kv" else L.MAP_U32_KEYS
                items[i].op = e.get("op", L.REDUCE_COUNT)
                items[i].key_range = e.get("key_range", 0)
                ck = max(1, e["cap_keys"])
                kt = torch.empty(ck, dtype=torch.int32, device=dev)
                vt = torch.empty(ck, dtype=torch.int64 if items[i].op == L.REDUCE_SUM else torch.int32, device=dev)
                o = L.Output()
                o.keys, o.values, o.cap_keys = kt.data_ptr(), vt.data_ptr(), ck
                k = (kt, vt)
            outs[i] = o
            keep.append(k)
        return items, outs, keep

    def batch_run(self, prepared, check: bool = True):
        """One mr_batch_run over prepared items; returns the status (MR_OK unless check is False)."""
        items, outs, keep = prepared
        st = self.lib.mr_batch_run(self.h, items, len(keep), outs)
        if check:
            L.check(st, "mr_batch_run")
        return st

    @staticmethod
    def batch_result(prepared, i):
        """Result of item i of a run batch: WordsResult or U32Result."""
        items, outs, keep = prepared
        o, nk = outs[i], int(outs[i].n_keys)
        if items[i].kind == L.MAP_WORDS:
            return WordsResult(keep[i][0][:o.key_bytes_used], keep[i][1][:nk + 1], keep[i][2][:nk], _stats(o))
        return U32Result(keep[i][0][:nk], keep[i][1][:nk], _stats(o))

    def hash_words(self, data, stream: bool = True, units: int = 64, block: int = 4096, schedule: bool = False):
        """mr_hash_words: FNV-1a 64 of every word of a uint8 CUDA tensor, in
        input order; returns (hashes as int64, schedule [n][3] int32 or None,
        kernel ms)."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        nb = int(data.numel())
        cap = nb // 2 + 1
        h = torch.empty(cap, dtype=torch.int64, device=dev)
        sch = torch.empty(cap, 3, dtype=torch.int32, device=dev) if schedule else None
        n = C.c_uint64(0)
        ms = C.c_float(0.0)
        L.check(self.lib.mr_hash_words(self.h, _ptr(data), nb, 1 if stream else 0, units, block, h.data_ptr(),
                                       None if sch is None else sch.data_ptr(), cap, C.byref(n), C.byref(ms)),
                "mr_hash_words")
        k = int(n.value)
        return h[:k], (None if sch is None else sch[:k]), float(ms.value)

    # -------------------------------------------------------------- histogram
    def rgb_hist(self, data, out=None):
        """768 bins (3 x 256, uint64 counts as int64) of interleaved RGB bytes.

        out: optional int64 CUDA tensor of 768 elements to write the bins
        into; a repeated call on the same input, size and output replays a
        captured HIP graph."""
        torch = self.torch
        if out is None:
            out = torch.empty(768, dtype=torch.int64, device=f"cuda:{self.device}")
        elif out.dtype != torch.int64 or out.numel() != 768 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 tensor of 768 elements")
        o = L.Output()
        o.values = out.data_ptr()
        L.check(self.lib.mr_run(self.h, L.MAP_RGB_HIST, L.REDUCE_COUNT, _ptr(data), int(data.numel()), None, 0, 0,
                                C.byref(o)), "mr_run(rgb)")
        return out.view(3, 256), _stats(o)

    def rgb_hist_static(self, data, out):
        """mr_rgb_hist_static: the histogram into `out` (contiguous int64 CUDA
        tensor of 768) with the library's static scratch; enqueued on the job's
        stream, no allocation and no synchronisation."""
        torch = self.torch
        if out.dtype != torch.int64 or out.numel() != 768 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int64 tensor of 768 elements")
        L.check(self.lib.mr_rgb_hist_static(self.h, _ptr(data), int(data.numel()), out.data_ptr()),
                "mr_rgb_hist_static")
        return out.view(3, 256)

    # ------------------------------------------------------------- u32 keys
    def u32(self, keys, values=None, op: int = L.REDUCE_COUNT, key_range: int = 0, cap_keys: int | None = None):
        """keys: int32 CUDA tensor (uint32 bit pattern); values likewise or None.

        With values the input is interleaved (key, value) pairs, as mr_run expects."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        if values is not None:
            data = torch.stack([keys.view(torch.int32), values.view(torch.int32)], dim=1).contiguous()
            kind = L.MAP_U32_KV
        else:
            data = keys.view(torch.int32).contiguous()
            kind = L.MAP_U32_KEYS
        n = int(keys.numel())
        if cap_keys is None:
            cap_keys = max(1, min(n, key_range) if key_range else n)
        wide = op == L.REDUCE_SUM
        for _ in range(2):
            k = torch.empty(max(cap_keys, 1), dtype=torch.int32, device=dev)
            v = torch.empty(max(cap_keys, 1), dtype=torch.int64 if wide else torch.int32, device=dev)
            o = L.Output()
            o.keys, o.values, o.cap_keys = k.data_ptr(), v.data_ptr(), cap_keys
            st = self.lib.mr_run(self.h, kind, op, data.data_ptr(), data.numel() * 4, None, 0, key_range, C.byref(o))
            if st == L.MR_ERR_CAPACITY and o.n_keys > cap_keys:
                cap_keys = int(o.n_keys)
                continue
            L.check(st, "mr_run(u32)")
            nk = int(o.n_keys)
            return U32Result(k[:nk], v[:nk], _stats(o))
        raise MRError(L.MR_ERR_CAPACITY, "output capacity retry failed")

    # -------------------------------------------------------------- k-means
    def kmeans(self, X):
        """One Lloyd step on float32 CUDA tensor X [n, d] from the job's current centroids."""
        torch = self.torch
        if self._km is None:
            raise ValueError("job was created without k-means centroids")
        k, d = self._km.shape
        n = int(X.shape[0])
        dev = f"cuda:{self.device}"
        assign = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
        sums = torch.empty(k, d, dtype=torch.float32, device=dev)
        counts = torch.empty(k, dtype=torch.int32, device=dev)
        cents = torch.empty(k, d, dtype=torch.float32, device=dev)
        o = L.Output()
        o.assign, o.sums, o.counts, o.centroids = assign.data_ptr(), sums.data_ptr(), counts.data_ptr(), cents.data_ptr()
        L.check(self.lib.mr_run(self.h, L.MAP_KMEANS, L.REDUCE_SUM, _ptr(X), n * d * 4, None, 0, 0, C.byref(o)),
                "mr_run(kmeans)")
        return assign[:n], sums, counts, cents, _stats(o)

    # ---------------------------------------------------------- Reverse Index
    def links(self, data, record_offsets=None, cap_keys: int | None = None, cap_bytes: int | None = None,
              cap_ids: int | None = None) -> "LinksResult":
        """Reverse index of uint8 CUDA tensor data; record_offsets (uint64 CUDA tensor) cut it into files."""
        torch = self.torch
        dev = f"cuda:{self.device}"
        n = int(data.numel())
        ro = record_offsets
        n_rec = int(ro.numel()) - 1 if ro is not None else 0
        ck = cap_keys if cap_keys is not None else max(16, n // 64)
        cb = cap_bytes if cap_bytes is not None else max(64, n // 8)
        ci = cap_ids if cap_ids is not None else max(16, n // 64)
        for _ in range(3):
            kb = torch.empty(max(cb, 1), dtype=torch.uint8, device=dev)
            ko = torch.empty(ck + 1, dtype=torch.int64, device=dev)
            v = torch.empty(max(ck, 1), dtype=torch.int32, device=dev)
            lo = torch.empty(ck + 1, dtype=torch.int64, device=dev)
            ids = torch.empty(max(ci, 1), dtype=torch.int32, device=dev)
            o = L.Output()
            o.key_bytes, o.key_offsets, o.values, o.cap_keys, o.cap_key_bytes = (kb.data_ptr(), ko.data_ptr(), v.data_ptr(),
                                                                                ck, cb)
            o.list_offsets, o.list_ids, o.cap_list_ids = lo.data_ptr(), ids.data_ptr(), ci
            st = self.lib.mr_run(self.h, L.MAP_LINKS, L.REDUCE_COUNT, _ptr(data), n, _ptr(ro), n_rec, 0, C.byref(o))
            if st == L.MR_ERR_CAPACITY:
                ck, cb, ci = max(ck, int(o.n_keys)), max(cb, int(o.key_bytes_used)), max(ci, int(o.n_list_ids))
                continue
            L.check(st, "mr_run(links)")
            nk, ni = int(o.n_keys), int(o.n_list_ids)
            return LinksResult(kb[:int(o.key_bytes_used)], ko[:nk + 1], v[:nk], lo[:nk + 1], ids[:ni], _stats(o))
        raise MRError(L.MR_ERR_CAPACITY, "output capacity retry failed")

    # ---------------------------------------------------------- Bloom filter
    def bloom(self, data, m: int):
        """Bloom filter of the k-mers of uint8 CUDA tensor data (DNA bytes) with m bits.

        Returns the filter as an int32 tensor of ceil(m / 32) words (bit b in
        bit b % 32 of word b / 32) and the stats."""
        torch = self.torch
        n_words = (int(m) + 31) // 32
        words = torch.empty(max(n_words, 1), dtype=torch.int32, device=f"cuda:{self.device}")
        o = L.Output()
        o.values, o.cap_keys = words.data_ptr(), n_words
        L.check(self.lib.mr_run(self.h, L.MAP_BLOOM, L.REDUCE_COUNT, _ptr(data), int(data.numel()), None, 0, int(m),
                                C.byref(o)), "mr_run(bloom)")
        return words[:n_words], _stats(o)
