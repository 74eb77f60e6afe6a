"""Oracle: plain, slow CPU reference implementations. TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library never imports, links or calls it, and
it shares no code with the GPU library.

* Word count, integer-key reduce, the RGB histogram, the Reverse Index and
  the Bloom filter build run in a small C++
  library (oracle.cpp, built with g++) that follows the paper's programming
  model (Section II-A): map every input element, reduce all pairs with equal
  keys, output in key order.
* One k-means step (assign + update) and the strategy-selector MLP are written
  here in float64 numpy. Neither appears in the paper; they follow their
  textbook definitions (Lloyd's step; a fully connected ReLU network trained
  with masked mean squared error and Adam).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile oracle.cpp with g++ into liboracle.so (plain -O2, no GPU code)."""
    src = os.path.join(_HERE, "oracle.cpp")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + ".tmp"
        subprocess.check_call(["g++", "-std=c++17", "-O2", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        build()
        lib = C.CDLL(_SO)
        P, U64, I = C.c_void_p, C.c_uint64, C.c_int
        lib.oracle_words_run.restype = P
        lib.oracle_words_run.argtypes = [P, U64, P, U64]
        lib.oracle_words_n.restype = U64
        lib.oracle_words_n.argtypes = [P]
        lib.oracle_words_bytes.restype = U64
        lib.oracle_words_bytes.argtypes = [P]
        lib.oracle_words_copy.argtypes = [P, P, P, P]
        lib.oracle_words_free.argtypes = [P]
        lib.oracle_u32_run.restype = P
        lib.oracle_u32_run.argtypes = [P, P, U64, I]
        lib.oracle_u32_n.restype = U64
        lib.oracle_u32_n.argtypes = [P]
        lib.oracle_u32_copy.argtypes = [P, P, P]
        lib.oracle_u32_free.argtypes = [P]
        lib.oracle_rgb_run.argtypes = [P, U64, P]
        lib.oracle_links_run.restype = P
        lib.oracle_links_run.argtypes = [P, U64, P, U64]
        for f in ("oracle_links_n", "oracle_links_bytes", "oracle_links_ids"):
            getattr(lib, f).restype = U64
            getattr(lib, f).argtypes = [P]
        lib.oracle_links_copy.argtypes = [P, P, P, P, P, P]
        lib.oracle_links_free.argtypes = [P]
        lib.oracle_fmix64.restype = U64
        lib.oracle_fmix64.argtypes = [U64]
        lib.oracle_bloom_run.restype = U64
        lib.oracle_bloom_run.argtypes = [P, U64, C.c_uint32, C.c_uint32, U64, P]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ----------------------------------------------------------------------------
# word count
# ----------------------------------------------------------------------------

class WordsResult:
    """Sorted distinct words: key_bytes (concatenated), key_offsets (n+1), values (u64)."""

    def __init__(self, key_bytes, key_offsets, values):
        self.key_bytes = key_bytes
        self.key_offsets = key_offsets
        self.values = values

    def __len__(self):
        return len(self.values)

    def items(self):
        kb = self.key_bytes.tobytes()
        o = self.key_offsets
        return [(kb[o[i]:o[i + 1]], int(self.values[i])) for i in range(len(self.values))]


def words(buf: np.ndarray, record_offsets: np.ndarray | None = None) -> WordsResult:
    """Word count over `buf` (uint8). Raises ValueError on malformed offsets."""
    lib = _load()
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    if record_offsets is not None:
        record_offsets = np.ascontiguousarray(record_offsets, dtype=np.uint64)
        n_rec = len(record_offsets) - 1
        if n_rec < 0:
            raise ValueError("record offsets need at least one entry")
    else:
        n_rec = 0
    h = lib.oracle_words_run(_ptr(buf), len(buf), _ptr(record_offsets), n_rec)
    if not h:
        raise ValueError("malformed record offsets")
    try:
        n = lib.oracle_words_n(h)
        nb = lib.oracle_words_bytes(h)
        kb = np.empty(nb, np.uint8)
        ko = np.empty(n + 1, np.uint64)
        v = np.empty(n, np.uint64)
        lib.oracle_words_copy(h, _ptr(kb), _ptr(ko), _ptr(v))
    finally:
        lib.oracle_words_free(h)
    return WordsResult(kb, ko, v)


# ----------------------------------------------------------------------------
# integer keys
# ----------------------------------------------------------------------------

OPS = {"count": 0, "sum": 1, "min": 2, "max": 3}


def u32(keys: np.ndarray, vals: np.ndarray | None = None, op: str = "count"):
    """Distinct keys ascending and their reduced values (u64)."""
    lib = _load()
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    if vals is not None:
        vals = np.ascontiguousarray(vals, dtype=np.uint32)
        assert len(vals) == len(keys)
    h = lib.oracle_u32_run(_ptr(keys), _ptr(vals), len(keys), OPS[op])
    try:
        n = lib.oracle_u32_n(h)
        k = np.empty(n, np.uint32)
        v = np.empty(n, np.uint64)
        lib.oracle_u32_copy(h, _ptr(k), _ptr(v))
    finally:
        lib.oracle_u32_free(h)
    return k, v


# ----------------------------------------------------------------------------
# RGB histogram
# ----------------------------------------------------------------------------

def rgb(buf: np.ndarray) -> np.ndarray:
    """uint64[3, 256] channel-major bins."""
    lib = _load()
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    bins = np.zeros(768, np.uint64)
    lib.oracle_rgb_run(_ptr(buf), len(buf), _ptr(bins))
    return bins.reshape(3, 256)


# ----------------------------------------------------------------------------
# Reverse Index
# ----------------------------------------------------------------------------

class LinksResult:
    """Sorted distinct URLs: key_bytes, key_offsets (n+1), counts (links per
    URL), list_offsets (n+1) and ids (files holding each URL, ascending)."""

    def __init__(self, key_bytes, key_offsets, counts, list_offsets, ids):
        self.key_bytes, self.key_offsets, self.counts = key_bytes, key_offsets, counts
        self.list_offsets, self.ids = list_offsets, ids

    def __len__(self):
        return len(self.counts)

    def items(self):
        kb = self.key_bytes.tobytes()
        o, lo = self.key_offsets, self.list_offsets
        return [(kb[o[i]:o[i + 1]], int(self.counts[i]), self.ids[lo[i]:lo[i + 1]].tolist())
                for i in range(len(self.counts))]


def links(buf: np.ndarray, record_offsets: np.ndarray | None = None) -> LinksResult:
    """Reverse index of the links in `buf` (uint8), records = files. Raises ValueError on malformed offsets."""
    lib = _load()
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    n_rec = 0
    if record_offsets is not None:
        record_offsets = np.ascontiguousarray(record_offsets, dtype=np.uint64)
        n_rec = len(record_offsets) - 1
        if n_rec < 0:
            raise ValueError("record offsets need at least one entry")
    h = lib.oracle_links_run(_ptr(buf), len(buf), _ptr(record_offsets), n_rec)
    if not h:
        raise ValueError("malformed record offsets")
    try:
        n, nb, ni = lib.oracle_links_n(h), lib.oracle_links_bytes(h), lib.oracle_links_ids(h)
        kb, ko, c = np.empty(nb, np.uint8), np.empty(n + 1, np.uint64), np.empty(n, np.uint64)
        lo, ids = np.empty(n + 1, np.uint64), np.empty(ni, np.uint32)
        lib.oracle_links_copy(h, _ptr(kb), _ptr(ko), _ptr(c), _ptr(lo), _ptr(ids))
    finally:
        lib.oracle_links_free(h)
    return LinksResult(kb, ko, c, lo, ids)


# ----------------------------------------------------------------------------
# Bloom filter build
# ----------------------------------------------------------------------------

def fmix64(x: int) -> int:
    """MurmurHash3's 64-bit finaliser, as the oracle computes it."""
    return int(_load().oracle_fmix64(int(x) & 0xFFFFFFFFFFFFFFFF))


def bloom(buf: np.ndarray, m: int, k: int = 20, h: int = 7) -> tuple[np.ndarray, int]:
    """Bloom filter of the valid k-mers of DNA bytes `buf`: (uint32 words[ceil(m/32)], k-mers inserted)."""
    lib = _load()
    buf = np.ascontiguousarray(buf, dtype=np.uint8)
    words = np.zeros((m + 31) // 32, np.uint32)
    n = lib.oracle_bloom_run(_ptr(buf), len(buf), k, h, m, _ptr(words))
    return words, int(n)


# ----------------------------------------------------------------------------
# k-means: one Lloyd step, float64 throughout
# ----------------------------------------------------------------------------

def kmeans_distances(X: np.ndarray, Cn: np.ndarray) -> np.ndarray:
    """Squared Euclidean distances d[i, j] = sum_t (x_it - c_jt)^2, direct form, float64."""
    X64 = np.asarray(X, np.float64)
    C64 = np.asarray(Cn, np.float64)
    out = np.empty((len(X64), len(C64)), np.float64)
    step = max(1, (1 << 22) // max(1, C64.size))
    for lo in range(0, len(X64), step):
        diff = X64[lo:lo + step, None, :] - C64[None, :, :]
        out[lo:lo + step] = (diff * diff).sum(axis=2)
    return out


def kmeans_assign(X: np.ndarray, Cn: np.ndarray) -> np.ndarray:
    """a_i = argmin_j d_ij; on an exact tie the lowest j wins (np.argmin takes the first)."""
    a = np.empty(len(X), np.int32)
    step = 1 << 16
    for lo in range(0, len(X), step):
        a[lo:lo + step] = np.argmin(kmeans_distances(X[lo:lo + step], Cn), axis=1)
    return a


def kmeans_update(X: np.ndarray, assign: np.ndarray, Cn: np.ndarray):
    """Per-cluster sums S (float64), counts n, and new centroids S/n (old centroid if empty)."""
    k, d = Cn.shape
    X64 = np.asarray(X, np.float64)
    S = np.zeros((k, d), np.float64)
    np.add.at(S, assign, X64)
    n = np.bincount(assign, minlength=k).astype(np.int64)
    newC = np.asarray(Cn, np.float64).copy()
    nz = n > 0
    newC[nz] = S[nz] / n[nz, None]
    return S, n, newC


def kmeans_abs_sums(X: np.ndarray, assign: np.ndarray, k: int) -> np.ndarray:
    """sum_i |x_id| per (cluster, dim): the scale used by the float32-sum tolerance."""
    A = np.zeros((k, X.shape[1]), np.float64)
    np.add.at(A, assign, np.abs(np.asarray(X, np.float64)))
    return A


def kmeans_step(X: np.ndarray, Cn: np.ndarray):
    a = kmeans_assign(X, Cn)
    S, n, newC = kmeans_update(X, a, Cn)
    return a, S, n, newC


# ----------------------------------------------------------------------------
# strategy-selector MLP: 12 -> 64 -> 64 -> 4, ReLU, masked MSE, Adam (float64)
# ----------------------------------------------------------------------------

MLP_SHAPES = [("W1", (64, 12)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (4, 64)), ("b3", (4,))]
MLP_NPARAM = sum(int(np.prod(s)) for _, s in MLP_SHAPES)


def mlp_unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shp in MLP_SHAPES:
        sz = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + sz], np.float64).reshape(shp)
        o += sz
    return out


def mlp_forward(theta: np.ndarray, X: np.ndarray):
    """Returns (y, cache). y[b] = W3 relu(W2 relu(W1 x_b + b1) + b2) + b3."""
    p = mlp_unpack(theta)
    X = np.asarray(X, np.float64)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, z1, h1, z2, h2)


def mlp_loss(theta: np.ndarray, X: np.ndarray, T: np.ndarray, M: np.ndarray) -> float:
    """Masked mean squared error: sum m (y - t)^2 / sum m."""
    y, _ = mlp_forward(theta, X)
    M = np.asarray(M, np.float64)
    return float((M * (y - T) ** 2).sum() / max(M.sum(), 1.0))


def mlp_grad(theta: np.ndarray, X: np.ndarray, T: np.ndarray, M: np.ndarray):
    """(loss, gradient) by the chain rule written out layer by layer."""
    p = mlp_unpack(theta)
    y, (X, z1, h1, z2, h2) = mlp_forward(theta, X)
    M = np.asarray(M, np.float64)
    denom = max(M.sum(), 1.0)
    loss = float((M * (y - T) ** 2).sum() / denom)
    dy = 2.0 * M * (y - T) / denom              # dL/dy
    gW3 = dy.T @ h2
    gb3 = dy.sum(0)
    dh2 = dy @ p["W3"]
    dz2 = dh2 * (z2 > 0)
    gW2 = dz2.T @ h1
    gb2 = dz2.sum(0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (z1 > 0)
    gW1 = dz1.T @ X
    gb1 = dz1.sum(0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, g


def adam_step(theta, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; t is the 1-based step number. Returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------
# selector regret
# ----------------------------------------------------------------------------

def regret(times: np.ndarray, feasible: np.ndarray, chosen: np.ndarray) -> np.ndarray:
    """t(chosen) / t(best feasible) - 1 per job."""
    t = np.where(feasible, times, np.inf)
    best = t.min(axis=1)
    return times[np.arange(len(times)), chosen] / best - 1.0


# ----------------------------------------------------------------------------
# string hashing of the words, one character per step (Section III-C)
# ----------------------------------------------------------------------------

FNV64_BASIS = 0xCBF29CE484222325
FNV64_PRIME = 0x100000001B3


def fnv1a64(s: bytes) -> int:
    """FNV-1a, 64 bits: for each byte, xor it in, then multiply by the prime (mod 2^64)."""
    h = FNV64_BASIS
    for b in s:
        h = ((h ^ b) * FNV64_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def word_spans(buf: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(offsets, lengths) of the words of buf in input order: maximal runs of
    bytes outside {09, 0A, 0B, 0C, 0D, 20}."""
    b = np.asarray(buf, np.uint8)
    sep = (b == 0x20) | ((b >= 0x09) & (b <= 0x0D))
    word = np.concatenate([[False], ~sep, [False]])
    d = np.diff(word.astype(np.int8))
    starts = np.flatnonzero(d == 1)
    ends = np.flatnonzero(d == -1)
    return starts.astype(np.uint64), (ends - starts).astype(np.uint64)


def word_hashes(buf: np.ndarray) -> np.ndarray:
    """FNV-1a 64 of every word of buf, in input order (uint64)."""
    raw = np.asarray(buf, np.uint8).tobytes()
    offs, lens = word_spans(buf)
    return np.array([fnv1a64(raw[o:o + l]) for o, l in zip(offs.tolist(), lens.tolist())], np.uint64)


def stream_schedule(lengths, units: int):
    """SIMDH-Stream: `units` lanes hash a stream of strings, one character per
    lane per iteration (iterations numbered from 1), the terminator taking an
    iteration of its own. A lane that meets its string's terminator takes the
    next unprocessed string at the next iteration; lanes freed together take
    the next strings in lane order. Returns [unit, first iteration, last
    iteration] per string."""
    n = len(lengths)
    out = [None] * n
    cur = [-1] * units
    pos = [0] * units
    nxt = 0
    it = 0
    while True:
        it += 1
        for u in range(units):
            if cur[u] < 0 and nxt < n:
                cur[u], pos[u] = nxt, 0
                out[nxt] = [u, it, None]
                nxt += 1
        if all(c < 0 for c in cur):
            break
        for u in range(units):
            c = cur[u]
            if c < 0:
                continue
            if pos[u] == lengths[c]:  # the terminator: this string ends here
                out[c][2] = it
                cur[u] = -1
            else:
                pos[u] += 1
    return out


def padding_schedule(lengths, units: int):
    """SIMDH-Padding: rounds of `units` consecutive strings; a round lasts as
    many iterations as its longest string has characters, plus its
    terminator; shorter strings are padded (their lanes idle). Returns
    [unit, first iteration, last iteration] per string."""
    out = []
    start = 1
    for r0 in range(0, len(lengths), units):
        grp = lengths[r0:r0 + units]
        for u, l in enumerate(grp):
            out.append([u, start, start + int(l)])
        start += int(max(grp)) + 1
    return out
