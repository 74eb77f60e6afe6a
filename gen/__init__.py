"""Seeded synthetic inputs for the MapReduce workloads.

This module only draws random inputs. It holds none of the method's
arithmetic (no tokenising, hashing, counting or reducing), so both the
CPU oracle and the GPU path can consume its outputs without sharing code.

Every generator is deterministic in its seed. Large arrays are drawn in
fixed chunks from independent Philox streams keyed by (seed, stream id,
chunk index), so the bytes do not depend on the number of threads used.

Input recipes (the paper names the workloads but ships none of its data):

* text: a vocabulary of V distinct lowercase words with lengths uniform in
  [lmin, lmax] (a duplicate draw is redrawn whole), tokens drawn from a
  finite Zipf law P(rank r) ~ r^-s over r = 1..V, rank mapped to a word by a
  seeded permutation; each token is followed by '\\n' with probability 1/12,
  else ' '; no partial word at the end; padded to the exact size with '\\n'.
* rgb: interleaved 8-bit RGB; each byte picks one of three Gaussians
  (means 40/128/210, sd 25) with equal weight, rounds half-to-even, clips.
* kmeans: k centres uniform in [-10, 10]^d, points = centre + N(0, 0.5^2 I),
  component uniform, stored as float32.
* u32 keys: Zipf ranks over C distinct keys mapped through a seeded
  bijection onto [0, C); optional u32 values.
* html: n_files files of synthetic HTML. URL vocabulary of V distinct URLs
  ("http://" + 5-14 lowercase letters + ".com/" + 1-40 bytes of
  [a-z0-9/_-] + ".html"); every link picks a URL by a finite Zipf(s) law
  over a seeded permutation and a file uniformly; each file's filler is a
  slice of a pool of words and tags (including near-misses such as
  <A HREF="x">, <a href='x'> and <a href=x>, never the exact link marker),
  cut at random points where its links <a href="URL">w</a> are inserted.
  File sizes are uniform in [mean/2, 3 mean/2]. The planted (file, URL id)
  pairs are returned with the bytes.
* dna: bases A, C, G, T uniform and independent; each position starts a run
  of 'N' (an unknown base, as in assembled chromosomes) with probability
  n_rate, of length uniform in [1, 200], cut at the end of its chunk.
"""
from __future__ import annotations

import concurrent.futures as _cf
import os
from dataclasses import dataclass

import numpy as np

CHUNK = 1 << 24  # bytes / elements per independent Philox chunk

_STREAM_VOCAB = 1
_STREAM_PERM = 2
_STREAM_TOKENS = 3
_STREAM_SEPS = 4
_STREAM_RGB = 5
_STREAM_KM_CENTRES = 6
_STREAM_KM_POINTS = 7
_STREAM_U32 = 8
_STREAM_JOBS = 9
_STREAM_UNIFORM = 10
_STREAM_DNA = 11
_STREAM_HTML = 12


def _rng(seed: int, stream: int, chunk: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=[seed & 0xFFFFFFFFFFFFFFFF, (stream << 40) | chunk]))


def _threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ----------------------------------------------------------------------------
# text
# ----------------------------------------------------------------------------

def vocabulary(seed: int, V: int, lmin: int = 3, lmax: int = 12) -> tuple[np.ndarray, np.ndarray]:
    """V distinct random lowercase words.

    Returns (W, L): W is uint8[V, lmax] zero padded, L is int64[V] lengths.
    A drawn word that duplicates an earlier one is discarded and redrawn
    whole, so the length mix skews slightly away from the shortest lengths
    when short words run out.
    """
    n_possible = sum(26 ** l for l in range(lmin, lmax + 1))
    if V > n_possible:
        raise ValueError("vocabulary larger than the number of possible words")
    rng = _rng(seed, _STREAM_VOCAB)
    W = np.zeros((0, lmax), np.uint8)
    L = np.zeros(0, np.int64)
    seen = np.zeros(0, dtype=f"V{lmax + 1}")
    while len(L) < V:
        need = V - len(L)
        m = int(need * 1.05) + 16
        lens = rng.integers(lmin, lmax + 1, size=m)
        letters = rng.integers(ord("a"), ord("z") + 1, size=(m, lmax), dtype=np.uint8)
        letters[np.arange(lmax)[None, :] >= lens[:, None]] = 0
        rec = np.empty((m, lmax + 1), np.uint8)
        rec[:, 0] = lens
        rec[:, 1:] = letters
        keys = np.ascontiguousarray(rec).view(f"V{lmax + 1}").ravel()
        # first occurrence within the batch, not seen before
        _, first = np.unique(keys, return_index=True)
        first.sort()
        cand = first[~np.isin(keys[first], seen)]
        cand = cand[:need]
        W = np.concatenate([W, letters[cand]])
        L = np.concatenate([L, lens[cand]])
        seen = np.concatenate([seen, keys[cand]])
    return W, L


def zipf_ranks(rng: np.random.Generator, V: int, s: float, n: int) -> np.ndarray:
    """n draws from the finite Zipf law P(r) ~ r^-s over r = 0..V-1 (0-based)."""
    w = np.arange(1, V + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = rng.random(n)
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, V - 1)


def _assemble(W: np.ndarray, L: np.ndarray, word_ids: np.ndarray, seps: np.ndarray) -> np.ndarray:
    """Bytes of word_ids[i] followed by seps[i], concatenated."""
    n = len(word_ids)
    lmax = W.shape[1]
    M = np.zeros((n, lmax + 1), np.uint8)
    M[:, :lmax] = W[word_ids]
    lens = L[word_ids]
    M[np.arange(n), lens] = seps
    keep = np.arange(lmax + 1)[None, :] <= lens[:, None]
    return M[keep]


def text(seed: int, size: int, V: int = 50_000, s: float = 1.0, lmin: int = 3, lmax: int = 12,
         newline_p: float = 1.0 / 12.0) -> np.ndarray:
    """Exactly `size` bytes of Zipf-distributed word text (uint8 array)."""
    W, L = vocabulary(seed, V, lmin, lmax)
    perm = _rng(seed, _STREAM_PERM).permutation(V)
    mean_len = float(np.mean(L)) + 1.0
    out = np.full(size, ord("\n"), np.uint8)
    pos = 0
    chunk = 0
    while True:
        want = int(min(CHUNK, (size - pos) / mean_len * 1.02 + 64))
        rng_t = _rng(seed, _STREAM_TOKENS, chunk)
        rng_s = _rng(seed, _STREAM_SEPS, chunk)
        chunk += 1
        ids = perm[zipf_ranks(rng_t, V, s, want)]
        seps = np.where(rng_s.random(want) < newline_p, ord("\n"), ord(" ")).astype(np.uint8)
        tok_len = L[ids] + 1
        cum = np.cumsum(tok_len)
        fit = int(np.searchsorted(cum, size - pos, side="right"))
        b = _assemble(W, L, ids[:fit], seps[:fit])
        out[pos:pos + len(b)] = b
        pos += len(b)
        if fit < want or pos >= size:
            break
    return out


# ----------------------------------------------------------------------------
# rgb
# ----------------------------------------------------------------------------

RGB_MEANS = (40.0, 128.0, 210.0)
RGB_SD = 25.0


def _rgb_chunk(seed: int, c: int, n: int) -> np.ndarray:
    rng = _rng(seed, _STREAM_RGB, c)
    comp = rng.integers(0, 3, size=n, dtype=np.uint8)
    v = np.asarray(RGB_MEANS)[comp] + RGB_SD * rng.standard_normal(n)
    np.rint(v, out=v)
    np.clip(v, 0, 255, out=v)
    return v.astype(np.uint8)


def rgb(seed: int, n_bytes: int | None = None) -> np.ndarray:
    """Interleaved RGB bytes. Default size: floor(2^30 / 3) pixels."""
    if n_bytes is None:
        n_bytes = (2 ** 30 // 3) * 3
    out = np.empty(n_bytes, np.uint8)
    nch = (n_bytes + CHUNK - 1) // CHUNK

    def work(c):
        lo = c * CHUNK
        hi = min(n_bytes, lo + CHUNK)
        out[lo:hi] = _rgb_chunk(seed, c, hi - lo)

    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nch)))
    return out


# ----------------------------------------------------------------------------
# k-means
# ----------------------------------------------------------------------------

def kmeans(seed: int, n: int = 1 << 24, d: int = 32, k: int = 64, sd: float = 0.5,
           box: float = 10.0) -> tuple[np.ndarray, np.ndarray]:
    """(X float32[n, d], init_centroids float32[k, d] = first k rows)."""
    centres = _rng(seed, _STREAM_KM_CENTRES).uniform(-box, box, size=(k, d))
    X = np.empty((n, d), np.float32)
    rows = max(1, CHUNK // d)
    nch = (n + rows - 1) // rows

    def work(c):
        lo = c * rows
        hi = min(n, lo + rows)
        rng = _rng(seed, _STREAM_KM_POINTS, c)
        comp = rng.integers(0, k, size=hi - lo)
        X[lo:hi] = (centres[comp] + sd * rng.standard_normal((hi - lo, d))).astype(np.float32)

    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nch)))
    return X, X[:k].copy()


# ----------------------------------------------------------------------------
# u32 keys
# ----------------------------------------------------------------------------

def u32_keys(seed: int, n: int, C: int, s: float, with_values: bool = False,
             bijection_seed: int | None = None) -> tuple[np.ndarray, np.ndarray | None]:
    """n keys in [0, C) whose frequencies follow Zipf(s) over C distinct keys.

    Returns (keys uint32[n], values uint32[n] or None).
    """
    bs = seed if bijection_seed is None else bijection_seed
    perm = _rng(bs, _STREAM_PERM, 1).permutation(C).astype(np.uint32)
    keys = np.empty(n, np.uint32)
    vals = np.empty(n, np.uint32) if with_values else None
    w = np.arange(1, C + 1, dtype=np.float64) ** (-float(s))
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    nch = (n + CHUNK - 1) // CHUNK

    def work(c):
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        rng = _rng(seed, _STREAM_U32, c)
        r = np.minimum(np.searchsorted(cdf, rng.random(hi - lo), side="right"), C - 1)
        keys[lo:hi] = perm[r]
        if vals is not None:
            vals[lo:hi] = rng.integers(0, 2 ** 32, size=hi - lo, dtype=np.uint32)

    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nch)))
    return keys, vals


def uniform_keys(seed: int, n: int, C: int) -> np.ndarray:
    """n uint32 keys drawn uniformly from [0, C) (the large-range histogram input)."""
    keys = np.empty(n, np.uint32)
    nch = (n + CHUNK - 1) // CHUNK

    def work(c):
        lo = c * CHUNK
        hi = min(n, lo + CHUNK)
        keys[lo:hi] = _rng(seed, _STREAM_UNIFORM, c).integers(0, C, size=hi - lo, dtype=np.uint32)

    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, range(nch)))
    return keys


_HTML_TAGS = [b"<p>", b"</p>", b"<div class=\"c\">", b"</div>", b"<b>", b"</b>", b"<a name=\"n\">", b"</a>",
              b"<img src=\"i.png\">", b"\n", b"<li>", b"<A HREF=\"X\">", b"<a href='y'>", b"<a href=z>",
              b"<a  href=\"w\">"]


@dataclass
class Html:
    buf: np.ndarray        # uint8 bytes of all files
    rec: np.ndarray        # uint64 file offsets [n_files + 1]
    urls: list             # URL vocabulary (bytes)
    link_file: np.ndarray  # uint32 file of each planted link
    link_url: np.ndarray   # uint32 URL id of each planted link


def html(seed: int, n_files: int = 78_355, n_links: int = 307_921, size: int = 1 << 30, V: int = 100_000,
         s: float = 1.0) -> Html:
    """Synthetic HTML files with planted links (see the module docstring)."""
    rng = _rng(seed, _STREAM_HTML)
    letters = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz", np.uint8)
    path_chars = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789/_-", np.uint8)
    urls, seen = [], set()
    while len(urls) < V:
        host = letters[rng.integers(0, 26, size=int(rng.integers(5, 15)))].tobytes()
        path = path_chars[rng.integers(0, len(path_chars), size=int(rng.integers(1, 41)))].tobytes()
        u = b"http://" + host + b".com/" + path + b".html"
        if u not in seen:
            seen.add(u)
            urls.append(u)
    perm = rng.permutation(V)
    link_url = perm[zipf_ranks(rng, V, s, n_links) - 1].astype(np.uint32)
    link_file = np.sort(rng.integers(0, n_files, size=n_links)).astype(np.uint32)
    # filler pool: words and tags
    n_tok = max(1 << 16, size // 5)
    pool_tokens = []
    vocab = [letters[rng.integers(0, 26, size=int(rng.integers(2, 11)))].tobytes() + b" " for _ in range(4096)]
    kinds = rng.random(n_tok // 16 + 1)
    tok_ids = rng.integers(0, 4096, size=n_tok // 16 + 1)
    tag_ids = rng.integers(0, len(_HTML_TAGS), size=n_tok // 16 + 1)
    for kd, w, t in zip(kinds, tok_ids, tag_ids):
        pool_tokens.append(_HTML_TAGS[t] if kd < 0.25 else vocab[w])
    pool = np.frombuffer(b"".join(pool_tokens), np.uint8)
    mean = size / n_files
    sizes = rng.integers(int(mean // 2), int(mean * 3 // 2) + 1, size=n_files)
    starts = rng.integers(0, max(1, len(pool) - int(sizes.max()) - 1), size=n_files)
    first = np.searchsorted(link_file, np.arange(n_files + 1))
    parts, rec = [], [0]
    total = 0
    for f in range(n_files):
        ln = int(sizes[f])
        body = pool[starts[f]:starts[f] + ln]
        lo, hi = first[f], first[f + 1]
        if hi > lo:
            cuts = np.sort(rng.integers(0, ln + 1, size=hi - lo))
            prev = 0
            for c, li in zip(cuts, range(lo, hi)):
                parts.append(body[prev:c])
                parts.append(np.frombuffer(b'<a href="' + urls[link_url[li]] + b'">w</a>', np.uint8))
                total += int(c) - prev
                prev = int(c)
                total += len(parts[-1])
            parts.append(body[prev:])
            total += ln - prev
        else:
            parts.append(body)
            total += ln
        rec.append(total)
    buf = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    return Html(buf, np.array(rec, np.uint64), urls, link_file, link_url)


def _dna_chunk(seed: int, c: int, n: int, n_rate: float) -> np.ndarray:
    rng = _rng(seed, _STREAM_DNA, c)
    out = np.frombuffer(b"ACGT", np.uint8)[rng.integers(0, 4, size=n, dtype=np.uint8)]
    starts = np.flatnonzero(rng.random(n) < n_rate)
    lens = rng.integers(1, 201, size=len(starts))
    for a, ln in zip(starts, lens):
        out[a:a + ln] = ord("N")
    return out


def dna(seed: int, n: int, n_rate: float = 1e-5) -> np.ndarray:
    """n DNA bytes (uint8): uniform A/C/G/T with occasional runs of N."""
    out = np.empty(n, np.uint8)
    chunks = [(c, c * CHUNK, min(n, (c + 1) * CHUNK)) for c in range((n + CHUNK - 1) // CHUNK)]

    def work(t):
        c, lo, hi = t
        out[lo:hi] = _dna_chunk(seed, c, hi - lo, n_rate)

    with _cf.ThreadPoolExecutor(_threads()) as ex:
        list(ex.map(work, chunks))
    return out


def interleave_kv(keys: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """(key, value) u32 pairs as one little-endian byte buffer."""
    kv = np.empty((len(keys), 2), np.uint32)
    kv[:, 0] = keys
    kv[:, 1] = vals
    return kv.reshape(-1).view(np.uint8)


# ----------------------------------------------------------------------------
# job specs for the batched and selector workloads
# ----------------------------------------------------------------------------

@dataclass
class JobSpec:
    kind: str          # "words" or "u32"
    size: int          # input bytes
    card: int          # vocabulary size / number of distinct possible keys
    s: float           # Zipf exponent
    lmin: int = 3
    lmax: int = 16
    op: str = "count"  # "count" or "sum" (u32 only)
    declare_range: bool = False
    seed: int = 0


def batched_specs(seed: int = 4, n_jobs: int = 256, size_lo: int = 64 << 10, size_hi: int = 16 << 20,
                  v_lo: int = 1000, v_hi: int = 1_000_000, s_lo: float = 0.6, s_hi: float = 1.4) -> list[JobSpec]:
    """Word-count jobs with log-uniform sizes and vocabularies, Zipf s uniform."""
    rng = _rng(seed, _STREAM_JOBS)
    sizes = np.exp(rng.uniform(np.log(size_lo), np.log(size_hi), n_jobs)).astype(np.int64)
    vocab = np.exp(rng.uniform(np.log(v_lo), np.log(v_hi), n_jobs)).astype(np.int64)
    ss = rng.uniform(s_lo, s_hi, n_jobs)
    return [JobSpec("words", int(sizes[i]), int(vocab[i]), float(ss[i]), 3, 16, "count", False,
                    seed * 100_003 + i) for i in range(n_jobs)]


def selector_specs(seed: int = 5, n_jobs: int = 2000, size_lo: int = 1 << 20, size_hi: int = 256 << 20,
                   c_lo: int = 16, c_hi: int = 1 << 24, s_hi: float = 1.5) -> list[JobSpec]:
    """Mixed u32/word jobs: cardinality log-uniform, Zipf s uniform in [0, s_hi]."""
    rng = _rng(seed, _STREAM_JOBS)
    sizes = np.exp(rng.uniform(np.log(size_lo), np.log(size_hi), n_jobs)).astype(np.int64)
    card = np.exp(rng.uniform(np.log(c_lo), np.log(c_hi), n_jobs)).astype(np.int64)
    ss = rng.uniform(0.0, s_hi, n_jobs)
    is_word = rng.random(n_jobs) < 0.5
    is_sum = rng.random(n_jobs) < 0.5
    declare = rng.random(n_jobs) < 0.5
    out = []
    for i in range(n_jobs):
        if is_word[i]:
            out.append(JobSpec("words", int(sizes[i]), int(card[i]), float(ss[i]), 3, 16, "count", False,
                               seed * 100_003 + i))
        else:
            sz = int(sizes[i]) // 8 * 8
            out.append(JobSpec("u32", sz, int(card[i]), float(ss[i]), 0, 0,
                               "sum" if is_sum[i] else "count", bool(declare[i]), seed * 100_003 + i))
    return out


def _job_input_worker(spec: "JobSpec") -> np.ndarray:
    return job_input(spec)


def job_pool(workers: int | None = None):
    """A warmed-up process pool for job_inputs.

    Create it before the process touches a GPU: all workers are started here
    and no process is started later, so a GPU-initialised process never forks
    or execs."""
    import concurrent.futures as cf
    import multiprocessing as mp
    import time as _time
    w = workers or _threads()
    pool = cf.ProcessPoolExecutor(w, mp_context=mp.get_context("spawn"))
    list(pool.map(_time.sleep, [0.5] * w))  # one task per worker starts every worker now
    return pool


def job_inputs(specs: list, workers: int | None = None, pool=None) -> list:
    """Inputs of many job specs: in `pool` (see job_pool) if given, else in threads."""
    if pool is not None:
        return list(pool.map(_job_input_worker, specs, chunksize=1))
    w = workers or _threads()
    if w <= 1 or len(specs) <= 1:
        return [job_input(s) for s in specs]
    with _cf.ThreadPoolExecutor(w) as ex:
        return list(ex.map(job_input, specs))


def job_input(spec: JobSpec) -> np.ndarray:
    """The input bytes of one job spec."""
    if spec.kind == "words":
        n_possible = sum(26 ** l for l in range(spec.lmin, spec.lmax + 1))
        V = int(min(spec.card, n_possible))
        return text(spec.seed, spec.size, V=V, s=spec.s, lmin=spec.lmin, lmax=spec.lmax)
    if spec.op == "sum":
        n = spec.size // 8
        k, v = u32_keys(spec.seed, n, spec.card, spec.s, with_values=True)
        return interleave_kv(k, v)
    n = spec.size // 4
    k, _ = u32_keys(spec.seed, n, spec.card, spec.s)
    return k.view(np.uint8)
