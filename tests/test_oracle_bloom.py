"""Pins of the Bloom-filter oracle (benchmark application "Bloom Filter":
k-mers of DNA bytes, h positions each, OR into one array of m bits; the
large array container of Section III-E).

The hashing is a reading (the paper does not give one): k-mer packed two bits
per base (A 0, C 1, G 2, T 3, first base most significant), x = fmix64 (the
MurmurHash3 finaliser), g_i = low32(x) + i * (high32(x) | 1) mod 2^32,
position floor(g_i * m / 2^32). These tests pin the oracle to facts that do
not come from its own code:

* a 32-mer built from a chosen hash value through the inverse of fmix64
  (the inverse uses modular inverses of MurmurHash3's published
  multipliers) sets exactly the arithmetic progression of bits that the
  chosen value dictates; this pins the base codes, their order, fmix64 and
  the position map at once; a shorter k-mer packs like the 32-mer padded
  with leading A bases;
* fmix64(0) = 0, so a run of A gives bits floor(i * m / 2^32) only;
* OR-decomposition: the filter of a sequence is the OR of the filters of two
  pieces that overlap by k - 1 bytes, and a non-ACGT byte splits it;
* the fill fraction of a filter of n random k-mers matches its exact
  expectation under uniform hashing within five standard deviations.
"""
import numpy as np
import pytest

import gen
import oracle

M64 = (1 << 64) - 1
C1, C2 = 0xFF51AFD7ED558CCD, 0xC4CEB9FE1A85EC53  # MurmurHash3 fmix64 multipliers


def inv_fmix64(x: int) -> int:
    """Inverse of fmix64: xor-shift by 33 is its own inverse on 64 bits."""
    x ^= x >> 33
    x = (x * pow(C2, -1, 1 << 64)) & M64
    x ^= x >> 33
    x = (x * pow(C1, -1, 1 << 64)) & M64
    x ^= x >> 33
    return x


def kmer_of(v: int, k: int) -> bytes:
    """The k bases whose two-bit codes, first base most significant, spell v."""
    return bytes(b"ACGT"[(v >> (2 * (k - 1 - q))) & 3] for q in range(k))


def bits_of(words: np.ndarray) -> np.ndarray:
    return np.flatnonzero(np.unpackbits(words.view(np.uint8), bitorder="little"))


def arr(b: bytes) -> np.ndarray:
    return np.frombuffer(b, np.uint8)


def test_inverse_is_an_inverse():
    rng = np.random.default_rng(3)
    for v in rng.integers(0, 1 << 63, size=64, dtype=np.int64):
        assert inv_fmix64(oracle.fmix64(int(v))) == int(v)
    assert oracle.fmix64(0) == 0


@pytest.mark.parametrize("a_hi,step,h", [(5, 3, 7), (4000, 17, 8), (0, 1, 1), (123, 4095, 5)])
def test_chosen_hash_sets_its_progression(a_hi, step, h):
    """x = (b << 32) | a with a = a_hi * 2^12 and b = step * 2^12 + 1; with
    m = 2^20 the positions are (g_i >> 12) = a_hi + i * step (mod 2^20)."""
    k, m = 32, 1 << 20
    a = a_hi << 12
    b = (step << 12) | 1
    v = inv_fmix64((b << 32) | a)
    words, n = oracle.bloom(arr(kmer_of(v, k)), m, k=k, h=h)
    assert n == 1
    expect = sorted({(a_hi + i * step) % m for i in range(h)})
    assert bits_of(words).tolist() == expect


def test_short_kmer_packs_like_a_padded_32mer():
    """A leading A is a zero digit, so a k-mer packs to the same code as the
    32-mer of 32 - k A bases followed by it; their filters must agree."""
    m, h = 1_000_003, 7
    rng = np.random.default_rng(5)
    for k in (1, 5, 12, 20, 31):
        for _ in range(8):
            s = bytes(b"ACGT"[c] for c in rng.integers(0, 4, size=k))
            a, n_a = oracle.bloom(arr(s), m, k=k, h=h)
            b, n_b = oracle.bloom(arr(b"A" * (32 - k) + s), m, k=32, h=h)
            assert n_a == n_b == 1 and np.array_equal(a, b)


def test_poly_a_sets_only_the_bits_of_zero_hash():
    m, h = 300_000_000, 7
    words, n = oracle.bloom(arr(b"A" * 100), m, k=20, h=h)
    assert n == 81
    assert bits_of(words).tolist() == sorted({(i * m) >> 32 for i in range(h)}) == [0]


def test_or_decomposition_and_splitting():
    k, m, h = 20, 1_000_003, 7
    s = gen.dna(11, 50_000, n_rate=0)
    full, n_full = oracle.bloom(s, m, k, h)
    for cut in (0, 1, 777, 25_000, 49_980):
        left, n_l = oracle.bloom(s[:cut + k - 1], m, k, h)
        right, n_r = oracle.bloom(s[cut:], m, k, h)
        assert np.array_equal(full, left | right)
        assert n_l + n_r == n_full
    t = s.copy()
    t[30_000] = ord("N")
    split, n_split = oracle.bloom(t, m, k, h)
    a, n_a = oracle.bloom(t[:30_000], m, k, h)
    b, n_b = oracle.bloom(t[30_001:], m, k, h)
    assert np.array_equal(split, a | b) and n_split == n_a + n_b == n_full - k
    # lower case and other bytes are not bases
    low = oracle.bloom(arr(b"acgt" * 10), m, 4, h)
    assert low[1] == 0 and not low[0].any()


def test_counts_and_range():
    k, h = 20, 7
    s = gen.dna(12, 10_000)
    for m in (1, 31, 33, 4096 * 32 + 5):
        w, n = oracle.bloom(s, m, k, h)
        b = bits_of(w)
        assert len(w) == (m + 31) // 32 and (len(b) == 0 or b[-1] < m)
        assert len(b) <= h * n
    assert oracle.bloom(s[:k - 1], 100, k, h)[1] == 0
    assert oracle.bloom(s[:k], 100, k, h)[1] == 1


def test_fill_fraction_matches_uniform_hashing():
    """n distinct random k-mers, h positions each: bin b receives c_b of the
    2^32 hash values (c_b = ceil((b+1) 2^32 / m) - ceil(b 2^32 / m)), so it
    stays clear with probability (1 - c_b / 2^32)^(h n). The observed count
    of set bits must be within 5 sd (balls-into-bins variance bound) of the
    expectation."""
    k, h, m = 24, 7, 10_000_019
    s = gen.dna(13, 2_000_000, n_rate=0)
    w, n = oracle.bloom(s, m, k, h)
    set_bits = int(np.unpackbits(w.view(np.uint8)).sum())
    lo = (1 << 32) // m
    n_hi = (1 << 32) - lo * m  # bins that receive lo + 1 values
    p_clear = lambda c: (1 - c / 2**32) ** (h * n)  # noqa: E731
    expect_clear = n_hi * p_clear(lo + 1) + (m - n_hi) * p_clear(lo)
    sd = np.sqrt(expect_clear)  # the empty-bin count has variance below its mean
    assert abs((m - set_bits) - expect_clear) < 5 * sd
    # a run with the i * b term dropped (all h positions equal) would fill only ~ 1 - exp(-n/m)
    assert set_bits > 1.5 * m * (1 - np.exp(-n / m))
