// Word count on gfx950: split, tokenise, hash, combine (LDS), reduce (global
// hash table), compact, sort and output.
//
// Paper mapping (arXiv 1309.0215):
//   * split (Fig. "basic workflow", Section II-A): the input is cut into 16 KiB
//     tiles; each workgroup takes a contiguous run of tiles. A word belongs to
//     the 16-byte chunk that holds its first byte.
//   * map + vectorisation-friendly emit (Section III-B): every lane tokenises
//     its own 16-byte chunk with a branch-free separator mask and finds word
//     starts with bit arithmetic, so no lane writes a shared container before
//     its words are found.
//   * SIMD hash (Section III-C): each lane hashes its own words (the
//     SIMDH-Padding arrangement: lanes with shorter or fewer words idle until
//     the wave's longest finishes). Words of up to 16 bytes are hashed as one
//     zero-padded 16-byte block; longer words block by block.
//   * combiner with a bounded local container (Sections III-A and III-D): a
//     per-workgroup LDS hash table holds whole keys inline; when a key finds no
//     free slot within a few probes it goes to the global table directly, and
//     at the end of the workgroup's tiles the LDS table is flushed once. When
//     every key fits, this degrades to a single flush, as the paper's
//     pipelined model does when the final table is small.
//   * global container (Section III-A hash table): open addressing with linear
//     probing. A slot is one 64-bit word {occurrence offset:32, length:16,
//     hash:16} claimed with a 64-bit CAS, plus a 32-bit count updated with
//     atomicAdd. Because the claim word carries the offset of an occurrence in
//     the (immutable) input, a thread that finds a matching tag compares the
//     full key against input bytes that are already visible: no publication
//     protocol or cache-wide fence is needed.
//   * ordered output (Section II-A): a sample sort of the distinct keys in
//     unsigned bytewise order, then key bytes, offsets and counts.
#include "common.h"
#include "jobs.h"
#include "launch.h"

namespace mr {

// ----------------------------------------------------------------------------
// byte access helpers
// ----------------------------------------------------------------------------

MR_DEV uint4 spaces4() { return make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u); }

// The 16-byte aligned block at absolute address blk, or spaces when the block
// holds no byte of [a0, a1). A block that holds one valid byte lies inside the
// caller's allocation (blocks never straddle a page), so the load is safe.
MR_DEV uint4 load_block(uint64_t a0, uint64_t a1, uint64_t blk) {
  if (blk + 16 > a0 && blk < a1) return gload16(reinterpret_cast<const void*>(blk));
  return spaces4();
}

// Bits [lo, hi) of a 32-bit mask (clamped to 0..32).
MR_DEV uint32_t range_mask32(int64_t lo, int64_t hi) {
  lo = lo < 0 ? 0 : lo;
  hi = hi > 32 ? 32 : hi;
  if (hi <= lo) return 0u;
  return (uint32_t)(((1ull << hi) - 1ull) & ~((1ull << lo) - 1ull));
}

// Bytes [s, s + len) of a 32-byte window (w[0] = bytes 0..3), zero padded to
// 16 bytes. Requires s <= 16 and len <= 16. Uses selects and byte funnel
// shifts instead of dynamic register indexing.
MR_DEV uint32_t sel32(bool c, uint32_t x, uint32_t y) { return c ? x : y; }

MR_DEV uint4 extract16(const uint32_t w[8], uint32_t s, uint32_t len) {
  // Written out by hand: a loop here is turned into a dynamically indexed
  // private array (scratch memory) before it is unrolled.
  const bool q2 = (s & 8u) != 0, q1 = (s & 4u) != 0;
  const uint32_t rb = s & 3u;
  const uint32_t w0 = w[0], w1 = w[1], w2 = w[2], w3 = w[3], w4 = w[4], w5 = w[5], w6 = w[6], w7 = w[7];
  const uint32_t v0 = sel32(q2, w2, w0), v1 = sel32(q2, w3, w1), v2 = sel32(q2, w4, w2);
  const uint32_t v3 = sel32(q2, w5, w3), v4 = sel32(q2, w6, w4), v5 = sel32(q2, w7, w5);
  const uint32_t a0 = sel32(q1, v1, v0), a1 = sel32(q1, v2, v1), a2 = sel32(q1, v3, v2);
  const uint32_t a3 = sel32(q1, v4, v3), a4 = sel32(q1, v5, v4);
  const uint32_t r0 = __builtin_amdgcn_alignbyte(a1, a0, rb);
  const uint32_t r1 = __builtin_amdgcn_alignbyte(a2, a1, rb);
  const uint32_t r2 = __builtin_amdgcn_alignbyte(a3, a2, rb);
  const uint32_t r3 = __builtin_amdgcn_alignbyte(a4, a3, rb);
  return make_uint4(keep_bytes(r0, (int)len), keep_bytes(r1, (int)len - 4), keep_bytes(r2, (int)len - 8),
                    keep_bytes(r3, (int)len - 12));
}

// The key of length len <= 16 that starts at input offset off, zero padded.
MR_DEV uint4 load_key16(const uint8_t* in, uint64_t off, uint32_t len) {
  const uint64_t a = (uint64_t)in + off;
  const uint64_t blk = a & ~15ull;
  const uint32_t s = (uint32_t)(a & 15u);
  uint32_t w[8];
  const uint4 b0 = gload16(reinterpret_cast<const void*>(blk));
  w[0] = b0.x; w[1] = b0.y; w[2] = b0.z; w[3] = b0.w;
  if (s + len > 16u) {
    const uint4 b1 = gload16(reinterpret_cast<const void*>(blk + 16));
    w[4] = b1.x; w[5] = b1.y; w[6] = b1.z; w[7] = b1.w;
  } else {
    w[4] = w[5] = w[6] = w[7] = 0u;
  }
  return extract16(w, s, len);
}

// Three-way unsigned bytewise compare of in[oa + s, oa + m) and in[ob + s, ob + m),
// 16 bytes per step.
MR_DEV int input_cmp(const uint8_t* in, uint64_t oa, uint64_t ob, uint64_t s, uint64_t m) {
  for (uint64_t b = s; b < m; b += 16) {
    const uint32_t take = (uint32_t)((m - b) < 16 ? (m - b) : 16);
    const uint4 x = load_key16(in, oa + b, take), y = load_key16(in, ob + b, take);
    if (x.x != y.x) return bswap32(x.x) < bswap32(y.x) ? -1 : 1;
    if (x.y != y.y) return bswap32(x.y) < bswap32(y.y) ? -1 : 1;
    if (x.z != y.z) return bswap32(x.z) < bswap32(y.z) ? -1 : 1;
    if (x.w != y.w) return bswap32(x.w) < bswap32(y.w) ? -1 : 1;
  }
  return 0;
}

// Placement hash of an inline key (len <= 16, zero padded): 32 bits from
// three multiplies. It places the key in the LDS cache, and key_hash16
// extends it for the global table.
MR_DEV uint32_t lds_hash32(uint4 k, uint32_t len, uint32_t debug_hash) {
  // forced collisions (debug_hash): the key bytes are left out, so every key
  // of one length gets one hash (a mask, not a branch, keeps the code straight)
  const uint32_t keep = debug_hash ? 0u : ~0u;
  const uint32_t a = ((k.x ^ __builtin_amdgcn_alignbit(k.z, k.z, 16)) & keep) * 0x9E3779B1u;
  const uint32_t b = (((k.y ^ __builtin_amdgcn_alignbit(k.w, k.w, 16)) & keep) ^ len) * 0x85EBCA77u;
  uint32_t h = a ^ __builtin_amdgcn_alignbit(b, b, 15);
  h ^= h >> 16;
  h *= 0x7FEB352Du;
  return h ^ (h >> 15);
}

// Global-table hash of an inline key from its 32-bit placement hash: the low
// word (the table index) is the placement hash itself; the high word (slot
// tag and flush queue) is a second mix of it.
MR_DEV uint64_t hash_from32(uint32_t h) {
  const uint32_t hi = (h ^ (h >> 15)) * 0x2C1B3C6Du;
  return ((uint64_t)(hi ^ (hi >> 12)) << 32) | h;
}

MR_DEV uint64_t key_hash16(uint4 k, uint32_t len, uint32_t debug_hash) {
  return hash_from32(lds_hash32(k, len, debug_hash));
}

// Hash of a key of any length stored in the input, block by block: the
// global-table hash of keys longer than 16 bytes (in the word map) and of
// every Reverse Index URL. A key always takes the same one of the two hashes
// (it depends only on the length and the map), so equal keys meet.
MR_DEV uint64_t key_hash_global(const uint8_t* in, uint64_t off, uint64_t len, uint32_t debug_hash) {
  if (debug_hash) return (uint64_t)(len < 0xFFFFu ? len : 0xFFFFu) * 0x9E3779B97F4A7C15ULL;
  uint64_t h = hash_seed((uint32_t)(len < 0xFFFFFFFFull ? len : 0xFFFFFFFFull));
  for (uint64_t b = 0; b < len; b += 16) {
    const uint32_t take = (uint32_t)((len - b) < 16 ? (len - b) : 16);
    const uint4 k = load_key16(in, off + b, take);
    h = hash_block(h, ((uint64_t)k.y << 32) | k.x, ((uint64_t)k.w << 32) | k.z);
  }
  return h;
}

// Index of the first record offset >= pos (offsets may be malformed: the
// search stays inside [0, n_rec] whatever their values).
MR_DEV uint64_t rec_lower_bound(const uint64_t* rec, uint64_t n_rec, uint64_t pos) {
  uint64_t lo = 0, hi = n_rec + 1;
  while (lo < hi) {
    const uint64_t mid = (lo + hi) >> 1;
    if (gp(rec)[mid] < pos) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Length of the word starting at input offset start (slow path for long words).
MR_DEV uint64_t word_length_slow(const WordJob& J, uint64_t vlo, uint64_t vhi, uint64_t start) {
  uint64_t end = vhi;
  if (J.rec) {
    const uint64_t r = rec_lower_bound(J.rec, J.n_rec, start + 1);
    if (r <= J.n_rec && gp(J.rec)[r] < end) end = gp(J.rec)[r];
  }
  uint64_t p = start + 1;
  while (p < end && !is_sep_byte(gp(J.in)[p])) ++p;
  return p - start;
}

// ----------------------------------------------------------------------------
// global table
// ----------------------------------------------------------------------------

MR_DEV uint64_t gword(uint64_t off, uint64_t len, uint64_t h) {
  return (off << 32) | ((len < 0xFFFFull ? len : 0xFFFFull) << 16) | (h >> 48);
}

// An occurrence offset read back from the table must lie inside the input;
// anything else means the table was not clean, which is reported, never read.
MR_DEV bool rep_in_bounds(const WordJob& J, uint64_t rep_off, uint64_t len) {
  if (rep_off + len <= J.n) return true;
  __hip_atomic_fetch_or(gp(&J.st->flags), kFlagInternal, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return false;
}

// Full-key equality of a word given inline (len <= 16) against the occurrence at rep_off.
MR_DEV bool rep_equals_inline(const WordJob& J, uint64_t rep_off, uint4 k, uint32_t len) {
  if (!rep_in_bounds(J, rep_off, len)) return false;
  const uint4 r = load_key16(J.in, rep_off, len);
  return r.x == k.x && r.y == k.y && r.z == k.z && r.w == k.w;
}

// Full-key equality of two occurrences in the input with equal length tags.
MR_DEV bool rep_equals_global(const WordJob& J, uint64_t vlo, uint64_t vhi, uint64_t rep_off, uint64_t off, uint64_t len) {
  if (rep_off == off) return true;
  if (!rep_in_bounds(J, rep_off, len)) return false;
  // the length tag saturates at 0xFFFF: then compare the true lengths too
  if (len >= 0xFFFFull && word_length_slow(J, vlo, vhi, rep_off) != len) return false;
  return input_cmp(J.in, rep_off, off, 0, len) == 0;
}

// Longest probe sequence before the table counts as full. At the planned
// load (half the slots or less) a run of this many occupied slots does not
// happen with a mixing hash; meeting one means the table is filling up, and
// probing on would make each insert scan a large part of the table.
constexpr uint64_t kMaxProbe = 512;

// Insert one key with value v. Inline keys (len <= 16) come with k; longer
// keys are compared against the input at off. Returns false on a full table;
// otherwise the key's slot goes to *slot_out when it is given. v = 0 claims
// or finds the slot without touching its count. kWorkgroup: the caller's
// workgroup is the only writer of the key's table region while it runs (the
// summing kernel of the partition queues), so workgroup-scope atomics do,
// which complete in the L2 instead of at the device's coherence point.
template <bool kInline, bool kWorkgroup = false>
MR_DEV bool g_insert(const WordJob& J, uint64_t vlo, uint64_t vhi, uint64_t off, uint64_t len, uint64_t h, uint4 k,
                     uint32_t v, uint32_t debug_hash, uint64_t* slot_out = nullptr) {
  constexpr int kScope = kWorkgroup ? __HIP_MEMORY_SCOPE_WORKGROUP : __HIP_MEMORY_SCOPE_AGENT;
  const uint64_t word = gword(off, len, h);
  // the key's region of the table (the whole table, or its partition's region)
  const uint64_t mask = J.region_log2 ? (1ull << J.region_log2) - 1 : J.cap - 1;
  const uint64_t base = J.region_log2 ? (h >> J.part_shift) << J.region_log2 : 0ull;
  // (with every key forced onto one hash the whole table is one run)
  const uint64_t limit = (debug_hash || mask < kMaxProbe) ? mask : kMaxProbe;
  uint64_t r = h & mask;
  for (uint64_t p = 0; p <= limit; ++p) {
    const uint64_t i = base + r;
    // A relaxed load may be stale only as 0 (slots are written once per run);
    // the CAS below then returns the current word.
    unsigned long long cur = __hip_atomic_load(gp(&J.tw[i]), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == 0ull) {
      unsigned long long old = 0ull;
      __hip_atomic_compare_exchange_strong(gp(&J.tw[i]), &old, (unsigned long long)word, __ATOMIC_RELAXED,
                                           __ATOMIC_RELAXED, kScope);
      if (old == 0ull) {
        if (v) __hip_atomic_fetch_add(gp(&J.tc[i]), v, __ATOMIC_RELAXED, kScope);
        if (slot_out) *slot_out = i;
        return true;
      }
      cur = old;
    }
    if ((uint32_t)cur == (uint32_t)word) {
      const uint64_t rep = cur >> 32;
      const bool eq = kInline ? rep_equals_inline(J, rep, k, (uint32_t)len) : rep_equals_global(J, vlo, vhi, rep, off, len);
      if (eq) {
        if (v) __hip_atomic_fetch_add(gp(&J.tc[i]), v, __ATOMIC_RELAXED, kScope);
        if (slot_out) *slot_out = i;
        return true;
      }
    }
    r = (r + 1) & mask;
    if ((p & 255u) == 255u &&
        (__hip_atomic_load(gp(&J.st->flags), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagTableFull))
      return false;
  }
  __hip_atomic_fetch_or(gp(&J.st->flags), kFlagTableFull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return false;
}

// ----------------------------------------------------------------------------
// prep: validate record offsets and publish the valid byte range
// ----------------------------------------------------------------------------

// Without record offsets one block per job (blockIdx.y) clears the job's
// state and publishes its whole input as the valid range: the state's only
// writer here, so no separate clearing launch is needed. With them the states
// are cleared by k_zero_states beforehand (the blocks of a job report bad
// offsets into its flags).
__global__ void k_words_prep(const WordJob* __restrict__ jobs, uint32_t n_jobs, uint32_t clear) {
  const uint32_t j = blockIdx.y;
  if (j >= n_jobs) return;
  const WordJob J = jobs[j];
  if (clear) {
    uint32_t* w = reinterpret_cast<uint32_t*>(J.st);
    for (uint32_t i = threadIdx.x; i < (uint32_t)(sizeof(JobState) / 4); i += blockDim.x) w[i] = 0u;
    __syncthreads();
  }
  if (!J.rec) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      J.st->valid_lo = 0;
      J.st->valid_hi = J.n;
    }
    return;
  }
  bool bad = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < J.n_rec; i += (uint64_t)gridDim.x * blockDim.x)
    if (J.rec[i] > J.rec[i + 1]) bad = true;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (J.rec[J.n_rec] > J.n) bad = true;
    J.st->valid_lo = J.rec[0] < J.n ? J.rec[0] : J.n;
    J.st->valid_hi = J.rec[J.n_rec] < J.n ? J.rec[J.n_rec] : J.n;
  }
  if (bad) atomicOr(&J.st->flags, kFlagBadInput);
}

// ----------------------------------------------------------------------------
// map + combine
// ----------------------------------------------------------------------------

// Probe groups: 4 consecutive slots whose tags are read with one 16-byte LDS
// load. A word visits at most kLdsGroups groups before it goes global.
constexpr int kLdsGroups = 4;
// Word descriptors a wave lists per round (a multiple of 128: two words per
// lane per step): a window's 992 owned bytes hold at most 497 word starts
// (each but the first follows a separator), so one round takes every window;
// record boundaries can add starts, which take more rounds.
constexpr uint32_t kListCap = 512;

template <int kSlotsLog2>
struct LdsTable {
  static constexpr uint32_t kSlots = 1u << kSlotsLog2;
  uint32_t tag[kSlots];   // 0 empty; bit0 ready; bits 1..5 length; bits 6..31 hash (16-byte aligned groups)
  uint4 key[kSlots];
  uint32_t cnt[kSlots];
  uint32_t off[kSlots];   // offset of one occurrence, for the global flush
};


// Zero exactly when the two 16-byte keys are equal. The final OR is one
// three-input instruction the compiler cannot see through: written as plain
// code, the OR of the XORs is turned into four compares whose results are
// packed into a bit mask with 16-bit operations.
MR_DEV uint32_t key_diff(uint4 a, uint4 b) {
  uint32_t d;
  asm("v_or3_b32 %0, %1, %2, %3" : "=v"(d) : "v"(a.x ^ b.x), "v"(a.y ^ b.y), "v"((a.z ^ b.z) | (a.w ^ b.w)));
  return d;
}

// Bucketed linear probing: a group is searched for the key; a group with an
// empty slot ends the search (slots fill in order and are never freed, so the
// key would have been placed there), and the key claims that slot.
// Returns 0 = counted in a slot that held the key, 4 = counted in a slot the
// key has just claimed, 1 = a matching slot is still being written or the
// claim was lost (retry), 2 = not in the table and not inserted (its groups
// are full: go global). The caller counts claims where it needs a fill level
// (one shared LDS counter would serialise every claim of the workgroup).
// With a job array (the summing of a batch's queues), a slot holds a key of
// one job: equality takes the job index too.
template <int L, int kGroups = kLdsGroups>
MR_DEV int lds_insert(LdsTable<L>& T, uint32_t tg, uint32_t h, uint4 k, uint32_t off, uint32_t v = 1u,
                      uint32_t* slot_job = nullptr, uint32_t job = 0u) {
  constexpr uint32_t kGroupMask = LdsTable<L>::kSlots / 4 - 1;
  uint32_t g = h & kGroupMask;
  for (int p = 0; p < kGroups; ++p) {
    // the group's four tags in one 16-byte read, classified without branches
    const uint4 t4 = reinterpret_cast<const uint4*>(T.tag)[g];
    const uint32_t tq = tg | 1u;
    const uint32_t match = ((t4.x | 1u) == tq ? 1u : 0u) | ((t4.y | 1u) == tq ? 2u : 0u) |
                           ((t4.z | 1u) == tq ? 4u : 0u) | ((t4.w | 1u) == tq ? 8u : 0u);
    const uint32_t ready = (t4.x & 1u) | ((t4.y & 1u) << 1) | ((t4.z & 1u) << 2) | ((t4.w & 1u) << 3);
    const uint32_t empty = (t4.x == 0u ? 1u : 0u) | (t4.y == 0u ? 2u : 0u) | (t4.z == 0u ? 4u : 0u) |
                           (t4.w == 0u ? 8u : 0u);
    // ready slots with the key's tag: compare the whole key with one 16-byte read each
    for (uint32_t rm = match & ready; rm; rm &= rm - 1u) {
      const uint32_t i = 4 * g + (uint32_t)__builtin_ctz(rm);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // key bytes after the ready tag
      if (key_diff(T.key[i], k) == 0u && (!slot_job || slot_job[i] == job)) {
        atomicAdd(&T.cnt[i], v);
        return 0;
      }
    }
    if (match & ~ready) return 1;  // a slot with the key's tag is still being written
    if (empty) {
      const uint32_t i = 4 * g + (uint32_t)__builtin_ctz(empty);  // slots fill in order: the first empty one
      if (atomicCAS(&T.tag[i], 0u, tg) != 0u) return 1;  // lost the slot: look again
      T.key[i] = k;
      T.off[i] = off;
      T.cnt[i] = v;
      if (slot_job) slot_job[i] = job;
      __hip_atomic_store(&T.tag[i], tg | 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
      return 4;
    }
    g = (g + 1) & kGroupMask;
  }
  return 2;
}

template <int L>
MR_DEV void lds_flush(LdsTable<L>& T, const WordJob& J, uint64_t vlo, uint64_t vhi, uint32_t debug_hash) {
  for (uint32_t i = threadIdx.x; i < LdsTable<L>::kSlots; i += blockDim.x) {
    const uint32_t tg = T.tag[i];
    if (tg & 1u) {
      const uint32_t len = (tg >> 1) & 31u;
      const uint4 k = T.key[i];
      const uint64_t h = key_hash16(k, len, debug_hash);
      g_insert<true>(J, vlo, vhi, T.off[i], len, h, k, T.cnt[i], debug_hash);
    }
    T.tag[i] = 0u;
  }
}

// One record of a partition queue: key bytes as loaded, offset of an
// occurrence, length, count, and the index of the job in its batch (the
// queues of a batch are shared by its jobs).
struct FlushRec {
  uint4 k;
  uint32_t off, len, cnt, job;
};

// Appends a record to this workgroup's sub-queue of partition q: 16 bytes
// (key bytes 0..7, offset, length | count << 4 | job << 16) for a key of up
// to 8 bytes with a count below 4096 and a job index below 65536, 32 bytes
// otherwise; the positions come from the workgroup's LDS fill counters.
// Returns false when that sub-queue is full (the caller inserts globally).
MR_DEV bool queue_append(const WordJob& J, uint32_t* mfill, uint32_t* sfill, uint32_t q, uint4 k, uint32_t off, uint32_t len,
                         uint32_t cnt, uint32_t job) {
  const uint64_t sub = (uint64_t)q * J.mq_grid + blockIdx.x;
  if (len <= 8u && cnt < 4096u && job < 65536u) {
    const uint32_t at = atomicAdd(&sfill[q], 1u);
    if (at >= J.sq_cap) return false;
    gstore16(reinterpret_cast<uint4*>(J.sq) + sub * J.sq_cap + at, make_uint4(k.x, k.y, off, len | (cnt << 4) | (job << 16)));
    return true;
  }
  const uint32_t at = atomicAdd(&mfill[q], 1u);
  if (at >= J.mq_cap) return false;
  FlushRec* dst = reinterpret_cast<FlushRec*>(J.mq) + sub * J.mq_cap + at;
  gstore16(&dst->k, k);
  gstore16(&dst->off, make_uint4(off, len, cnt, job));
  return true;
}

// Two-phase reduce, first phase, for the cache: every entry of the
// workgroup's LDS cache goes to the workgroup's own sub-queue of its key's
// partition, after the words the cache missed; an entry that finds its
// sub-queue full is inserted globally at once. J is job `job` of the batch.
// The cache is cleared. Called by the whole workgroup.
template <int L>
MR_DEV void lds_flush_parts(LdsTable<L>& T, const WordJob& J, uint32_t job, uint32_t* mfill, uint32_t* sfill, uint64_t vlo,
                            uint64_t vhi, uint32_t debug_hash) {
  for (uint32_t i = threadIdx.x; i < LdsTable<L>::kSlots; i += blockDim.x) {
    const uint32_t tg = T.tag[i];
    if (tg & 1u) {
      const uint32_t len = (tg >> 1) & 31u;
      const uint4 k = T.key[i];
      const uint64_t h = key_hash16(k, len, debug_hash);
      if (!queue_append(J, mfill, sfill, (uint32_t)(h >> J.part_shift), k, T.off[i], len, T.cnt[i], job))
        g_insert<true>(J, vlo, vhi, T.off[i], len, h, k, T.cnt[i], debug_hash);
    }
    T.tag[i] = 0u;
  }
}

MR_DEV uint32_t find_job(const uint64_t* __restrict__ tile_base, uint32_t n_jobs, uint64_t t) {
  uint32_t lo = 0, hi = n_jobs;  // last j with tile_base[j] <= t
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (tile_base[mid] <= t) lo = mid; else hi = mid;
  }
  return lo;
}

// Separator mask of a 16-byte block.
MR_DEV uint32_t sep16(uint4 b) { return sep_mask16(b.x, b.y, b.z, b.w); }

// Four 32-bit words read at any byte address.
typedef uint32_t u32x4_u __attribute__((ext_vector_type(4), aligned(1)));

// Wave-level combiner: `rounds` times, the first lane still holding a word
// is the leader; every lane whose word equals the leader's (same LDS hash,
// length and bytes) adds its count to the leader and drops out. `v` is this
// lane's count (0 after it merged into a leader). Uniform control flow.
MR_DEV void wave_combine_words(bool has, uint32_t h, uint32_t len, uint4 k, uint32_t& v, int rounds) {
  uint64_t left = __ballot(has);
  for (int r = 0; r < rounds && left; ++r) {
    const int ld = __ffsll((long long)left) - 1;
    auto rl = [ld](uint32_t x) { return (uint32_t)__builtin_amdgcn_readlane((int)x, ld); };
    const uint32_t lh = rl(h), ll = rl(len), k0 = rl(k.x), k1 = rl(k.y), k2 = rl(k.z), k3 = rl(k.w);
    const bool same = has && v && h == lh && len == ll && k.x == k0 && k.y == k1 && k.z == k2 && k.w == k3;
    const uint64_t eq = __ballot(same);
    if ((int)lane_id() == ld) v = popc64(eq);
    else if (same) v = 0u;
    left &= ~eq;
  }
}

// Lanes per window and owned chunks: wave w's window of a tile is 64
// consecutive 16-byte chunks, one per lane. Lane 0 holds the chunk before the
// owned run (its last byte decides whether the first owned byte starts a
// word) and lane 63 the chunk after it (words of up to 16 bytes that start in
// lane 62's chunk end there); lanes 1..62 own their chunks. Windows of
// neighbouring parts overlap by two chunks.
constexpr uint32_t kOwnChunks = kWave - 2;
static_assert(kMapTileChunks == (kMapThreads / kWave) * kOwnChunks, "tile = one owned run per wave");

// One workgroup per run of tiles; wave w takes the w-th run of 62 owned
// chunks of every tile of the run. The waves share the LDS hash cache but no
// barrier between tiles: each moves on to its next part as soon as it is
// done, so the latency one wave waits on (a global probe, a slow word) is
// hidden by the others instead of holding the whole workgroup at a barrier.
// For each part:
//   1. every lane loads one 16-byte chunk of the window (loaded two tiles
//      ahead) and stores it in the wave's LDS copy; it computes its chunk's
//      separator mask, and takes the next lane's mask and the previous
//      lane's last bit with DPP lane shifts;
//   2. each owning lane appends one descriptor per word start (offset in the
//      window, length; 31 marks a word longer than 16 bytes) to the wave's
//      list, placed by a wave prefix sum;
//   3. the wave takes the list one word per lane (all lanes busy): key bytes
//      from the LDS copy, LDS hash, optionally the wave combiner, LDS cache
//      insert; words the cache cannot take are packed and inserted globally,
//      one per lane.
// Workgroup barriers remain where the run moves to another job (the cache is
// flushed into the old job's table) and at the end.
template <int L, bool kRecords, bool kCombine>
__global__ __launch_bounds__(kMapThreads) void k_words_map(const WordJob* __restrict__ jobs, const uint64_t* __restrict__ tile_base,
                                                           uint32_t n_jobs, uint64_t total_tiles, uint32_t debug_hash) {
  constexpr uint32_t kWaves = kMapThreads / kWave;
  __shared__ LdsTable<L> T;
  __shared__ uint4 stage[kWaves][kWave];
  __shared__ __attribute__((aligned(16))) uint16_t wlist[kWaves][kListCap];
  // byte masks of the inline key lengths (entry n keeps bytes [0, n); the
  // entries past 16 are all zero)
  __shared__ __attribute__((aligned(16))) uint32_t s_kmask[64][4];
  constexpr uint32_t kBndWords = kWave * 16 / 32;  // boundary bits of the 1 KiB window
  __shared__ uint32_t bnd[kRecords ? kWaves : 1][kRecords ? kBndWords + 1 : 1];
  __shared__ uint32_t s_mfill[kMaxWordParts], s_sfill[kMaxWordParts];  // this workgroup's sub-queue fills

  for (uint32_t i = threadIdx.x; i < LdsTable<L>::kSlots; i += blockDim.x) T.tag[i] = 0u;
  for (uint32_t i = threadIdx.x; i < kMaxWordParts; i += blockDim.x) {
    s_mfill[i] = 0u;
    s_sfill[i] = 0u;
  }
  if (threadIdx.x < 256) {
    const uint32_t n = threadIdx.x >> 2, w = threadIdx.x & 3u;
    const int keep = n <= 16u ? (int)n - 4 * (int)w : 0;
    s_kmask[n][w] = keep >= 4 ? ~0u : (keep <= 0 ? 0u : (1u << (8 * keep)) - 1u);
  }
  __syncthreads();

  const uint64_t t_begin = total_tiles * blockIdx.x / gridDim.x;
  const uint64_t t_end = total_tiles * (blockIdx.x + 1) / gridDim.x;
  const uint32_t wave = threadIdx.x / kWave;
  const uint32_t lane = lane_id();
  uint4* const ws = stage[wave];
  int cur = -1;
  uint64_t vlo = 0, vhi = 0;
  auto wave_sync = [] {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
  };

  // This lane's chunk of the wave's window of tile t: chunk c0 - 1 + lane of
  // the job, c0 = the first owned chunk (spaces outside the job's input).
  auto load_part = [&](uint64_t t) -> uint4 {
    const uint32_t jn = find_job(tile_base, n_jobs, t);
    const WordJob& Jn = jobs[jn];
    const uint64_t an0 = (uint64_t)Jn.in, an1 = an0 + Jn.n;
    const int64_t ci = (int64_t)((t - tile_base[jn]) * kMapTileChunks + wave * kOwnChunks) - 1 + (int64_t)lane;
    return (ci >= 0 && (uint64_t)ci < Jn.n_chunks) ? load_block(an0, an1, (Jn.chunk0 + (uint64_t)ci) * 16) : spaces4();
  };
  // The job's flags, read for the abort test. Every lane reads them at an
  // address offset by a zero the compiler cannot see through, so the value
  // stays in a vector register until the test reads its first lane: a value
  // the compiler knows to be uniform is moved to a scalar register as soon as
  // it is loaded, which waits for every load issued before it.
  uint32_t zv;
  asm("v_mov_b32 %0, 0" : "=v"(zv));
  auto flags_of = [&](uint64_t t) -> uint32_t {
    return __hip_atomic_load(gp(&jobs[find_job(tile_base, n_jobs, t)].st->flags + zv), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  };
  // Tiles are prefetched two ahead into two register sets used in turn (the
  // tile body below is emitted once for each), so that moving on to the next
  // tile takes no register copy: copying a register whose load is still in
  // flight waits for that load. For the same reason the flags for the next
  // tile are read before its prefetch is issued and tested one tile later.
  uint4 pa = spaces4(), pb = spaces4();
  if (t_begin < t_end) pa = load_part(t_begin);
  if (t_begin + 1 < t_end) pb = load_part(t_begin + 1);
  uint32_t fl_next = t_begin < t_end ? flags_of(t_begin) : 0u;

  auto tile = [&](uint64_t t, uint4& buf) {
    const uint32_t j = find_job(tile_base, n_jobs, t);
    if ((int)j != cur) {
      // every wave meets this point at the same tile
      __syncthreads();
      if (cur >= 0) {
        if (jobs[cur].mq)
          lds_flush_parts<L>(T, jobs[cur], (uint32_t)cur, s_mfill, s_sfill, vlo, vhi, debug_hash);
        else lds_flush<L>(T, jobs[cur], vlo, vhi, debug_hash);
        __syncthreads();
      }
      cur = (int)j;
      vlo = gp(jobs[j].st)->valid_lo;
      vhi = gp(jobs[j].st)->valid_hi;
    }
    const WordJob& J = jobs[j];
    const uint32_t fl = fl_next;
    const uint64_t lt = t - tile_base[j];
    const uint64_t a0 = (uint64_t)J.in;
    // absolute address of the window's first byte (lane 0's chunk)
    const uint64_t win = (J.chunk0 + lt * kMapTileChunks + wave * kOwnChunks - 1) * 16;
    // input offset of the window's first byte, modulo 2^32 (inputs are below 4 GiB)
    const uint32_t win_off = (uint32_t)(win - a0);

    // the previous part's list and copy are no longer read by any lane of the wave
    wave_sync();
    uint32_t bd = 0u, bd_next = 0u;
    if constexpr (kRecords) {
      for (uint32_t i = lane; i <= kBndWords; i += kWave) bnd[wave][i] = 0u;
      wave_sync();
      // record boundaries falling in the window; in a batch that mixes jobs
      // with and without records, the latter keep an empty bitmap
      if (J.rec) {
        const int64_t lo_rel = (int64_t)(win - a0);
        const uint64_t r0 = rec_lower_bound(J.rec, J.n_rec, lo_rel < 0 ? 0 : (uint64_t)lo_rel);
        for (uint64_t r = r0 + lane; r <= J.n_rec; r += kWave) {
          const uint64_t pa = a0 + gp(J.rec)[r];
          if (pa < win) continue;
          const uint64_t bit = pa - win;
          if (bit >= 32ull * kBndWords) break;
          atomicOr(&bnd[wave][bit >> 5], 1u << (bit & 31));
        }
      }
      wave_sync();
      const uint32_t wv = bnd[wave][lane >> 1];
      bd = (lane & 1u) ? (wv >> 16) : (wv & 0xFFFFu);
      bd_next = from_next_lane(bd, 0u);
    }

    // 1. the window into LDS; separator masks
    ws[lane] = buf;
    uint32_t sep = sep16(buf);
    // buf is free: the tile two ahead goes into it, after the flags for the next tile
    if (t + 1 < t_end) fl_next = flags_of(t + 1);
    if (t + 2 < t_end) buf = load_part(t + 2);
    if (__builtin_amdgcn_readfirstlane(fl) & (kFlagTableFull | kFlagBadInput)) return;  // uniform over the wave
    // bytes outside the valid range count as separators (only windows that
    // reach past it need the per-lane check)
    if (win < a0 + vlo || win + 16ull * kWave > a0 + vhi) {
      const uint64_t B = win + 16ull * lane;
      sep |= ~range_mask32((int64_t)(a0 + vlo) - (int64_t)B, (int64_t)(a0 + vhi) - (int64_t)B) & 0xFFFFu;
    }
    const uint32_t sep_next = from_next_lane(sep, 0xFFFFu);
    const uint32_t prev = from_prev_lane(sep >> 15, 1u);
    const uint32_t starts = (lane - 1u < kOwnChunks) ? (~sep & ((sep << 1) | prev | bd) & 0xFFFFu) : 0u;
    const uint32_t ends = sep | (sep_next << 16) | bd | (bd_next << 16);

    // 2. one descriptor per word start, placed by a wave prefix sum
    const uint32_t n_mine = __builtin_popcount(starts);
    const uint32_t incl = wave_incl_scan(n_mine);
    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, kWave - 1);
    const uint32_t first = incl - n_mine;
    wave_sync();  // the window copy is complete

    // 3. rounds of up to kListCap words, two words per lane per step.
    // Descriptor: offset in the window << 6 | length, where 17..32 mark a word
    // longer than 16 bytes (no end within the 16 bytes after its start; bit 31
    // of the shifted end mask stands in for "no end", giving 32).
    uint16_t* const wl = wlist[wave];
    const uint32_t ends1 = (ends >> 1) | 0x80000000u;
    const uint32_t lane16 = lane * 16u;
    for (uint32_t base = 0; base < total; base += kListCap) {
      {
        uint32_t p = first - base;  // entries outside [0, kListCap) belong to other rounds
        auto put = [&](uint32_t m) {
          const uint32_t s = __builtin_ctz(m);
          const uint32_t len = (uint32_t)__builtin_ctz(ends1 >> s) + 1u;
          wl[p] = (uint16_t)(((lane16 + s) << 6) | len);
        };
        if (total <= kListCap) {  // uniform: the whole list fits this round
          for (uint32_t m = starts; m; m &= m - 1u, ++p) put(m);
        } else {
          for (uint32_t m = starts; m; m &= m - 1u, ++p)
            if (p < kListCap) put(m);
        }
      }
      wave_sync();
      const uint32_t nr = (total - base) < kListCap ? (total - base) : kListCap;
      // a word the cache did not take goes to the job's miss queue (or the
      // global table); a word longer than 16 bytes is measured, hashed and
      // inserted from the input
      auto miss = [&](bool lng, uint32_t off, uint32_t len, uint32_t h, uint4 k, uint32_t v) {
        if (lng) {
          const uint64_t wlen = word_length_slow(J, vlo, vhi, off);
          g_insert<false>(J, vlo, vhi, off, wlen, key_hash_global(J.in, off, wlen, debug_hash), make_uint4(0, 0, 0, 0),
                          1u, debug_hash);
          return;
        }
        const uint64_t h64 = hash_from32(h);
        // into this workgroup's sub-queue of the key's partition
        if (J.mq && queue_append(J, s_mfill, s_sfill, (uint32_t)(h64 >> J.part_shift), k, off, len, v, j)) return;
        g_insert<true>(J, vlo, vhi, off, len, h64, k, v, debug_hash);
      };
      // the home-group lookup could not decide: the full insert, retried
      // while a slot is being written
      auto slow = [&](uint32_t tg, uint32_t h, uint4 k, uint32_t off, uint32_t v) -> int {
        int r = 1;
        for (uint32_t spin = 0; r == 1; ++spin) {
          r = lds_insert<L, 1>(T, tg, h, k, off, v);
          if (r == 1 && spin > (1u << 22)) {
            __hip_atomic_fetch_or(gp(&J.st->flags), kFlagSpin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            r = 0;
          }
        }
        return r;
      };
      constexpr uint32_t kGroupMask = LdsTable<L>::kSlots / 4 - 1;
#pragma unroll 1
      for (uint32_t i0 = 0; i0 < nr; i0 += 2 * kWave) {
        // Straight-line code over the step's two words, so that the LDS reads
        // of one overlap the arithmetic of the other. Key bytes come from the
        // wave's copy of the window (16 bytes at any byte offset: LDS reads
        // need no alignment here, and o <= 62 * 16 + 15 keeps the read inside
        // the wave's 1 KiB), masked to the word's length.
        uint4 k[2];
        uint32_t h[2], len[2], o[2], v[2], slot[2];
        bool has[2], inl[2];
        int r[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t i = i0 + lane + u * kWave;  // < kListCap: i0 <= kListCap - 128
          has[u] = i < nr;
          const uint32_t d0 = wl[i];
          const uint32_t d = has[u] ? d0 : 0u;
          o[u] = d >> 6;
          len[u] = d & 63u;
          const u32x4_u x = *reinterpret_cast<const u32x4_u*>(reinterpret_cast<const uint8_t*>(ws) + o[u]);
          const uint4 mk = *reinterpret_cast<const uint4*>(s_kmask[len[u]]);
          k[u] = make_uint4(x[0] & mk.x, x[1] & mk.y, x[2] & mk.z, x[3] & mk.w);
          inl[u] = has[u] && len[u] <= 16u;
          h[u] = lds_hash32(k[u], len[u], debug_hash);
          v[u] = 1u;
        }
        if constexpr (kCombine) {
          wave_combine_words(inl[0], h[0], len[0], k[0], v[0], 4);
          wave_combine_words(inl[1], h[1], len[1], k[1], v[1], 4);
        }
        // home group: one 16-byte tag read each, then the key of the slot
        // whose ready tag matches (read whether or not one does); the steps
        // go over both words in turn, so that their LDS reads overlap
        uint4 t4[2];
        uint32_t c[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          t4[u] = reinterpret_cast<const uint4*>(T.tag)[h[u] & kGroupMask];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          // first slot with the ready tag (4: none); plain selects and bitwise
          // logic, so that the compiler emits no branches here
          const uint32_t tq = (h[u] & 0xFFFFFFC0u) | (len[u] << 1) | 1u;
          const uint32_t c3 = t4[u].w == tq ? 3u : 4u;
          const uint32_t c2 = t4[u].z == tq ? 2u : c3;
          const uint32_t c1 = t4[u].y == tq ? 1u : c2;
          c[u] = t4[u].x == tq ? 0u : c1;
          slot[u] = 4u * (h[u] & kGroupMask) + (c[u] & 3u);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");  // key bytes after the ready tags
        uint4 kk[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) kk[u] = T.key[slot[u]];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const uint32_t tg = (h[u] & 0xFFFFFFC0u) | (len[u] << 1);
          const uint32_t kd = key_diff(kk[u], k[u]);
          const bool go = inl[u] & (v[u] != 0u);
          const bool hit = go & (c[u] < 4u) & (kd == 0u);
          if (hit) atomicAdd(&T.cnt[slot[u]], v[u]);
          // no ready slot with the key: undecided while the group has a free
          // slot (tag 0), a slot with this tag still being written, or a
          // ready slot whose tag matched another key
          const uint4 t = t4[u];
          const uint32_t free_min = min(min(t.x, t.y), min(t.z, t.w));
          const uint32_t pend_min = min(min(t.x ^ tg, t.y ^ tg), min(t.z ^ tg, t.w ^ tg));
          const bool undecided = (c[u] < 4u) | (free_min == 0u) | (pend_min == 0u);
          r[u] = (go & !hit) ? (undecided ? 3 : 2) : 0;
        }
        if (__ballot(r[0] == 3 || r[1] == 3)) {
#pragma unroll
          for (int u = 0; u < 2; ++u)
            if (r[u] == 3) r[u] = slow((h[u] & 0xFFFFFFC0u) | (len[u] << 1), h[u], k[u], win_off + o[u], v[u]);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const bool lng = has[u] && len[u] > 16u;
          if (r[u] == 2 || lng) miss(lng, win_off + o[u], len[u], h[u], k[u], v[u]);
        }
      }
      wave_sync();
    }
  };
  for (uint64_t t = t_begin; t < t_end; t += 2) {
    tile(t, pa);
    if (t + 1 < t_end) tile(t + 1, pb);
  }
  __syncthreads();
  if (cur >= 0) {
    if (jobs[cur].mq) lds_flush_parts<L>(T, jobs[cur], (uint32_t)cur, s_mfill, s_sfill, vlo, vhi, debug_hash);
    else lds_flush<L>(T, jobs[cur], vlo, vhi, debug_hash);
  }
  // the sub-queue fills, once every flushed entry has taken its place (the
  // sub-queues are shared by the jobs of a batch; every workgroup writes all
  // of its entries, zero or not, so nothing needs clearing before)
  __syncthreads();
  const WordJob& J0 = jobs[0];
  if (J0.mq)
    for (uint32_t q = threadIdx.x; q < (1u << (64 - J0.part_shift)); q += blockDim.x) {
      const uint32_t f = s_mfill[q], g = s_sfill[q];
      J0.mq_fill[q * J0.mq_grid + blockIdx.x] = f < J0.mq_cap ? f : J0.mq_cap;
      J0.sq_fill[q * J0.mq_grid + blockIdx.x] = g < J0.sq_cap ? g : J0.sq_cap;
    }
}

// Two-phase flush, second phase: one workgroup per partition sums the
// records of its flush queue and of every map workgroup's miss sub-queue by
// (job, key) in an LDS table and inserts each summed key into its job's table,
// so that the keys every workgroup meets no longer meet on one global slot
// from every workgroup. The records are taken in rounds of one per thread
// (the next round's record is loaded meanwhile); after a round that leaves
// the table more than half full, the table is flushed into the global tables
// (one insert per summed key, all threads at once) and cleared, so records
// never fall back to one global insert each. A round adds at most blockDim
// keys, which keeps the table below three quarters full.
constexpr uint32_t kMaxMapGrid = 1024;  // map workgroups (miss sub-queues per partition)
template <int L>
__global__ __launch_bounds__(kMapThreads) void k_words_parts(const WordJob* __restrict__ jobs, uint32_t debug_hash) {
  constexpr uint32_t kSlots = LdsTable<L>::kSlots;
  static_assert(kSlots / 2 + kMapThreads <= kSlots / 4 * 3, "a round cannot fill the table");
  __shared__ LdsTable<L> T;
  __shared__ uint32_t s_job[kSlots];
  // first record of each segment: map workgroup w's 32-byte sub-queue (w),
  // then its 16-byte one (G + w)
  __shared__ uint32_t s_pre[2 * kMaxMapGrid + 1];
  __shared__ uint32_t s_used;
  const WordJob& Q = jobs[0];  // the queues (shared by the jobs of a batch)
  const uint32_t p = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kSlots; i += blockDim.x) T.tag[i] = 0u;
  if (threadIdx.x == 0) s_used = 0;
  // exclusive prefix of the segment sizes, blockDim at a time
  __shared__ uint32_t s_wsum[kMapThreads / kWave];
  const uint32_t G = Q.mq_grid, NS = 2 * G;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t carry = 0;
  for (uint32_t b0 = 0; b0 < NS; b0 += blockDim.x) {
    const uint32_t w = b0 + threadIdx.x;
    const uint32_t c = w < G ? *gp(&Q.mq_fill[p * G + w]) : (w < NS ? *gp(&Q.sq_fill[p * G + (w - G)]) : 0u);
    const uint32_t incl = wave_incl_scan(c);
    if (lane == kWave - 1) s_wsum[wv] = incl;
    __syncthreads();
    uint32_t before = carry, all = 0;
    for (uint32_t q = 0; q < nw; ++q) {
      if (q < wv) before += s_wsum[q];
      all += s_wsum[q];
    }
    if (w < NS) s_pre[w] = before + incl - c;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) s_pre[NS] = carry;
  __syncthreads();
  const uint32_t total = carry;
  // record r of the partition: the last segment starting at or before it.
  // A thread's records only move forward, so the search gallops on from its
  // previous segment (steps 1, 2, 4, ...) and then bisects.
  // record r of the partition: the last segment starting at or before it.
  // A thread's records only move forward, so the search gallops on from its
  // previous segment (steps 1, 2, 4, ...) and then bisects. The record's two
  // 16-byte halves are loaded (the second is zero for a 16-byte record; the
  // caller decodes by `wide`).
  uint32_t seg = 0;
  auto load_rec = [&](uint32_t r, uint4& a, uint4& b, bool& wide) {
    uint32_t lo = seg, hi = seg + 1, step = 1;  // s_pre[lo] <= r < total = s_pre[NS]
    while (hi < NS && s_pre[hi] <= r) {
      lo = hi;
      step <<= 1;
      hi = lo + step;
    }
    if (hi > NS) hi = NS;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_pre[mid] <= r) lo = mid; else hi = mid;
    }
    seg = lo;
    const uint32_t e = r - s_pre[seg];
    wide = seg < G;
    if (wide) {
      const FlushRec* rp = reinterpret_cast<const FlushRec*>(Q.mq) + ((uint64_t)p * G + seg) * Q.mq_cap + e;
      a = gload16(&rp->k);
      b = gload16(&rp->off);
    } else {
      a = gload16(reinterpret_cast<const uint4*>(Q.sq) + ((uint64_t)p * G + (seg - G)) * Q.sq_cap + e);
      b = make_uint4(0, 0, 0, 0);
    }
  };
  // a summed key into its job's table: with the table split into partition
  // regions, this workgroup is the region's only writer
  auto insert = [&](const WordJob& J, uint32_t off, uint32_t len, uint64_t h, uint4 k, uint32_t v) {
    if (J.region_log2) g_insert<true, true>(J, 0, 0, off, len, h, k, v, debug_hash);
    else g_insert<true>(J, 0, 0, off, len, h, k, v, debug_hash);
  };
  auto consume = [&](uint4 k, uint4 m) -> bool {  // m: off, len, count, job; true: claimed a slot
    const uint32_t hk = lds_hash32(k, m.y, debug_hash);
    // the LDS placement mixes in the job; the global table takes the key's own hash
    const uint32_t h32 = hk ^ (m.w * 0x9E3779B1u);
    const uint32_t tg = (h32 & 0xFFFFFFC0u) | (m.y << 1);
    int r = 1;
    for (uint32_t spin = 0; r == 1; ++spin) {
      r = lds_insert<L>(T, tg, h32, k, m.x, m.z, s_job, m.w);
      if (r == 1 && spin > (1u << 22)) {
        __hip_atomic_fetch_or(gp(&jobs[m.w].st->flags), kFlagSpin, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        r = 0;
      }
    }
    // the key's probe groups are full (rare below three quarters load)
    if (r == 2) insert(jobs[m.w], m.x, m.y, hash_from32(hk), k, m.z);
    return r == 4;
  };
  // the summed keys into their jobs' tables; the table is cleared
  auto flush = [&]() {
    for (uint32_t i = threadIdx.x; i < kSlots; i += blockDim.x) {
      const uint32_t tg = T.tag[i];
      if (tg & 1u) {
        const uint32_t len = (tg >> 1) & 31u;
        const uint4 k = T.key[i];
        insert(jobs[s_job[i]], T.off[i], len, key_hash16(k, len, debug_hash), k, T.cnt[i]);
      }
      T.tag[i] = 0u;
    }
  };
  uint4 na = make_uint4(0, 0, 0, 0), nb = make_uint4(0, 0, 0, 0);
  bool nwide = true;
  if (threadIdx.x < total) load_rec(threadIdx.x, na, nb, nwide);
  for (uint32_t base = 0; base < total; base += blockDim.x) {
    const bool have = base + threadIdx.x < total;
    // this round's record as (key, {offset, length, count, job})
    const uint4 k = nwide ? na : make_uint4(na.x, na.y, 0u, 0u);
    const uint4 m = nwide ? nb : make_uint4(na.z, na.w & 15u, (na.w >> 4) & 0xFFFu, na.w >> 16);
    const uint32_t nx = base + blockDim.x + threadIdx.x;
    if (nx < total) load_rec(nx, na, nb, nwide);
    const bool claimed = have && consume(k, m);
    // the round's claims, one LDS add per wave
    const uint32_t nc = popc64(__ballot(claimed));
    if (lane == 0 && nc) atomicAdd(&s_used, nc);
    __syncthreads();
    const bool full = s_used > kSlots / 2;  // uniform: read after the barrier
    __syncthreads();
    if (full) {
      flush();
      if (threadIdx.x == 0) s_used = 0;
      __syncthreads();
    }
  }
  __syncthreads();
  flush();
}

// ----------------------------------------------------------------------------
// compaction: table slots -> records (and the table is cleared for reuse)
// ----------------------------------------------------------------------------

constexpr uint32_t kCompactThreads = 256;
// slots per work item (one job-counter update each): 1024 for small tables,
// where more workgroups help, 4096 for large ones, where fewer updates do
constexpr uint32_t kCompactSmall = 1024, kCompactLarge = 4096;

// The entry of slot i, or 0 (empty, or an occurrence offset outside the
// input, which is reported and skipped).
MR_DEV unsigned long long compact_entry(const WordJob& J, uint64_t i) {
  if (i >= J.cap) return 0ull;
  const unsigned long long w = J.tw[i];
  if (w && !rep_in_bounds(J, w >> 32, (w >> 16) & 0xFFFFull)) return 0ull;
  return w;
}

// Work item = `item` slots of one job's table, 1024 or 4096 (tables are
// powers of two >= 4096 slots at 4096-aligned arena offsets, so no item
// straddles two tables). Pass 1 counts the entries, one atomic reserves their
// places, pass 2 writes the records and clears the slots.
__global__ __launch_bounds__(kCompactThreads) void k_words_compact(const WordJob* __restrict__ jobs, uint32_t n_jobs,
                                                                   uint64_t total_slots, uint32_t item) {
  __shared__ uint32_t s_cnt, s_pos;
  __shared__ unsigned long long s_base, s_bytes;
  for (uint64_t t0 = (uint64_t)blockIdx.x * item; t0 < total_slots; t0 += (uint64_t)gridDim.x * item) {
    uint32_t lo = 0, hi = n_jobs;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (jobs[mid].slot_base <= t0) lo = mid; else hi = mid;
    }
    const WordJob& J = jobs[lo];
    const uint64_t i0 = t0 - J.slot_base;
    if (threadIdx.x == 0) {
      s_cnt = 0;
      s_pos = 0;
      s_bytes = 0;
    }
    __syncthreads();
    uint32_t mine = 0;
    for (uint32_t q = threadIdx.x; q < item; q += kCompactThreads) mine += compact_entry(J, i0 + q) ? 1u : 0u;
    if (mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0) s_base = s_cnt ? atomicAdd(&J.st->n_recs, (unsigned long long)s_cnt) : 0ull;
    __syncthreads();
    unsigned long long bytes = 0;
    for (uint32_t q = threadIdx.x; q < item; q += kCompactThreads) {
      const uint64_t i = i0 + q;
      const unsigned long long w = compact_entry(J, i);
      if (!w) continue;
      const uint32_t cnt = J.tc[i];
      J.tw[i] = 0ull;
      J.tc[i] = 0u;
      const uint64_t off = w >> 32;
      uint64_t len = (w >> 16) & 0xFFFFull;
      if (len == 0xFFFFull) len = word_length_slow(J, J.st->valid_lo, J.st->valid_hi, off);
      const uint4 k = load_key16(J.in, off, (uint32_t)(len < 16 ? len : 16));
      WRec r;
      r.p[0] = bswap32(k.x); r.p[1] = bswap32(k.y); r.p[2] = bswap32(k.z); r.p[3] = bswap32(k.w);
      r.len = (uint32_t)len;
      r.off = (uint32_t)off;
      r.cnt = cnt;
      r.pad = (uint32_t)i;  // the table slot, for callers that map slots to output ranks
      reinterpret_cast<WRec*>(J.recs)[s_base + atomicAdd(&s_pos, 1u)] = r;
      bytes += len;
    }
    if (bytes) atomicAdd(&s_bytes, bytes);
    __syncthreads();
    if (threadIdx.x == 0 && s_bytes) atomicAdd(&J.st->key_bytes, s_bytes);
  }
}

// ----------------------------------------------------------------------------
// sample sort of the distinct keys (unsigned bytewise order, prefix first)
// ----------------------------------------------------------------------------

// A record read with two 16-byte global loads (records are 32-byte aligned).
// A plain copy through a generic pointer becomes flat word loads, which may
// alias LDS and therefore wait for each other around the LDS stores that
// follow them.
MR_DEV WRec load_wrec(const WRec* p) {
  const uint4 a = gload16(p), b = gload16(reinterpret_cast<const uint8_t*>(p) + 16);
  WRec r;
  r.p[0] = a.x;
  r.p[1] = a.y;
  r.p[2] = a.z;
  r.p[3] = a.w;
  r.len = b.x;
  r.off = b.y;
  r.cnt = b.z;
  r.pad = b.w;
  return r;
}

MR_DEV void store_wrec(WRec* p, const WRec& r) {
  gstore16(p, make_uint4(r.p[0], r.p[1], r.p[2], r.p[3]));
  gstore16(reinterpret_cast<uint8_t*>(p) + 16, make_uint4(r.len, r.off, r.cnt, r.pad));
}

// Three-way compare of two records of the same job.
MR_DEV int wrec_cmp(const WordJob& J, const WRec& a, const WRec& b) {
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (a.p[q] != b.p[q]) return a.p[q] < b.p[q] ? -1 : 1;
  if (a.len > 16u && b.len > 16u) {
    const int c = input_cmp(J.in, a.off, b.off, 16, a.len < b.len ? a.len : b.len);
    if (c) return c;
  }
  return a.len < b.len ? -1 : (a.len > b.len ? 1 : 0);
}

// Bitonic sort (all-ascending "flip" form) of a[0, m) by the whole workgroup.
// Indices >= m act as +infinity and are never touched, so no padding is
// needed; works on LDS or global memory (callers synchronise the workgroup).
MR_DEV void bitonic_sort(const WordJob& J, WRec* a, uint32_t m) {
  uint32_t n = 1;
  while (n < m) n <<= 1;
  for (uint32_t k = 2; k <= n; k <<= 1) {
    for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
      for (uint32_t t = threadIdx.x; t < n / 2; t += blockDim.x) {
        // t-th pair: i has bit jj clear
        const uint32_t i = ((t & ~(jj - 1)) << 1) | (t & (jj - 1));
        const uint32_t l = (jj == (k >> 1)) ? (i ^ (k - 1)) : (i | jj);
        if (l < m) {
          const WRec x = a[i], y = a[l];
          if (wrec_cmp(J, x, y) > 0) {
            a[i] = y;
            a[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Keys of up to CAP records in LDS: 16-byte prefixes, lengths and record
// indices in separate arrays (a search step reads one prefix and one length).
template <uint32_t CAP>
struct LdsKeys {
  uint4 k[CAP];
  uint32_t len[CAP];
  uint32_t ix[CAP];  // record index
};

// a < b for keys given by their 16-byte prefixes (x the most significant
// word) and lengths, read as 160-bit numbers: the borrow out of a - b, one
// subtract-with-borrow per word, all in the vector unit. Keys longer than
// 16 bytes with one prefix are ordered by the caller.
MR_DEV bool lex_less(uint4 a, uint32_t al, uint4 b, uint32_t bl) {
  uint32_t d, r;
  uint64_t c;
  asm("v_sub_co_u32_e64 %0, %2, %3, %4\n\t"
      "v_subb_co_u32_e64 %0, %2, %5, %6, %2\n\t"
      "v_subb_co_u32_e64 %0, %2, %7, %8, %2\n\t"
      "v_subb_co_u32_e64 %0, %2, %9, %10, %2\n\t"
      "v_subb_co_u32_e64 %0, %2, %11, %12, %2\n\t"
      "v_cndmask_b32_e64 %1, 0, 1, %2"
      : "=&v"(d), "=v"(r), "=&s"(c)
      : "v"(al), "v"(bl), "v"(a.w), "v"(b.w), "v"(a.z), "v"(b.z), "v"(a.y), "v"(b.y), "v"(a.x), "v"(b.x));
  return r != 0;
}

// Sort of entries [0, m) of K (m <= E * blockDim.x, m <= CAP) by merging.
// At the level of runs of L entries, the entry at place i counts the entries
// of its partner run below it by a binary search of that run; with its own
// index in its run that gives its place in the merged run of 2L (the keys
// are distinct). Each thread keeps E entries in registers and follows them
// from place to place: every search reads K, a barrier, then every entry is
// written to its new place. There are ceil(log2 m) levels and no padding.
template <uint32_t E, uint32_t CAP>
MR_DEV void merge_sort(const uint8_t* in, const WRec* recs, LdsKeys<CAP>& K, uint32_t m) {
  const uint32_t T = blockDim.x, t = threadIdx.x;
  uint4 xk[E];
  uint32_t xl[E], xi[E], at[E];  // an entry's key, record and present place
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    at[e] = e * T + t;
    if (at[e] < m) {
      xk[e] = K.k[at[e]];
      xl[e] = K.len[at[e]];
      xi[e] = K.ix[at[e]];
    }
  }
  for (uint32_t L = 1; L < m; L <<= 1) {
    uint32_t dst[E];
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const uint32_t i = at[e];
      dst[e] = i;
      if (i < m) {
        const uint32_t b0 = (i ^ L) & ~(L - 1);  // the partner run
        const uint32_t blen = b0 >= m ? 0u : (m - b0 < L ? m - b0 : L);
        uint32_t pos = 0;  // entries of the partner run below entry i
        for (uint32_t step = L; step; step >>= 1) {
          const uint32_t q = pos + step;
          if (q <= blen) {
            const uint32_t j = b0 + q - 1;
            const uint4 bk = K.k[j];
            const uint32_t bl = K.len[j];
            bool below = lex_less(bk, bl, xk[e], xl[e]);
            const uint32_t ml = bl < xl[e] ? bl : xl[e];
            if (ml > 16u) {
              // two keys longer than 16 bytes: when they share the prefix
              // their bytes in the input decide (the empty asm keeps these
              // compares inside the branch)
              uint4 pk = bk;
              asm volatile("" : "+v"(pk.x), "+v"(pk.y), "+v"(pk.z), "+v"(pk.w));
              if (pk.x == xk[e].x && pk.y == xk[e].y && pk.z == xk[e].z && pk.w == xk[e].w) {
                const int c = input_cmp(in, recs[K.ix[j]].off, recs[xi[e]].off, 16, ml);
                below = c < 0 || (c == 0 && bl < xl[e]);
              }
            }
            if (below) pos = q;
          }
        }
        dst[e] = (i & ~(2 * L - 1)) + (i & (L - 1)) + pos;
      }
    }
    __syncthreads();  // every search has read the previous order
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      if (at[e] < m) {
        K.k[dst[e]] = xk[e];
        K.len[dst[e]] = xl[e];
        K.ix[dst[e]] = xi[e];
        at[e] = dst[e];
      }
    }
    __syncthreads();
  }
}

constexpr uint32_t kSortThreads = 1024;
constexpr uint32_t kBucketKeys = 512;       // keys per sort bucket, on average
constexpr uint32_t kBucketThreads = 1024;   // threads of a bucket's workgroup
constexpr uint32_t kOversample = 4;
constexpr uint32_t kMaxSamples = kMaxBuckets * kOversample;
constexpr uint32_t kRankRows = kSortThreads / kWave;  // samples ranked per work item of k_sort_ranks (one per wave)
constexpr uint32_t kRankJobs = 4;                     // batches of up to this many jobs take k_sort_ranks

// Samples per bucket of a job with nb > 1 buckets: 4 * kOversample while the
// sample fits half of kMaxSamples, 2 * kOversample while it fits all of it,
// else kOversample. The largest bucket sets the bucket sort's time, and more
// samples keep it closer to the mean (a bucket larger than the workgroup
// takes two entries per thread and about twice the time).
MR_DEV uint32_t sample_ov(uint32_t nb) {
  return nb * 4 * kOversample <= kMaxSamples / 2 ? 4 * kOversample
                                                 : (nb * 2 * kOversample <= kMaxSamples ? 2 * kOversample : kOversample);
}

// Sort plan of one job of n distinct keys: buckets, record tiles and rank
// work items (the last only for jobs of more than one bucket).
MR_DEV void job_plan(uint64_t n, uint32_t& nb, uint32_t& rt, uint32_t& si) {
  nb = 1;
  si = 0;
  if (n > kBucketCap) {
    const uint64_t want = (n + kBucketKeys - 1) / kBucketKeys;
    nb = (uint32_t)(want < kMaxBuckets ? want : kMaxBuckets);
    si = (nb * sample_ov(nb) + kRankRows - 1) / kRankRows;
  }
  rt = (uint32_t)((n + kRecTile - 1) / kRecTile);
}

// Plan the sort of every job: bucket counts and global bucket / record-tile
// bases. One workgroup; the jobs are taken blockDim at a time, one per
// thread, and the bases come from a workgroup scan of the counts.
__global__ __launch_bounds__(kSortThreads) void k_sort_plan(const WordJob* __restrict__ jobs, uint32_t n_jobs,
                                                             uint32_t* totals /*[2]*/) {
  __shared__ uint32_t w_nb[kSortThreads / kWave], w_rt[kSortThreads / kWave];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t carry_b = 0, carry_r = 0;
  for (uint32_t base = 0; base < n_jobs; base += blockDim.x) {
    const uint32_t j = base + threadIdx.x;
    uint32_t nb = 0, rt = 0, si;
    if (j < n_jobs) job_plan(jobs[j].st->n_recs, nb, rt, si);
    const uint32_t inb = wave_incl_scan(nb), irt = wave_incl_scan(rt);
    if (lane == kWave - 1) {
      w_nb[wv] = inb;
      w_rt[wv] = irt;
    }
    __syncthreads();
    uint32_t pb = carry_b, pr = carry_r, tb = 0, tr = 0;
    for (uint32_t q = 0; q < nw; ++q) {
      if (q < wv) {
        pb += w_nb[q];
        pr += w_rt[q];
      }
      tb += w_nb[q];
      tr += w_rt[q];
    }
    if (j < n_jobs) {
      JobState* st = jobs[j].st;
      st->nb = nb;
      st->bucket_base = pb + inb - nb;
      st->rtile_base = pr + irt - rt;
    }
    carry_b += tb;
    carry_r += tr;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    totals[0] = carry_b;
    totals[1] = carry_r;
  }
}

// Splitters of one job: its sample is S = nb * ov evenly spaced records,
// sorted in LDS by the merge sort, and the splitter of bucket b is the
// sample entry of rank (b + 1) * ov - 1. One workgroup per job (the jobs of
// a batch run side by side); it also clears the job's bucket counters.
__global__ __launch_bounds__(kSortThreads) void k_sort_splitters(const WordJob* __restrict__ jobs, uint32_t n_jobs,
                                                                  uint32_t* bucket_cnt, unsigned long long* bucket_bytes,
                                                                  uint32_t* bucket_fill) {
  static_assert(kMaxSamples <= 4 * kSortThreads, "a sample takes at most four entries per thread");
  __shared__ LdsKeys<kMaxSamples> smp;
  const uint32_t j = blockIdx.x;
  if (j >= n_jobs) return;
  const WordJob& J = jobs[j];
  const uint32_t nb = J.st->nb;
  const uint32_t bb = J.st->bucket_base;
  for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
    bucket_cnt[bb + b] = 0;
    bucket_bytes[bb + b] = 0;
    bucket_fill[bb + b] = 0;
  }
  if (nb <= 1) return;
  const uint64_t n = J.st->n_recs;
  const uint32_t ov = sample_ov(nb), S = nb * ov;
  const WRec* recs = reinterpret_cast<const WRec*>(J.recs);
  for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
    const uint32_t ix = (uint32_t)((uint64_t)i * n / S);
    const WRec r = load_wrec(&recs[ix]);
    smp.k[i] = make_uint4(r.p[0], r.p[1], r.p[2], r.p[3]);
    smp.len[i] = r.len;
    smp.ix[i] = ix;
  }
  __syncthreads();
  if (S <= blockDim.x) merge_sort<1>(J.in, recs, smp, S);
  else if (S <= 2 * blockDim.x) merge_sort<2>(J.in, recs, smp, S);
  else merge_sort<4>(J.in, recs, smp, S);
  WRec* spl = reinterpret_cast<WRec*>(J.splitters);
  for (uint32_t b = threadIdx.x; b + 1 < nb; b += blockDim.x) store_wrec(&spl[b], load_wrec(&recs[smp.ix[(b + 1) * ov - 1]]));
}

// Order of two keys by their 16-byte prefixes and lengths (plain compares,
// no branches); `tie` marks two keys longer than 16 bytes with one prefix,
// whose order needs their bytes in the input.
MR_DEV void key_order(uint4 a, uint32_t al, uint4 b, uint32_t bl, bool& lt, bool& tie) {
  const bool e0 = a.x == b.x, e1 = a.y == b.y, e2 = a.z == b.z, e3 = a.w == b.w;
  lt = (a.x < b.x) | (e0 & ((a.y < b.y) | (e1 & ((a.z < b.z) | (e2 & ((a.w < b.w) | (e3 & (al < bl))))))));
  tie = e0 & e1 & e2 & e3 & (al > 16u) & (bl > 16u);
}


// The same splitters without a sort, for a batch of a few jobs: a single
// sort of the sample would leave all but one CU idle. The keys are
// distinct, so a sample's rank is the number of samples below it, found by
// comparing it with every sample: work item g ranks kRankRows samples of one
// job, one per wave, each lane taking every 64th sample and a ballot adding
// up the lanes; the items of all jobs are spread over the grid. The kernel
// also plans the sort of its (at most kRankJobs) jobs, as k_sort_plan would:
// every workgroup works the plan out for itself, workgroup 0 stores it for
// the kernels that follow, and the grid clears every bucket's counters.
__global__ __launch_bounds__(kSortThreads) void k_sort_ranks(const WordJob* __restrict__ jobs, uint32_t n_jobs,
                                                              uint32_t* totals, uint32_t* bucket_cnt,
                                                              unsigned long long* bucket_bytes, uint32_t* bucket_fill) {
  __shared__ uint4 ck[kMaxSamples];
  __shared__ uint32_t cl[kMaxSamples];
  __shared__ uint32_t s_nb[kRankJobs], s_rank_base[kRankJobs + 1], s_tot[3];
  if (threadIdx.x == 0) {
    uint32_t tb = 0, tr = 0, ts = 0;
    for (uint32_t j = 0; j < n_jobs; ++j) {
      uint32_t nb, rt, si;
      job_plan(jobs[j].st->n_recs, nb, rt, si);
      s_nb[j] = nb;
      s_rank_base[j] = ts;
      if (blockIdx.x == 0) {
        JobState* st = jobs[j].st;
        st->nb = nb;
        st->bucket_base = tb;
        st->rtile_base = tr;
      }
      tb += nb;
      tr += rt;
      ts += si;
    }
    s_rank_base[n_jobs] = ts;
    s_tot[0] = tb;
    s_tot[1] = tr;
    s_tot[2] = ts;
    if (blockIdx.x == 0) {
      totals[0] = tb;
      totals[1] = tr;
    }
  }
  __syncthreads();
  const uint32_t n_buckets = s_tot[0];
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < n_buckets; b += gridDim.x * blockDim.x) {
    bucket_cnt[b] = 0;
    bucket_bytes[b] = 0;
    bucket_fill[b] = 0;
  }
  const uint32_t items = s_tot[2];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  for (uint32_t g = blockIdx.x; g < items; g += gridDim.x) {
    uint32_t j = 0;  // the job whose items hold g
    while (j + 1 < n_jobs && s_rank_base[j + 1] <= g) ++j;
    const WordJob& J = jobs[j];
    const uint32_t nb = s_nb[j];
    const uint64_t n = J.st->n_recs;
    const uint32_t ov = sample_ov(nb), S = nb * ov;
    const WRec* recs = reinterpret_cast<const WRec*>(J.recs);
    __syncthreads();  // the previous item's reads of the sample are done
    for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
      const WRec r = load_wrec(&recs[(uint64_t)i * n / S]);
      ck[i] = make_uint4(r.p[0], r.p[1], r.p[2], r.p[3]);
      cl[i] = r.len;
    }
    __syncthreads();
    const uint32_t row = (g - s_rank_base[j]) * kRankRows + wv;
    if (row < S) {
      const uint4 rk = ck[row];
      const uint32_t rl = cl[row];
      const uint64_t rix = (uint64_t)row * n / S;
      uint32_t rank = 0;
      for (uint32_t c0 = 0; c0 < S; c0 += kWave) {
        const uint32_t c = c0 + lane;
        bool below = false;
        if (c < S) {
          const uint32_t l = cl[c];
          bool tie;
          key_order(ck[c], l, rk, rl, below, tie);
          if (tie) {  // rare: two long keys with one prefix
            const int cc = input_cmp(J.in, recs[(uint64_t)c * n / S].off, recs[rix].off, 16, l < rl ? l : rl);
            below = cc < 0 || (cc == 0 && l < rl);
          }
        }
        rank += (uint32_t)__popcll(__ballot(below));
      }
      if (lane == 0 && (rank + 1) % ov == 0) {
        const uint32_t b = (rank + 1) / ov - 1;
        if (b + 1 < nb) store_wrec(&reinterpret_cast<WRec*>(J.splitters)[b], load_wrec(&recs[rix]));
      }
    }
  }
}

// Bucket of each record: number of splitters strictly below it.
MR_DEV uint32_t bucket_of(const WordJob& J, const WRec* spl, uint32_t nb, const WRec& r) {
  uint32_t lo = 0, hi = nb - 1;  // count of splitters < r, in [0, nb - 1]
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (wrec_cmp(J, spl[mid], r) < 0) lo = mid + 1; else hi = mid;
  }
  return lo;
}

MR_DEV uint32_t find_rtile_job(const WordJob* jobs, uint32_t n_jobs, uint32_t t) {
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].st->rtile_base <= t) lo = mid; else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_sort_count(const WordJob* __restrict__ jobs, uint32_t n_jobs, const uint32_t* totals,
                                                    uint32_t* bucket_cnt, unsigned long long* bucket_bytes) {
  __shared__ WRec spl[kMaxBuckets - 1];
  __shared__ uint32_t h_cnt[kMaxBuckets];
  __shared__ unsigned long long h_bytes[kMaxBuckets];
  const uint32_t n_tiles = totals[1];
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint32_t j = find_rtile_job(jobs, n_jobs, t);
    const WordJob& J = jobs[j];
    const uint32_t nb = J.st->nb;
    const uint64_t n = J.st->n_recs;
    const uint64_t r0 = (uint64_t)(t - J.st->rtile_base) * kRecTile;
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
      h_cnt[b] = 0;
      h_bytes[b] = 0;
      if (b + 1 < nb) spl[b] = load_wrec(reinterpret_cast<const WRec*>(J.splitters) + b);
    }
    __syncthreads();
    const WRec* recs = reinterpret_cast<const WRec*>(J.recs);
    for (uint32_t q = threadIdx.x; q < kRecTile; q += blockDim.x) {
      const uint64_t i = r0 + q;
      if (i >= n) break;
      const WRec r = load_wrec(&recs[i]);
      const uint32_t b = nb > 1 ? bucket_of(J, spl, nb, r) : 0u;
      *gp(&J.rec_bucket[i]) = b;
      atomicAdd(&h_cnt[b], 1u);
      atomicAdd(&h_bytes[b], (unsigned long long)r.len);
    }
    __syncthreads();
    const uint32_t bb = J.st->bucket_base;
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) {
      if (h_cnt[b]) {
        atomicAdd(&bucket_cnt[bb + b], h_cnt[b]);
        atomicAdd(&bucket_bytes[bb + b], h_bytes[b]);
      }
    }
  }
}

// Exclusive scans of one job's bucket counts and bytes (one workgroup per
// job, chunks of blockDim buckets); capacity check.
__global__ __launch_bounds__(kSortThreads) void k_sort_scan(const WordJob* __restrict__ jobs, uint32_t n_jobs,
                                                             const uint32_t* bucket_cnt, const unsigned long long* bucket_bytes,
                                                             uint32_t* bucket_start, unsigned long long* bucket_bstart) {
  __shared__ uint32_t wc[kSortThreads / kWave];
  __shared__ unsigned long long wb[kSortThreads / kWave];
  const uint32_t j = blockIdx.x;
  if (j >= n_jobs) return;
  const WordJob& J = jobs[j];
  const uint32_t nb = J.st->nb, bb = J.st->bucket_base;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t carry_c = 0;
  unsigned long long carry_b = 0;
  for (uint32_t base = 0; base < nb; base += blockDim.x) {
    const uint32_t b = base + threadIdx.x;
    const uint32_t c = b < nb ? bucket_cnt[bb + b] : 0u;
    const unsigned long long y = b < nb ? bucket_bytes[bb + b] : 0ull;
    uint32_t ic = c;
    unsigned long long iy = y;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t tc = __shfl_up(ic, o);
      const unsigned long long ty = __shfl_up(iy, o);
      if (lane >= (uint32_t)o) {
        ic += tc;
        iy += ty;
      }
    }
    if (lane == kWave - 1) {
      wc[wv] = ic;
      wb[wv] = iy;
    }
    __syncthreads();
    uint32_t pc = carry_c, tot_c = 0;
    unsigned long long py = carry_b, tot_b = 0;
    for (uint32_t q = 0; q < nw; ++q) {
      if (q < wv) {
        pc += wc[q];
        py += wb[q];
      }
      tot_c += wc[q];
      tot_b += wb[q];
    }
    if (b < nb) {
      bucket_start[bb + b] = pc + ic - c;
      bucket_bstart[bb + b] = py + iy - y;
    }
    carry_c += tot_c;
    carry_b += tot_b;
    __syncthreads();
  }
  // the outputs' capacity; when they hold the job, the final entry of its
  // key offsets (the total of its key bytes)
  if (threadIdx.x == 0) {
    if (J.st->n_recs > J.cap_keys || J.st->key_bytes > J.cap_key_bytes) atomicOr(&J.st->flags, kFlagCapacity);
    else if (J.out_key_offsets) J.out_key_offsets[J.st->n_recs] = J.st->key_bytes;
  }
}

__global__ __launch_bounds__(256) void k_sort_scatter(const WordJob* __restrict__ jobs, uint32_t n_jobs, const uint32_t* totals,
                                                      const uint32_t* bucket_start, uint32_t* bucket_fill) {
  // One global reservation per (tile, bucket) instead of one atomic per record.
  __shared__ uint32_t h_cnt[kMaxBuckets];
  __shared__ uint32_t h_base[kMaxBuckets];
  const uint32_t n_tiles = totals[1];
  for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    const uint32_t j = find_rtile_job(jobs, n_jobs, t);
    const WordJob& J = jobs[j];
    const uint64_t n = J.st->n_recs;
    const uint32_t nb = J.st->nb;
    const uint64_t r0 = (uint64_t)(t - J.st->rtile_base) * kRecTile;
    const uint32_t bb = J.st->bucket_base;
    const WRec* recs = reinterpret_cast<const WRec*>(J.recs);
    WRec* out = reinterpret_cast<WRec*>(J.recs2);
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x) h_cnt[b] = 0;
    __syncthreads();
    constexpr uint32_t kPer = kRecTile / 256;
    uint32_t bk[kPer], loc[kPer];
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint64_t i = r0 + q * 256 + threadIdx.x;
      bk[q] = i < n ? *gp(&J.rec_bucket[i]) : 0xFFFFFFFFu;
      loc[q] = bk[q] != 0xFFFFFFFFu ? atomicAdd(&h_cnt[bk[q]], 1u) : 0u;
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
      h_base[b] = h_cnt[b] ? bucket_start[bb + b] + atomicAdd(&bucket_fill[bb + b], h_cnt[b]) : 0u;
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < kPer; ++q) {
      const uint64_t i = r0 + q * 256 + threadIdx.x;
      if (bk[q] != 0xFFFFFFFFu) store_wrec(&out[h_base[bk[q]] + loc[q]], load_wrec(&recs[i]));
    }
  }
}

MR_DEV uint32_t find_bucket_job(const WordJob* jobs, uint32_t n_jobs, uint32_t g) {
  uint32_t lo = 0, hi = n_jobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].st->bucket_base <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// Output key bytes of a bucket staged in LDS before they are written out in
// aligned 16-byte pieces (a bucket sorted in LDS whose keys are all inline).
constexpr uint32_t kStageBytes = 32512;  // with the sort arrays, under half the CU's LDS: two workgroups per CU

// Sort each bucket and write the job's outputs for it.
__global__ __launch_bounds__(kBucketThreads) void k_sort_buckets(const WordJob* __restrict__ jobs, uint32_t n_jobs, const uint32_t* totals,
                                                                const uint32_t* bucket_cnt, const unsigned long long* bucket_bytes,
                                                                const uint32_t* bucket_start,
                                                                const unsigned long long* bucket_bstart) {
  static_assert(kBucketCap <= 4 * kBucketThreads, "a bucket sorted in LDS takes at most four entries per thread");
  __shared__ LdsKeys<kBucketCap> a;
  __shared__ uint64_t wsum[kBucketThreads / kWave];
  __shared__ __attribute__((aligned(16))) uint8_t ob[kStageBytes];
  __shared__ uint32_t s_long;
  const uint32_t n_buckets = totals[0];
  for (uint32_t g = blockIdx.x; g < n_buckets; g += gridDim.x) {
    const uint32_t j = find_bucket_job(jobs, n_jobs, g);
    const WordJob& J = jobs[j];
    const uint32_t m = bucket_cnt[g];
    const uint32_t s0 = bucket_start[g];
    const uint64_t y0 = bucket_bstart[g];
    const bool write = !(__hip_atomic_load(&J.st->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagCapacity);
    WRec* src = reinterpret_cast<WRec*>(J.recs2) + s0;
    __syncthreads();
    if (m == 0) continue;
    const bool in_lds = m <= kBucketCap;
    if (threadIdx.x == 0) s_long = 0u;
    __syncthreads();
    if (in_lds) {
      for (uint32_t i = threadIdx.x; i < m; i += blockDim.x) {
        const WRec r = load_wrec(&src[i]);
        a.k[i] = make_uint4(r.p[0], r.p[1], r.p[2], r.p[3]);
        a.len[i] = r.len;
        a.ix[i] = i;
        if (r.len > 16u) s_long = 1u;
      }
      __syncthreads();
      if (m <= blockDim.x) {
        merge_sort<1>(J.in, src, a, m);
      } else if constexpr (kBucketCap <= 2 * kBucketThreads) {
        merge_sort<2>(J.in, src, a, m);
      } else {
        if (m <= 2 * blockDim.x) merge_sort<2>(J.in, src, a, m);
        else merge_sort<4>(J.in, src, a, m);
      }
    } else {
      if (threadIdx.x == 0) atomicAdd(&J.st->sort_spills, 1u);  // rare: sort the bucket in global memory
      bitonic_sort(J, src, m);
    }
    if (!write) continue;
    // The bucket's key bytes are [y0, y0 + nbytes) of the output. Staged:
    // byte y0 + e sits at ob[sh + e], where sh puts ob[0] at a 16-byte
    // aligned output address.
    const uint64_t nbytes = bucket_bytes[g];
    uint8_t* const dst0 = J.out_key_bytes + y0;
    const uint32_t sh = (uint32_t)((uintptr_t)dst0 & 15u);
    const bool stage = in_lds && !s_long && nbytes + sh <= kStageBytes;
    // byte positions: exclusive scan of lengths in chunks of blockDim
    uint64_t carry = 0;
    for (uint32_t base = 0; base < m; base += blockDim.x) {
      const uint32_t i = base + threadIdx.x;
      const uint64_t len = i < m ? (in_lds ? a.len[i] : src[i].len) : 0;
      // wave inclusive scan
      uint64_t x = len;
      const uint32_t ln = lane_id();
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint64_t y = __shfl_up(x, o);
        if (ln >= (uint32_t)o) x += y;
      }
      if (ln == kWave - 1) wsum[threadIdx.x / kWave] = x;
      __syncthreads();
      uint64_t wpre = 0;
      const uint32_t wv = threadIdx.x / kWave;
      for (uint32_t q = 0; q < wv; ++q) wpre += wsum[q];
      uint64_t tot = 0;
      for (uint32_t q = 0; q < blockDim.x / kWave; ++q) tot += wsum[q];
      const uint64_t excl = carry + wpre + x - len;
      if (i < m) {
        const WRec r = load_wrec(&src[in_lds ? a.ix[i] : i]);
        const uint64_t o = y0 + excl;
        J.out_key_offsets[s0 + i] = o;
        J.out_values[s0 + i] = r.cnt;
        if (J.slot_rank) J.slot_rank[r.pad] = (uint32_t)(s0 + i);
        if (stage) {
          // the key is the big-endian prefix itself
          uint8_t* const d = ob + sh + (uint32_t)excl;
#pragma unroll
          for (uint32_t b = 0; b < 16u; ++b)
            if (b < r.len) d[b] = (uint8_t)(r.p[b >> 2] >> (24 - 8 * (b & 3)));
        } else if (r.len <= 16u) {
#pragma unroll
          for (uint32_t b = 0; b < 16u; ++b)
            if (b < r.len) J.out_key_bytes[o + b] = (uint8_t)(r.p[b >> 2] >> (24 - 8 * (b & 3)));
        } else {
          for (uint32_t b0 = 0; b0 < r.len; b0 += 16) {  // 16 bytes loaded per step
            const uint32_t take = r.len - b0 < 16u ? r.len - b0 : 16u;
            const uint4 k = load_key16(J.in, r.off + b0, take);
            const uint32_t w[4] = {k.x, k.y, k.z, k.w};
#pragma unroll
            for (uint32_t b = 0; b < 16u; ++b)
              if (b < take) J.out_key_bytes[o + b0 + b] = (uint8_t)(w[b >> 2] >> (8 * (b & 3)));
          }
        }
      }
      carry += tot;
      __syncthreads();
    }
    if (stage) {
      // 16-byte pieces wholly inside the bucket's range as one store each;
      // the partial pieces at the two ends byte by byte (neighbouring
      // buckets own the rest of them)
      uint8_t* const base = dst0 - sh;  // 16-byte aligned
      const uint32_t end = sh + (uint32_t)nbytes;
      for (uint32_t c = threadIdx.x; c * 16u < end; c += blockDim.x) {
        const uint32_t lo = c * 16u, hi = lo + 16u;
        if (lo >= sh && hi <= end) {
          gstore16(base + lo, *reinterpret_cast<const uint4*>(ob + lo));
        } else {
          for (uint32_t b = lo < sh ? sh : lo; b < (hi < end ? hi : end); ++b) base[b] = ob[b];
        }
      }
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------------------------
// host side
// ----------------------------------------------------------------------------

int words_max_lds_log2() { return 12; }

// ----------------------------------------------------------------------------
// links: the map of the Reverse Index (Table of benchmark applications). A
// link is the nine bytes <a href=" followed by a URL of 1..4095 bytes other
// than a double quote and then a double quote, all inside one record (file).
// Every start position is tried, so links may overlap. Each URL goes into
// the job's global table (the same table, compaction and sort as words) and
// (table slot, record) into a pair list, from which the link counts and the
// file lists are built: counting in the table would serialise the many links
// of a popular URL on one atomic.
// ----------------------------------------------------------------------------

constexpr uint32_t kLinkMaxUrl = 4095;
constexpr uint32_t kLinkFindThreads = 256;
constexpr uint32_t kLinkGroup = 64;   // input bytes per lane per step (four 16-byte chunks)
constexpr uint32_t kLinkBuf = 4096;   // marker offsets staged per workgroup
constexpr uint32_t kLinkStepMax = kLinkFindThreads * (kLinkGroup / 9 + 1);  // markers one step can add
constexpr uint32_t kMarkW0 = 0x6820613Cu;  // '<' 'a' ' ' 'h'
constexpr uint32_t kMarkW1 = 0x3D666572u;  // 'r' 'e' 'f' '='
constexpr uint32_t kMarkW2 = 0x22u;        // '"'

// Bit i set when byte i of the 16-byte block may equal c (a superset of the
// true positions: each one is checked afterwards).
MR_DEV uint32_t byte_candidates16(uint4 b, uint32_t c) {
  const uint32_t rep = c * 0x01010101u;
  uint32_t m = 0;
  const uint32_t w[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t t = w[q] ^ rep;
    const uint32_t z = (t - 0x01010101u) & ~t & 0x80808080u;
    m |= (((z >> 7) & 1u) | ((z >> 14) & 2u) | ((z >> 21) & 4u) | ((z >> 28) & 8u)) << (4 * q);
  }
  return m;
}

__global__ void k_links_zero(unsigned long long* n_marks) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_marks = 0ull;
}

// Input offsets of every marker inside the valid byte range of job 0. Marks
// past mark_cap are counted but not stored (the caller grows the list and
// runs again).
__global__ __launch_bounds__(kLinkFindThreads) void k_links_find(const WordJob* __restrict__ jobs, uint32_t* __restrict__ marks,
                                                                 unsigned long long* __restrict__ n_marks, uint64_t mark_cap) {
  __shared__ uint32_t buf[kLinkBuf];
  __shared__ uint32_t cnt;
  __shared__ unsigned long long base;
  const WordJob J = jobs[0];
  const uint64_t a_in = (uint64_t)J.in;
  const uint64_t a0 = a_in + J.st->valid_lo, a1 = a_in + J.st->valid_hi;
  const uint64_t g0 = a0 / kLinkGroup, g1 = (a1 + kLinkGroup - 1) / kLinkGroup;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  auto flush = [&]() {
    if (threadIdx.x == 0) base = cnt ? atomicAdd(n_marks, (unsigned long long)cnt) : 0ull;
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cnt; i += blockDim.x)
      if (base + i < mark_cap) marks[base + i] = buf[i];
    __syncthreads();
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
  };
  // the step base is the same for every lane of the workgroup, so all lanes meet every barrier
  for (uint64_t step = g0 + (uint64_t)blockIdx.x * blockDim.x; step < g1; step += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t g = step + threadIdx.x;
    if (g < g1) {
      const uint64_t ga = g * kLinkGroup;
      uint4 blk[5];  // the group and the block after it (for markers that cross the group's end)
#pragma unroll
      for (int c = 0; c < 5; ++c) blk[c] = load_block(a0, a1, ga + 16ull * c);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        uint32_t cand = byte_candidates16(blk[c], '<');
        if (!cand) continue;
        const uint32_t w[8] = {blk[c].x, blk[c].y, blk[c].z, blk[c].w, blk[c + 1].x, blk[c + 1].y, blk[c + 1].z, blk[c + 1].w};
        while (cand) {
          const uint32_t sb = __builtin_ctz(cand);
          cand &= cand - 1;
          const uint64_t pa = ga + 16ull * c + sb;
          if (pa < a0 || pa + 9 > a1) continue;
          const uint4 k = extract16(w, sb, 9);
          if (k.x == kMarkW0 && k.y == kMarkW1 && k.z == kMarkW2) buf[atomicAdd(&cnt, 1u)] = (uint32_t)(pa - a_in);
        }
      }
    }
    __syncthreads();
    if (cnt > kLinkBuf - kLinkStepMax) flush();
  }
  __syncthreads();
  flush();
}

// One lane per marker: the record, the closing quote, the table insert and
// the (URL, record) pair: the URL's table slot, or all ones when the marker
// starts no link (or the table is full and the pass will be repeated).
__global__ __launch_bounds__(256) void k_links_insert(const WordJob* __restrict__ jobs, const uint32_t* __restrict__ marks,
                                                      const unsigned long long* __restrict__ n_marks, uint64_t mark_cap,
                                                      uint32_t* __restrict__ pair_slot, uint32_t* __restrict__ pair_file,
                                                      uint32_t debug_hash) {
  const WordJob J = jobs[0];
  const uint64_t nm = *n_marks < mark_cap ? *n_marks : mark_cap;
  const uint64_t vlo = J.st->valid_lo, vhi = J.st->valid_hi;
  const uint64_t a_in = (uint64_t)J.in;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nm; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t p = marks[i];
    uint64_t rend = vhi;
    uint32_t file = 0;
    bool ok = true;
    if (J.rec) {
      const uint64_t r = rec_lower_bound(J.rec, J.n_rec, p + 1);  // first record start above p
      ok = r >= 1 && r <= J.n_rec;
      if (ok) {
        file = (uint32_t)(r - 1);
        rend = J.rec[r] < vhi ? J.rec[r] : vhi;
      }
    }
    const uint64_t u = p + 9;
    ok = ok && u <= rend;
    uint64_t q = ~0ull;
    if (ok) {
      const uint64_t lim = (u + kLinkMaxUrl + 1) < rend ? (u + kLinkMaxUrl + 1) : rend;  // the quote lies in [u, lim)
      for (uint64_t blk = (a_in + u) & ~15ull; blk < a_in + lim && q == ~0ull; blk += 16) {
        const uint4 b = *reinterpret_cast<const uint4*>(blk);  // overlaps [in + u, in + lim), inside the input
        uint32_t m = byte_candidates16(b, '"');
        while (m) {
          const uint32_t sb = __builtin_ctz(m);
          m &= m - 1;
          const uint64_t at = blk + sb;
          if (at < a_in + u || at >= a_in + lim) continue;
          if (((sb < 4 ? b.x : sb < 8 ? b.y : sb < 12 ? b.z : b.w) >> (8 * (sb & 3)) & 0xFFu) != 0x22u) continue;
          q = at - a_in;
          break;
        }
      }
    }
    const uint64_t len = q != ~0ull ? q - u : 0ull;
    uint64_t slot = ~0ull;
    if (ok && len >= 1 && len <= kLinkMaxUrl) {
      const uint64_t h = key_hash_global(J.in, u, len, debug_hash);
      if (len <= 16) g_insert<true>(J, vlo, vhi, u, len, h, load_key16(J.in, u, (uint32_t)len), 0u, debug_hash, &slot);
      else g_insert<false>(J, vlo, vhi, u, len, h, make_uint4(0, 0, 0, 0), 0u, debug_hash, &slot);
    }
    pair_slot[i] = slot != ~0ull ? (uint32_t)slot : ~0u;
    pair_file[i] = file;
  }
}

__global__ void k_zero_states(JobState* st, uint32_t n) {
  uint32_t* p = reinterpret_cast<uint32_t*>(st);
  const uint32_t words = n * (uint32_t)(sizeof(JobState) / 4);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words; i += gridDim.x * blockDim.x) p[i] = 0u;
}

hipError_t words_enqueue_zero_states(const WordsLaunch& L, hipStream_t s) {
  // without record offsets the prep kernel clears each job's state itself
  if (L.any_records) hipLaunchKernelGGL(k_zero_states, dim3(1), dim3(256), 0, s, L.states, L.n_jobs);
  return hipGetLastError();
}

hipError_t words_enqueue_prep(const WordsLaunch& L, hipStream_t s) {
  if (L.any_records) {
    dim3 g(64, L.n_jobs);
    hipLaunchKernelGGL(k_words_prep, g, dim3(256), 0, s, L.jobs, L.n_jobs, 0u);
  } else {
    dim3 g(1, L.n_jobs);
    hipLaunchKernelGGL(k_words_prep, g, dim3(64), 0, s, L.jobs, L.n_jobs, 1u);
  }
  return hipGetLastError();
}

hipError_t words_enqueue_map(const WordsLaunch& L, hipStream_t s) {
  if (L.links) {
    hipLaunchKernelGGL(k_links_zero, dim3(1), dim3(64), 0, s, L.link_n);
    hipLaunchKernelGGL(k_links_find, dim3(L.link_grid), dim3(kLinkFindThreads), 0, s, L.jobs, L.link_marks, L.link_n,
                       L.link_cap);
    hipLaunchKernelGGL(k_links_insert, dim3(L.link_grid), dim3(256), 0, s, L.jobs, L.link_marks, L.link_n, L.link_cap,
                       L.link_pair_slot, L.link_pair_file, L.debug_hash);
    return hipGetLastError();
  }
  const dim3 grid(L.map_grid), block(kMapThreads);
#define MR_MAP_LAUNCH(LG, REC, CMB) \
  hipLaunchKernelGGL((k_words_map<LG, REC, CMB>), grid, block, 0, s, L.jobs, L.tile_base, L.n_jobs, L.total_tiles, L.debug_hash)
#define MR_MAP_CASE(LG)                                                   \
  case LG:                                                                 \
    if (L.any_records) {                                                   \
      if (L.wave_combine) MR_MAP_LAUNCH(LG, true, true);                   \
      else MR_MAP_LAUNCH(LG, true, false);                                 \
    } else {                                                               \
      if (L.wave_combine) MR_MAP_LAUNCH(LG, false, true);                  \
      else MR_MAP_LAUNCH(LG, false, false);                                \
    }                                                                      \
    break;
  switch (L.lds_log2) {
    MR_MAP_CASE(8)
    MR_MAP_CASE(10)
    MR_MAP_CASE(11)
    MR_MAP_CASE(12)
    default:
      return hipErrorInvalidValue;
  }
#undef MR_MAP_CASE
#undef MR_MAP_LAUNCH
  if (L.n_parts) hipLaunchKernelGGL((k_words_parts<12>), dim3(L.n_parts), dim3(kMapThreads), 0, s, L.jobs, L.debug_hash);
  return hipGetLastError();
}

hipError_t words_enqueue_reduce(const WordsLaunch& L, hipStream_t s) {
  const uint32_t item = L.total_slots <= (1ull << 20) ? kCompactSmall : kCompactLarge;
  const uint64_t tiles = (L.total_slots + item - 1) / item;
  const uint32_t cgrid = (uint32_t)(tiles < 4096 ? tiles : 4096);
  hipLaunchKernelGGL(k_words_compact, dim3(cgrid ? cgrid : 1), dim3(kCompactThreads), 0, s, L.jobs, L.n_jobs, L.total_slots,
                     item);
  if (L.n_jobs <= kRankJobs) {
    // plans the sort itself
    hipLaunchKernelGGL(k_sort_ranks, dim3(L.sort_grid), dim3(kSortThreads), 0, s, L.jobs, L.n_jobs, L.totals,
                       L.bucket_cnt, L.bucket_bytes, L.bucket_fill);
  } else {
    hipLaunchKernelGGL(k_sort_plan, dim3(1), dim3(kSortThreads), 0, s, L.jobs, L.n_jobs, L.totals);
    hipLaunchKernelGGL(k_sort_splitters, dim3(L.n_jobs), dim3(kSortThreads), 0, s, L.jobs, L.n_jobs, L.bucket_cnt,
                       L.bucket_bytes, L.bucket_fill);
  }
  hipLaunchKernelGGL(k_sort_count, dim3(L.sort_grid), dim3(256), 0, s, L.jobs, L.n_jobs, L.totals, L.bucket_cnt, L.bucket_bytes);
  hipLaunchKernelGGL(k_sort_scan, dim3(L.n_jobs), dim3(64), 0, s, L.jobs, L.n_jobs, L.bucket_cnt, L.bucket_bytes,
                     L.bucket_start, L.bucket_bstart);
  hipLaunchKernelGGL(k_sort_scatter, dim3(L.sort_grid), dim3(256), 0, s, L.jobs, L.n_jobs, L.totals, L.bucket_start,
                     L.bucket_fill);
  hipLaunchKernelGGL(k_sort_buckets, dim3(L.sort_grid), dim3(kBucketThreads), 0, s, L.jobs, L.n_jobs, L.totals, L.bucket_cnt,
                     L.bucket_bytes, L.bucket_start, L.bucket_bstart);
  return hipGetLastError();
}

}  // namespace mr
