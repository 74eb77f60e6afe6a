// Integer-key MapReduce on gfx950: four reduce containers for uint32 keys.
//
// map: element i emits (key_i, value_i) (value 1 for plain keys);
// reduce: COUNT, SUM (64-bit), MIN or MAX per distinct key; output ascending.
//
// Containers (Section III-A; the choice between the two arrays is the rule of
// Section III-E):
//   LDS_ARRAY    per-workgroup array in LDS for a small declared key range;
//                each workgroup writes its partial array, a second kernel
//                adds the partials key by key (no atomics on shared data).
//   GLOBAL_ARRAY one array over the declared range updated with atomics
//                ("eliminating local arrays"); lanes holding the same hot key
//                merge first so one atomic carries the wave's sum.
//   HASH         a per-workgroup LDS hash cache (the bounded local container of
//                Section III-D) in front of a global open-addressing table;
//                keys fit the CAS word, so claim and compare are one step.
//   SORT         LSD radix sort of the pairs, then a segmented reduce.
// Every container ends in a compaction to distinct keys in ascending order.
#include "common.h"
#include "launch.h"

namespace mr {

// value slot encodings (all start at zero)
//   COUNT: count            SUM: 64-bit sum
//   MIN:   ~min (atomicMax) MAX: max
MR_DEV uint32_t enc_minmax(int op, uint32_t v) { return op == 2 ? ~v : v; }
MR_DEV uint32_t dec_minmax(int op, uint32_t v) { return op == 2 ? ~v : v; }

// ----------------------------------------------------------------------------
// element access
// ----------------------------------------------------------------------------
struct IntIn {
  const uint32_t* p;  // keys, or interleaved (key, value) pairs
  uint64_t n;         // elements
  uint32_t kv;        // 1 when values are present
};

MR_DEV void load_elem(const IntIn& in, uint64_t i, uint32_t& k, uint32_t& v) {
  if (in.kv) {
    const uint2 e = reinterpret_cast<const uint2*>(in.p)[i];
    k = e.x;
    v = e.y;
  } else {
    k = in.p[i];
    v = 1u;
  }
}

// ----------------------------------------------------------------------------
// LDS array
// ----------------------------------------------------------------------------
constexpr int kIntThreads = 512;

// Partials layout: cnt_part[g * R + key], val_part[g * R + key] (val for SUM is 64-bit).
template <int OP>
__global__ __launch_bounds__(kIntThreads) void k_lds_array(IntIn in, uint32_t R, uint32_t G, uint32_t* __restrict__ cnt_part,
                                                           void* __restrict__ val_part, uint32_t* __restrict__ flags) {
  extern __shared__ uint8_t smem[];
  uint32_t* cnt = reinterpret_cast<uint32_t*>(smem);
  unsigned long long* sum = reinterpret_cast<unsigned long long*>(smem + ((4ull * R + 7) & ~7ull));
  uint32_t* mm = reinterpret_cast<uint32_t*>(smem + 4ull * R);
  for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) {
    cnt[i] = 0;
    if (OP == 1) sum[i] = 0;
    if (OP >= 2) mm[i] = 0;
  }
  __syncthreads();
  const uint64_t lo = in.n * blockIdx.x / G, hi = in.n * (blockIdx.x + 1) / G;
  bool bad = false;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    uint32_t k, v;
    load_elem(in, i, k, v);
    if (k >= R) {
      bad = true;
      continue;
    }
    atomicAdd(&cnt[k], 1u);
    if (OP == 1) atomicAdd(&sum[k], (unsigned long long)v);
    if (OP >= 2) atomicMax(&mm[k], enc_minmax(OP, v));
  }
  if (bad) atomicOr(flags, kFlagBadInput);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < R; i += blockDim.x) {
    cnt_part[(uint64_t)blockIdx.x * R + i] = cnt[i];
    if (OP == 1) reinterpret_cast<unsigned long long*>(val_part)[(uint64_t)blockIdx.x * R + i] = sum[i];
    if (OP >= 2) reinterpret_cast<uint32_t*>(val_part)[(uint64_t)blockIdx.x * R + i] = mm[i];
  }
}

// Dense arrays (count, value) from the partials: one thread per key.
template <int OP>
__global__ __launch_bounds__(256) void k_lds_array_reduce(uint32_t R, uint32_t G, const uint32_t* __restrict__ cnt_part,
                                                          const void* __restrict__ val_part, uint32_t* __restrict__ dcnt,
                                                          void* __restrict__ dval) {
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < R; k += gridDim.x * blockDim.x) {
    uint32_t c = 0;
    unsigned long long s = 0;
    uint32_t m = 0;
    for (uint32_t g = 0; g < G; ++g) {
      c += cnt_part[(uint64_t)g * R + k];
      if (OP == 1) s += reinterpret_cast<const unsigned long long*>(val_part)[(uint64_t)g * R + k];
      if (OP >= 2) m = max(m, reinterpret_cast<const uint32_t*>(val_part)[(uint64_t)g * R + k]);
    }
    dcnt[k] = c;
    if (OP == 1) reinterpret_cast<unsigned long long*>(dval)[k] = s;
    if (OP >= 2) reinterpret_cast<uint32_t*>(dval)[k] = m;
  }
}

// ----------------------------------------------------------------------------
// global array with wave-level aggregation
// ----------------------------------------------------------------------------

// Merge lanes that hold the same key as the current leader, for a few rounds:
// hot keys leave the wave as one atomic; the rest update directly.
constexpr int kAggRounds = 4;

template <int OP>
MR_DEV void wave_combine(uint32_t k, uint32_t v, bool active, uint32_t& cnt_out, unsigned long long& sum_out,
                         uint32_t& mm_out, bool& leader) {
  cnt_out = 0;
  sum_out = 0;
  mm_out = 0;
  leader = false;
  bool pending = active;
#pragma unroll 1
  for (int r = 0; r < kAggRounds; ++r) {
    const uint64_t m = __ballot(pending);
    if (!m) return;
    const int ld = __ffsll((long long)m) - 1;
    const uint32_t lk = __shfl(k, ld);
    const bool same = pending && k == lk;
    const uint64_t grp = __ballot(same);
    // reductions over the group
    unsigned long long s = same ? (unsigned long long)v : 0ull;
    uint32_t mx = same ? enc_minmax(OP, v) : 0u;
    if (OP == 1) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    }
    if (OP >= 2) {
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor((int)mx, o));
    }
    if ((int)lane_id() == ld) {
      leader = true;
      cnt_out = popc64(grp);
      sum_out = s;
      mm_out = mx;
    }
    if (same) pending = false;
  }
  if (pending) {  // not merged: update alone
    leader = true;
    cnt_out = 1;
    sum_out = v;
    mm_out = enc_minmax(OP, v);
  }
}

template <int OP>
__global__ __launch_bounds__(256) void k_global_array(IntIn in, uint32_t R, uint32_t* __restrict__ dcnt, void* __restrict__ dval,
                                                      uint32_t* __restrict__ flags) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  const uint64_t n_round = (in.n + stride - 1) / stride * stride;  // all lanes iterate together
  bool bad = false;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_round; i += stride) {
    uint32_t k = 0, v = 0;
    bool act = i < in.n;
    if (act) {
      load_elem(in, i, k, v);
      if (k >= R) {
        bad = true;
        act = false;
      }
    }
    uint32_t c, mm;
    unsigned long long s;
    bool lead;
    wave_combine<OP>(k, v, act, c, s, mm, lead);
    if (lead && c) {
      // a leader's own key is k (it leads its own group)
      atomicAdd(&dcnt[k], c);
      if (OP == 1) atomicAdd(&reinterpret_cast<unsigned long long*>(dval)[k], s);
      if (OP >= 2) atomicMax(&reinterpret_cast<uint32_t*>(dval)[k], mm);
    }
  }
  if (bad) atomicOr(flags, kFlagBadInput);
}

// ----------------------------------------------------------------------------
// global array over a large range, filled by key-range partitions (COUNT)
//
// Device-scope atomics run far below the load rate, so a large array is not
// updated element by element. Instead each tile of elements is ordered by
// 2^15-key range in LDS and written where it stands, as the elements' low 15
// bits, with the start of each range's run in the tile; then one workgroup
// per range counts that range's runs of every tile in an LDS array and
// writes the range's counts once. Every array entry is written exactly once;
// no global atomics on the array.
// ----------------------------------------------------------------------------
constexpr uint32_t kPartBits = 15;
constexpr uint32_t kPartKeys = 1u << kPartBits;  // keys per range: LDS counters of one workgroup (128 KB)
constexpr uint32_t kMaxParts = 2048;             // ranges (key range up to 2^26)
constexpr uint32_t kPartTile = 16384;            // elements per tile (a multiple of 8)
constexpr uint32_t kPartThreads = 1024;
static_assert(kPartTile % (4 * kPartThreads) == 0, "a held tile is whole 16-byte vectors, the same number per thread");
constexpr uint32_t kCompTile = 2048;  // keys per block of the ordered compaction of dense arrays (256 threads x 8)
static_assert(kPartKeys % kCompTile == 0, "a key range holds whole compaction blocks");

// Element i of a tile: keys are read 4 at a time (one 16-byte load) when the
// input is plain keys; pairs are read one by one.
template <typename F>
MR_DEV void for_tile_keys(const IntIn& in, uint64_t base, F&& f) {
  if (!in.kv && ((uintptr_t)in.p & 15u) == 0) {
    const uint64_t end = base + kPartTile < in.n ? base + kPartTile : in.n;
    const uint64_t nv = end > base ? (end - base) / 4 : 0;  // whole vectors
    const uint4* v = reinterpret_cast<const uint4*>(in.p + base);
    // loads in batches of kTileBatch per lane, issued before any of them is used
    constexpr uint32_t kTileBatch = 4;
    uint64_t q = threadIdx.x;
    for (; q + (kTileBatch - 1) * blockDim.x < nv; q += kTileBatch * blockDim.x) {
      uint4 x[kTileBatch];
#pragma unroll
      for (uint32_t u = 0; u < kTileBatch; ++u) x[u] = gload16(v + q + u * blockDim.x);
#pragma unroll
      for (uint32_t u = 0; u < kTileBatch; ++u) {
        f(x[u].x);
        f(x[u].y);
        f(x[u].z);
        f(x[u].w);
      }
    }
    for (; q < nv; q += blockDim.x) {
      const uint4 x = gload16(v + q);
      f(x.x);
      f(x.y);
      f(x.z);
      f(x.w);
    }
    for (uint64_t i = base + nv * 4 + threadIdx.x; i < end; i += blockDim.x) f(in.p[i]);
  } else {
    for (uint32_t q = threadIdx.x; q < kPartTile; q += blockDim.x) {
      const uint64_t i = base + q;
      if (i >= in.n) break;
      uint32_t k, v;
      load_elem(in, i, k, v);
      f(k);
    }
  }
}

// Dynamic LDS of k_part_tile: the range arrays, sized by P, so that for
// P <= 1024 two workgroups fit a CU (one streams its tile while the other
// scans its counts or writes its row).
constexpr uint32_t part_tile_lds(uint32_t P) { return (2 * P + 1) * 4; }

// Tile t writes its elements' in-range offsets ordered by range to
// part[t * kPartTile, ...) and the start of each range's run in the tile to
// runs[t * (P + 1) + p] (entry P: the tile's element count), both as whole
// contiguous rows.
__global__ __launch_bounds__(kPartThreads) void k_part_tile(IntIn in, uint64_t R, uint32_t P, uint32_t* __restrict__ runs,
                                                            uint16_t* __restrict__ part, uint32_t* __restrict__ flags) {
  extern __shared__ uint32_t ranges[];
  uint32_t* const lbase = ranges;         // [P + 1] start of each range's run in the tile (and the end)
  uint32_t* const lpos = ranges + P + 1;  // [P] counts, then the next free place of each range's run
  __shared__ __attribute__((aligned(16))) uint16_t sk[kPartTile];  // staged offsets, ordered by range
  __shared__ uint32_t wsum[kPartThreads / kWave];
  const uint32_t t = blockIdx.x;
  for (uint32_t q = threadIdx.x; q < P; q += blockDim.x) lpos[q] = 0u;
  __syncthreads();
  // A whole tile of aligned plain keys is held in registers between the count
  // and the placing (four 16-byte vectors per thread); other tiles are read
  // twice.
  constexpr uint32_t kHeld = kPartTile / 4 / kPartThreads;
  const bool held = !in.kv && ((uintptr_t)in.p & 15u) == 0 && (uint64_t)(t + 1) * kPartTile <= in.n &&
                    blockDim.x == kPartThreads;
  uint4 x[kHeld];
  // 1. the tile's count of each range
  bool bad = false;
  auto count = [&](uint32_t k) {
    if (k < R) atomicAdd(&lpos[k >> kPartBits], 1u);
    else bad = true;
  };
  if (held) {
    const uint4* v = reinterpret_cast<const uint4*>(in.p + (uint64_t)t * kPartTile);
#pragma unroll
    for (uint32_t u = 0; u < kHeld; ++u) x[u] = gload16(v + threadIdx.x + u * kPartThreads);
#pragma unroll
    for (uint32_t u = 0; u < kHeld; ++u) {
      count(x[u].x);
      count(x[u].y);
      count(x[u].z);
      count(x[u].w);
    }
  } else {
    for_tile_keys(in, (uint64_t)t * kPartTile, count);
  }
  if (bad) atomicOr(flags, kFlagBadInput);
  __syncthreads();
  // 2. run starts: exclusive scan of the counts (P <= kMaxParts: kPer per thread)
  constexpr uint32_t kPer = kMaxParts / kPartThreads;
  uint32_t c[kPer], sum = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t r = threadIdx.x * kPer + q;
    c[q] = r < P ? lpos[r] : 0u;
    sum += c[q];
  }
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  const uint32_t incl = wave_incl_scan(sum);
  if (lane == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  uint32_t pre = 0, m = 0;
  for (uint32_t w = 0; w < kPartThreads / kWave; ++w) {
    if (w < wv) pre += wsum[w];
    m += wsum[w];
  }
  uint32_t run = pre + incl - sum;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t r = threadIdx.x * kPer + q;
    if (r < P) {
      lbase[r] = run;
      lpos[r] = run;
    }
    run += c[q];
  }
  if (threadIdx.x == 0) lbase[P] = m;
  __syncthreads();
  uint32_t* const row = runs + (uint64_t)t * (P + 1);
  for (uint32_t q = threadIdx.x; q <= P; q += blockDim.x) row[q] = lbase[q];
  // 3. each element to its place
  auto place = [&](uint32_t k) {
    if (k < R) sk[atomicAdd(&lpos[k >> kPartBits], 1u)] = (uint16_t)(k & (kPartKeys - 1));
  };
  if (held) {
#pragma unroll
    for (uint32_t u = 0; u < kHeld; ++u) {
      place(x[u].x);
      place(x[u].y);
      place(x[u].z);
      place(x[u].w);
    }
  } else {
    for_tile_keys(in, (uint64_t)t * kPartTile, place);
  }
  __syncthreads();
  // 4. the staged offsets as one row, eight per 16-byte store
  uint16_t* const dst = part + (uint64_t)t * kPartTile;
  for (uint32_t i = threadIdx.x; i * 8u < m; i += blockDim.x) {
    if (i * 8u + 8u <= m) {
      gstore16(dst + i * 8u, *reinterpret_cast<const uint4*>(&sk[i * 8u]));
    } else {
      for (uint32_t e = i * 8u; e < m; ++e) dst[e] = sk[e];
    }
  }
}

// One workgroup per key range counts the range's runs of every tile in LDS
// (a thread takes whole tiles: it loads its tiles' run bounds together, then
// a run's covering 16-byte pieces, up to kFillVecs at once, before it counts
// them) and writes the range's counts once, with the present keys per
// compaction block (the ordered compaction's first pass, done here).
constexpr uint32_t kFillTilesPer = 8;  // tiles a thread takes at a time
constexpr uint32_t kFillVecs = 12;     // 16-byte pieces of a run loaded before counting

__global__ __launch_bounds__(1024) void k_part_fill_tiles(const uint16_t* __restrict__ part, const uint32_t* __restrict__ runs,
                                                          uint32_t P, uint32_t n_tiles, uint64_t R,
                                                          uint32_t* __restrict__ dcnt, uint32_t* __restrict__ blk) {
  __shared__ uint32_t c[kPartKeys + kWave / 2];  // the range's counters, then 32 sinks for entries outside a run
  // Workgroups are handed to the eight XCDs in turn; neighbouring ranges read
  // neighbouring words of every tile's run-start row and share the 128-byte
  // lines where their runs meet, so each XCD takes a contiguous block of
  // ranges and its L2 serves those lines once. The map is a permutation of
  // the ranges: another dispatch order costs cache hits, not correctness.
  const uint32_t p = (P % kXcds == 0u) ? (blockIdx.x % kXcds) * (P / kXcds) + blockIdx.x / kXcds : blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kPartKeys; i += blockDim.x) c[i] = 0;
  __syncthreads();
  const uint32_t sink = kPartKeys + (threadIdx.x & (kWave / 2 - 1));
  for (uint32_t t0 = 0; t0 < n_tiles; t0 += kFillTilesPer * blockDim.x) {
    uint32_t b0[kFillTilesPer], b1[kFillTilesPer];
#pragma unroll
    for (uint32_t u = 0; u < kFillTilesPer; ++u) {
      const uint32_t t = t0 + u * blockDim.x + threadIdx.x;
      b0[u] = b1[u] = 0u;
      if (t < n_tiles) {
        const uint32_t* row = runs + (uint64_t)t * (P + 1) + p;
        b0[u] = *gp(row);
        b1[u] = *gp(row + 1);
      }
    }
#pragma unroll 1
    for (uint32_t u = 0; u < kFillTilesPer; ++u) {
      const uint16_t* src = part + (uint64_t)(t0 + u * blockDim.x + threadIdx.x) * kPartTile;
      // the run [b0, b1) read as the aligned 16-byte pieces that cover it
      // (inside the tile's row, whose length is a multiple of 8 entries),
      // the entries outside it counted in a sink
      const uint32_t lo = b0[u], hi = b1[u];
      for (uint32_t v = lo & ~7u; v < hi; v += 8u * kFillVecs) {
        uint4 x[kFillVecs];
#pragma unroll
        for (uint32_t q = 0; q < kFillVecs; ++q)
          if (v + 8u * q < hi) x[q] = gload16(src + v + 8u * q);
#pragma unroll
        for (uint32_t q = 0; q < kFillVecs; ++q) {
          const uint32_t e0 = v + 8u * q;
          if (e0 >= hi) continue;
          // eight atomics whatever the piece's overlap with the run: an entry
          // outside it goes to one of the sinks, spread over the banks
          const uint32_t w[4] = {x[q].x, x[q].y, x[q].z, x[q].w};
#pragma unroll
          for (uint32_t i = 0; i < 8u; ++i) {
            const uint32_t key = (w[i >> 1] >> (16u * (i & 1u))) & 0xFFFFu;
            atomicAdd(&c[e0 + i - lo < hi - lo ? key : sink], 1u);
          }
        }
      }
    }
  }
  __syncthreads();
  const uint64_t key0 = (uint64_t)p * kPartKeys;
  const uint32_t nk = (uint32_t)(R - key0 < kPartKeys ? R - key0 : kPartKeys);
  for (uint32_t i = threadIdx.x; i < nk; i += blockDim.x) dcnt[key0 + i] = c[i];
  const uint32_t lane = lane_id();
  for (uint32_t b = threadIdx.x / kWave; b * kCompTile < nk; b += blockDim.x / kWave) {
    const uint32_t q1 = (b + 1) * kCompTile < nk ? (b + 1) * kCompTile : nk;
    uint32_t present = 0;
    for (uint32_t q = b * kCompTile; q < q1; q += kWave) {
      const uint32_t i = q + lane;
      present += (uint32_t)__popcll(__ballot(i < q1 && c[i] != 0));
    }
    if (lane == 0) blk[key0 / kCompTile + b] = present;
  }
}

// ----------------------------------------------------------------------------
// ordered compaction of dense arrays: keys with count > 0, ascending
// ----------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_dense_count(const uint32_t* __restrict__ dcnt, uint32_t R, uint32_t* __restrict__ blk) {
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kCompTile;
  uint32_t c = 0;
  for (uint32_t q = threadIdx.x; q < kCompTile; q += blockDim.x) {
    const uint64_t k = base + q;
    if (k < R && dcnt[k]) ++c;
  }
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) blk[blockIdx.x] = s;
}

// Exclusive scan of blk[0, nb) in place by one workgroup; total in *total.
__global__ __launch_bounds__(1024) void k_scan_small(uint32_t* __restrict__ blk, uint32_t nb, unsigned long long* total) {
  __shared__ uint32_t ws[1024 / kWave];
  uint32_t carry = 0;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  for (uint32_t base = 0; base < nb; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    const uint32_t x = i < nb ? blk[i] : 0u;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o);
      if (lane >= (uint32_t)o) inc += t;
    }
    if (lane == kWave - 1) ws[wv] = inc;
    __syncthreads();
    uint32_t pre = carry, tot = 0;
    for (uint32_t q = 0; q < blockDim.x / kWave; ++q) {
      if (q < wv) pre += ws[q];
      tot += ws[q];
    }
    if (i < nb) blk[i] = pre + inc - x;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Write the present keys of a dense array in order and clear the arrays.
template <int OP>
__global__ __launch_bounds__(256) void k_dense_write(uint32_t* __restrict__ dcnt, void* __restrict__ dval, uint32_t R,
                                                     const uint32_t* __restrict__ blk, uint32_t* __restrict__ out_keys,
                                                     void* __restrict__ out_vals, uint64_t cap, bool clear) {
  __shared__ uint32_t wsum[256 / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kCompTile;
  uint32_t carry = blk[blockIdx.x];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  for (uint32_t q0 = 0; q0 < kCompTile; q0 += blockDim.x) {
    const uint64_t k = base + q0 + threadIdx.x;
    uint32_t c = 0;
    if (k < R) c = dcnt[k];
    const bool p = c != 0;
    const uint64_t m = __ballot(p);
    if (lane == 0) wsum[wv] = popc64(m);
    __syncthreads();
    uint32_t pre = carry, tot = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) {
      if (w < wv) pre += wsum[w];
      tot += wsum[w];
    }
    if (p) {
      const uint64_t o = pre + mbcnt(m);
      if (o < cap) {
        out_keys[o] = (uint32_t)k;
        if (OP == 0) reinterpret_cast<uint32_t*>(out_vals)[o] = c;
        if (OP == 1) reinterpret_cast<unsigned long long*>(out_vals)[o] = reinterpret_cast<unsigned long long*>(dval)[k];
        if (OP >= 2) reinterpret_cast<uint32_t*>(out_vals)[o] = dec_minmax(OP, reinterpret_cast<uint32_t*>(dval)[k]);
      }
      if (clear) {
        dcnt[k] = 0;
        if (OP == 1) reinterpret_cast<unsigned long long*>(dval)[k] = 0;
        if (OP >= 2) reinterpret_cast<uint32_t*>(dval)[k] = 0;
      }
    }
    carry += tot;
    __syncthreads();
  }
}

// ----------------------------------------------------------------------------
// hash: LDS cache + global open-addressing table
// ----------------------------------------------------------------------------
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;  // key 0xFFFFFFFF itself is kept in a side slot

struct IntTable {
  uint32_t* keys;             // [cap], kEmptyKey when free
  uint32_t* cnt;              // [cap]
  void* val;                  // [cap] (64-bit for SUM)
  uint64_t cap;               // power of two
  uint32_t* claimed;          // slots claimed, in claim order
  unsigned long long* n_claimed;
  uint32_t* side_cnt;         // key 0xFFFFFFFF: count and value
  void* side_val;
  uint32_t* flags;
};

template <int OP>
MR_DEV void apply_global(const IntTable& T, uint64_t i, uint32_t c, unsigned long long s, uint32_t mm) {
  atomicAdd(&T.cnt[i], c);
  if (OP == 1) atomicAdd(&reinterpret_cast<unsigned long long*>(T.val)[i], s);
  if (OP >= 2) atomicMax(&reinterpret_cast<uint32_t*>(T.val)[i], mm);
}

template <int OP>
MR_DEV void g_int_insert(const IntTable& T, uint32_t k, uint32_t c, unsigned long long s, uint32_t mm, uint32_t debug_hash) {
  if (k == kEmptyKey) {
    atomicAdd(T.side_cnt, c);
    if (OP == 1) atomicAdd(reinterpret_cast<unsigned long long*>(T.side_val), s);
    if (OP >= 2) atomicMax(reinterpret_cast<uint32_t*>(T.side_val), mm);
    return;
  }
  const uint64_t mask = T.cap - 1;
  uint64_t i = (debug_hash ? 0ull : hash_u32(k)) & mask;
  for (uint64_t p = 0; p <= mask; ++p) {
    uint32_t cur = __hip_atomic_load(&T.keys[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (cur == kEmptyKey) {
      cur = atomicCAS(&T.keys[i], kEmptyKey, k);
      if (cur == kEmptyKey) {
        T.claimed[wave_claim(T.n_claimed)] = (uint32_t)i;
        apply_global<OP>(T, i, c, s, mm);
        return;
      }
    }
    if (cur == k) {
      apply_global<OP>(T, i, c, s, mm);
      return;
    }
    i = (i + 1) & mask;
    if ((p & 255u) == 255u && (__hip_atomic_load(T.flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kFlagTableFull)) return;
  }
  atomicOr(T.flags, kFlagTableFull);
}

template <int OP, int L>
__global__ __launch_bounds__(kIntThreads) void k_int_hash(IntIn in, IntTable T, uint32_t G, uint32_t debug_hash, uint64_t R) {
  constexpr uint32_t S = 1u << L;
  __shared__ uint32_t lk[S];
  __shared__ uint32_t lc[S];
  __shared__ unsigned long long ls[OP == 1 ? S : 1];
  __shared__ uint32_t lm[OP >= 2 ? S : 1];
  for (uint32_t i = threadIdx.x; i < S; i += blockDim.x) {
    lk[i] = kEmptyKey;
    lc[i] = 0;
    if (OP == 1) ls[i] = 0;
    if (OP >= 2) lm[i] = 0;
  }
  __syncthreads();
  const uint64_t lo = in.n * blockIdx.x / G, hi = in.n * (blockIdx.x + 1) / G;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    uint32_t k, v;
    load_elem(in, i, k, v);
    if (R && k >= R) atomicOr(T.flags, kFlagBadInput);
    bool done = false;
    if (k != kEmptyKey) {
      uint32_t s = (uint32_t)(debug_hash ? 0ull : hash_u32(k)) & (S - 1);
#pragma unroll 1
      for (int p = 0; p < 16; ++p) {
        uint32_t cur = lk[s];
        if (cur == kEmptyKey) cur = atomicCAS(&lk[s], kEmptyKey, k);
        if (cur == kEmptyKey || cur == k) {
          atomicAdd(&lc[s], 1u);
          if (OP == 1) atomicAdd(&ls[s], (unsigned long long)v);
          if (OP >= 2) atomicMax(&lm[s], enc_minmax(OP, v));
          done = true;
          break;
        }
        s = (s + 1) & (S - 1);
      }
    }
    if (!done) g_int_insert<OP>(T, k, 1u, v, enc_minmax(OP, v), debug_hash);
  }
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < S; s += blockDim.x) {
    if (lk[s] != kEmptyKey && lc[s])
      g_int_insert<OP>(T, lk[s], lc[s], OP == 1 ? ls[s] : 0ull, OP >= 2 ? lm[s] : 0u, debug_hash);
  }
}

// Claimed slots -> (key, value) records; slots are cleared for reuse.
template <int OP>
__global__ __launch_bounds__(256) void k_int_gather(IntTable T, uint32_t* __restrict__ rk, unsigned long long* __restrict__ rv) {
  const uint64_t n = *T.n_claimed;
  for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < n; q += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t i = T.claimed[q];
    rk[q] = T.keys[i];
    unsigned long long v;
    if (OP == 0) v = T.cnt[i];
    else if (OP == 1) v = reinterpret_cast<unsigned long long*>(T.val)[i];
    else v = dec_minmax(OP, reinterpret_cast<uint32_t*>(T.val)[i]);
    rv[q] = v;
    T.keys[i] = kEmptyKey;
    T.cnt[i] = 0;
    if (OP == 1) reinterpret_cast<unsigned long long*>(T.val)[i] = 0;
    if (OP >= 2) reinterpret_cast<uint32_t*>(T.val)[i] = 0;
  }
}

// ----------------------------------------------------------------------------
// LSD radix sort of (u64 key, u64 value) records, 8-bit digits, stable
// ----------------------------------------------------------------------------
constexpr uint32_t kSortTile = 2048;  // elements per block (256 threads x 8)

__global__ __launch_bounds__(256) void k_radix_hist(const unsigned long long* __restrict__ key, uint64_t n, int shift,
                                                    uint32_t n_tiles, uint32_t* __restrict__ hist /* [256][n_tiles] */) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  for (uint32_t q = threadIdx.x; q < kSortTile; q += blockDim.x) {
    const uint64_t i = base + q;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(uint64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// Device-wide exclusive scan of a (in place): per-block sums, scan of sums, add back.
constexpr uint32_t kScanTile = 4096;

__global__ __launch_bounds__(256) void k_scan_blocks(const uint32_t* __restrict__ a, uint64_t n, uint32_t* __restrict__ sums) {
  __shared__ uint32_t s;
  if (threadIdx.x == 0) s = 0;
  __syncthreads();
  uint32_t c = 0;
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  for (uint32_t q = threadIdx.x; q < kScanTile; q += blockDim.x)
    if (base + q < n) c += a[base + q];
  atomicAdd(&s, c);
  __syncthreads();
  if (threadIdx.x == 0) sums[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_scan_apply(uint32_t* __restrict__ a, uint64_t n, const uint32_t* __restrict__ sums) {
  __shared__ uint32_t ws[256 / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
  uint32_t carry = sums[blockIdx.x];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  for (uint32_t q0 = 0; q0 < kScanTile; q0 += blockDim.x) {
    const uint64_t i = base + q0 + threadIdx.x;
    const uint32_t x = i < n ? a[i] : 0u;
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o);
      if (lane >= (uint32_t)o) inc += t;
    }
    if (lane == kWave - 1) ws[wv] = inc;
    __syncthreads();
    uint32_t pre = carry, tot = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) {
      if (w < wv) pre += ws[w];
      tot += ws[w];
    }
    if (i < n) a[i] = pre + inc - x;
    carry += tot;
    __syncthreads();
  }
}

// Stable scatter: each tile sorts itself by the digit in LDS with eight
// one-bit splits, then writes each element to its digit's global offset.
__global__ __launch_bounds__(256) void k_radix_scatter(const unsigned long long* __restrict__ key_in,
                                                       const unsigned long long* __restrict__ val_in, uint64_t n, int shift,
                                                       uint32_t n_tiles, const uint32_t* __restrict__ hist,
                                                       unsigned long long* __restrict__ key_out,
                                                       unsigned long long* __restrict__ val_out) {
  __shared__ unsigned long long sk[kSortTile];
  __shared__ unsigned long long sv[kSortTile];
  __shared__ uint32_t dstart[256];
  __shared__ uint32_t dcount[256];
  __shared__ uint32_t ws[256 / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kSortTile;
  const uint32_t m = (uint32_t)((n - base) < kSortTile ? (n - base) : kSortTile);
  constexpr uint32_t E = kSortTile / 256;
  // each thread owns E consecutive elements
  unsigned long long k[E], v[E];
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t li = threadIdx.x * E + e;
    if (li < m) {
      k[e] = key_in[base + li];
      v[e] = val_in[base + li];
    } else {
      k[e] = ~0ull;  // padding sorts last and is never written
      v[e] = 0;
    }
  }
  dcount[threadIdx.x] = 0;
  __syncthreads();
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  for (int bit = 0; bit < 8; ++bit) {
    uint32_t ones = 0;
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) ones += (uint32_t)((k[e] >> (shift + bit)) & 1ull);
    const uint32_t zeros = E - ones;
    // block exclusive scan of zeros (DPP lane shifts within the wave)
    const uint32_t inc = wave_incl_scan(zeros);
    if (lane == kWave - 1) ws[wv] = inc;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
    for (uint32_t w = 0; w < 256 / kWave; ++w) {
      if (w < wv) pre += ws[w];
      tot += ws[w];
    }
    uint32_t zpos = pre + inc - zeros;               // zeros before this thread
    uint32_t opos = tot + threadIdx.x * E - zpos;     // ones before this thread, after all zeros
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      const bool one = (k[e] >> (shift + bit)) & 1ull;
      const uint32_t dst = one ? opos++ : zpos++;
      sk[dst] = k[e];
      sv[dst] = v[e];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t e = 0; e < E; ++e) {
      k[e] = sk[threadIdx.x * E + e];
      v[e] = sv[threadIdx.x * E + e];
    }
    __syncthreads();
  }
  // per-digit start within the tile, from the locally sorted order
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t li = threadIdx.x * E + e;
    if (li < m) atomicAdd(&dcount[(k[e] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  {
    const uint32_t x = dcount[threadIdx.x];
    uint32_t inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t t = __shfl_up(inc, o);
      if (lane >= (uint32_t)o) inc += t;
    }
    if (lane == kWave - 1) ws[wv] = inc;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t w = 0; w < wv; ++w) pre += ws[w];
    dstart[threadIdx.x] = pre + inc - x;
  }
  __syncthreads();
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t li = threadIdx.x * E + e;
    if (li < m) {
      const uint32_t d = (uint32_t)((k[e] >> shift) & 0xFFu);
      const uint64_t dst = (uint64_t)hist[(uint64_t)d * n_tiles + blockIdx.x] + (li - dstart[d]);
      key_out[dst] = k[e];
      val_out[dst] = v[e];
    }
  }
}

// ----------------------------------------------------------------------------
// sort strategy: build records, reduce runs
// ----------------------------------------------------------------------------

// Records for the sort: COUNT/SUM sort by key with the value alongside; MIN/MAX
// sort by (key << 32 | value), so each run starts with its minimum and ends
// with its maximum.
__global__ void k_sort_records(IntIn in, int op, uint64_t R, uint32_t* flags, unsigned long long* __restrict__ rk,
                               unsigned long long* __restrict__ rv) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < in.n; i += (uint64_t)gridDim.x * blockDim.x) {
    uint32_t k, v;
    load_elem(in, i, k, v);
    if (R && k >= R) atomicOr(flags, kFlagBadInput);
    rk[i] = op >= 2 ? (((unsigned long long)k << 32) | v) : (unsigned long long)k;
    rv[i] = v;
  }
}

// head[i] = 1 where a run of equal keys starts (key = bits 32.. for MIN/MAX).
__global__ void k_run_heads(const unsigned long long* __restrict__ rk, uint64_t n, int op, uint32_t* __restrict__ head) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t a = op >= 2 ? (rk[i] >> 32) : rk[i];
    const uint64_t b = i ? (op >= 2 ? (rk[i - 1] >> 32) : rk[i - 1]) : ~0ull;
    head[i] = (i == 0 || a != b) ? 1u : 0u;
  }
}

// Inclusive 64-bit prefix sums of the values (for SUM runs), in place: per-block
// partial sums are computed first, then added. Simple two-pass version.
constexpr uint32_t kPsTile = 4096;

__global__ __launch_bounds__(256) void k_ps64_blocks(const unsigned long long* __restrict__ a, uint64_t n,
                                                     unsigned long long* __restrict__ sums) {
  __shared__ unsigned long long s[256 / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kPsTile;
  unsigned long long c = 0;
  for (uint32_t q = threadIdx.x; q < kPsTile; q += blockDim.x)
    if (base + q < n) c += a[base + q];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o);
  if (lane_id() == 0) s[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < 256 / kWave; ++w) t += s[w];
    sums[blockIdx.x] = t;
  }
}

__global__ void k_ps64_scan_sums(unsigned long long* sums, uint32_t nb) {
  if (threadIdx.x || blockIdx.x) return;
  unsigned long long c = 0;
  for (uint32_t b = 0; b < nb; ++b) {
    const unsigned long long x = sums[b];
    sums[b] = c;
    c += x;
  }
}

__global__ __launch_bounds__(256) void k_ps64_apply(unsigned long long* __restrict__ a, uint64_t n,
                                                    const unsigned long long* __restrict__ sums) {
  __shared__ unsigned long long ws[256 / kWave];
  const uint64_t base = (uint64_t)blockIdx.x * kPsTile;
  unsigned long long carry = sums[blockIdx.x];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  for (uint32_t q0 = 0; q0 < kPsTile; q0 += blockDim.x) {
    const uint64_t i = base + q0 + threadIdx.x;
    const unsigned long long x = i < n ? a[i] : 0ull;
    unsigned long long inc = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const unsigned long long t = __shfl_up(inc, o);
      if (lane >= (uint32_t)o) inc += t;
    }
    if (lane == kWave - 1) ws[wv] = inc;
    __syncthreads();
    unsigned long long pre = carry, tot = 0;
    for (uint32_t w = 0; w < blockDim.x / kWave; ++w) {
      if (w < wv) pre += ws[w];
      tot += ws[w];
    }
    if (i < n) a[i] = pre + inc;  // inclusive
    carry += tot;
    __syncthreads();
  }
}

// Start position of every run: hpos[pos[i]] = i for each head i, and
// hpos[n_runs] = n.
__global__ void k_run_starts(const uint32_t* __restrict__ head, const uint32_t* __restrict__ pos, uint64_t n,
                             const unsigned long long* __restrict__ n_runs, uint32_t* __restrict__ hpos) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x)
    if (head[i]) hpos[pos[i]] = (uint32_t)i;
  if (blockIdx.x == 0 && threadIdx.x == 0) hpos[*n_runs] = (uint32_t)n;
}

// One output per run [hpos[r], hpos[r + 1]). COUNT: the run length; SUM: the
// difference of inclusive prefix sums; MIN / MAX: the first / last value
// (records were sorted by key then value).
__global__ void k_run_write(const unsigned long long* __restrict__ rk, const unsigned long long* __restrict__ ps,
                            const uint32_t* __restrict__ hpos, const unsigned long long* __restrict__ n_runs, int op,
                            uint32_t* __restrict__ out_keys, void* __restrict__ out_vals, uint64_t cap) {
  const uint64_t R = *n_runs;
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < R && r < cap; r += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t b = hpos[r], e = hpos[r + 1];
    out_keys[r] = (uint32_t)(op >= 2 ? (rk[b] >> 32) : rk[b]);
    if (op == 0) reinterpret_cast<uint32_t*>(out_vals)[r] = (uint32_t)(e - b);
    else if (op == 1) reinterpret_cast<unsigned long long*>(out_vals)[r] = ps[e - 1] - (b ? ps[b - 1] : 0ull);
    else if (op == 2) reinterpret_cast<uint32_t*>(out_vals)[r] = (uint32_t)rk[b];
    else reinterpret_cast<uint32_t*>(out_vals)[r] = (uint32_t)rk[e - 1];
  }
}

// Split sorted 64-bit records back into u32 keys and values (hash strategy output).
__global__ void k_split_out(const unsigned long long* __restrict__ rk, const unsigned long long* __restrict__ rv, uint64_t n,
                            int op, uint32_t* __restrict__ out_keys, void* __restrict__ out_vals, uint64_t cap) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n && i < cap; i += (uint64_t)gridDim.x * blockDim.x) {
    out_keys[i] = (uint32_t)rk[i];
    if (op == 1) reinterpret_cast<unsigned long long*>(out_vals)[i] = rv[i];
    else reinterpret_cast<uint32_t*>(out_vals)[i] = (uint32_t)rv[i];
  }
}

// Append the side slot (key 0xFFFFFFFF) after the sorted keys when present.
__global__ void k_side_append(const uint32_t* side_cnt, const void* side_val, int op, const unsigned long long* n_claimed,
                              unsigned long long* n_total, uint32_t* out_keys, void* out_vals, uint64_t cap) {
  if (threadIdx.x || blockIdx.x) return;
  uint64_t n = *n_claimed;
  if (*side_cnt) {
    if (n < cap) {
      out_keys[n] = kEmptyKey;
      if (op == 0) reinterpret_cast<uint32_t*>(out_vals)[n] = *side_cnt;
      else if (op == 1) reinterpret_cast<unsigned long long*>(out_vals)[n] = *reinterpret_cast<const unsigned long long*>(side_val);
      else reinterpret_cast<uint32_t*>(out_vals)[n] = dec_minmax(op, *reinterpret_cast<const uint32_t*>(side_val));
    }
    ++n;
  }
  *n_total = n;
}

// ----------------------------------------------------------------------------
// host launchers
// ----------------------------------------------------------------------------

static uint32_t blocks_for(uint64_t n, uint32_t per, uint32_t cap_blocks) {
  const uint64_t b = (n + per - 1) / per;
  return (uint32_t)(b == 0 ? 1 : (b < cap_blocks ? b : cap_blocks));
}

uint32_t int_lds_array_bytes(uint64_t R, uint32_t op) {
  const uint64_t b = 4ull * R + (op == 1 ? 8ull * R + 8 : (op >= 2 ? 4ull * R : 0));
  return (uint32_t)(b < 0xFFFFFFFFull ? b : 0xFFFFFFFFull);
}

hipError_t int_enqueue_lds_array(const IntLaunch& L, hipStream_t s) {
  const IntIn in{L.in, L.n, L.kv};
  const size_t lds = int_lds_array_bytes(L.R, L.op);
#define LDS_CASE(OP)                                                                                               \
  case OP:                                                                                                         \
    hipLaunchKernelGGL(k_lds_array<OP>, dim3(L.G), dim3(kIntThreads), lds, s, in, L.R, L.G, L.cnt_part, L.val_part, \
                       L.flags);                                                                                   \
    hipLaunchKernelGGL(k_lds_array_reduce<OP>, dim3(blocks_for(L.R, 256, 4096)), dim3(256), 0, s, L.R, L.G,        \
                       L.cnt_part, L.val_part, L.dcnt, L.dval);                                                    \
    break;
  switch (L.op) {
    LDS_CASE(0)
    LDS_CASE(1)
    LDS_CASE(2)
    LDS_CASE(3)
  }
#undef LDS_CASE
  return hipGetLastError();
}

hipError_t int_enqueue_global_array(const IntLaunch& L, hipStream_t s) {
  const IntIn in{L.in, L.n, L.kv};
  const uint32_t g = blocks_for(L.n, 256, 8192);
  switch (L.op) {
    case 0: hipLaunchKernelGGL(k_global_array<0>, dim3(g), dim3(256), 0, s, in, L.R, L.dcnt, L.dval, L.flags); break;
    case 1: hipLaunchKernelGGL(k_global_array<1>, dim3(g), dim3(256), 0, s, in, L.R, L.dcnt, L.dval, L.flags); break;
    case 2: hipLaunchKernelGGL(k_global_array<2>, dim3(g), dim3(256), 0, s, in, L.R, L.dcnt, L.dval, L.flags); break;
    case 3: hipLaunchKernelGGL(k_global_array<3>, dim3(g), dim3(256), 0, s, in, L.R, L.dcnt, L.dval, L.flags); break;
  }
  return hipGetLastError();
}

// Exclusive scan of a[0, n) in place by one workgroup, for n up to
// kScanOneMax: wave w takes a contiguous segment of whole 64-element steps.
// Each wave sums its segment (coalesced loads), the 16 wave totals are
// scanned in LDS, then each wave reads its segment again (from the cache)
// and scans it kScanOneBatch steps at a time with DPP lane shifts (the
// batch's scans are independent, so they overlap), adding a running carry.
// One launch instead of the block sums, their scan and the apply.
constexpr uint32_t kScanOneWaves = 16;
constexpr uint32_t kScanOneSteps = 64;  // 64-element steps per wave at most
constexpr uint32_t kScanOneBatch = 8;   // steps loaded and scanned together
constexpr uint64_t kScanOneMax = (uint64_t)kScanOneWaves * kWave * kScanOneSteps;

__global__ __launch_bounds__(kScanOneWaves * kWave) void k_scan_one(uint32_t* __restrict__ a, uint32_t n,
                                                                   unsigned long long* total) {
  __shared__ uint32_t ws[kScanOneWaves];
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  const uint32_t steps = (n + kScanOneWaves * kWave - 1) / (kScanOneWaves * kWave);  // <= kScanOneSteps
  const uint32_t b0 = wv * steps * kWave;
  auto at = [&](uint32_t q) { return b0 + q * kWave + lane; };
  uint32_t part = 0;
  for (uint32_t q0 = 0; q0 < steps; q0 += kScanOneBatch) {
    uint32_t v[kScanOneBatch];
#pragma unroll
    for (uint32_t u = 0; u < kScanOneBatch; ++u) v[u] = (q0 + u < steps && at(q0 + u) < n) ? a[at(q0 + u)] : 0u;
#pragma unroll
    for (uint32_t u = 0; u < kScanOneBatch; ++u) part += v[u];
  }
  const uint32_t wsum = wave_incl_scan(part);  // every lane takes part in the lane shifts
  if (lane == kWave - 1) ws[wv] = wsum;
  __syncthreads();
  uint32_t carry = 0, all = 0;
  for (uint32_t w = 0; w < kScanOneWaves; ++w) {
    if (w < wv) carry += ws[w];
    all += ws[w];
  }
  for (uint32_t q0 = 0; q0 < steps; q0 += kScanOneBatch) {
    uint32_t v[kScanOneBatch];
#pragma unroll
    for (uint32_t u = 0; u < kScanOneBatch; ++u) v[u] = (q0 + u < steps && at(q0 + u) < n) ? a[at(q0 + u)] : 0u;
#pragma unroll
    for (uint32_t u = 0; u < kScanOneBatch; ++u) v[u] = wave_incl_scan(v[u]);
#pragma unroll
    for (uint32_t u = 0; u < kScanOneBatch; ++u) {
      const uint32_t ex = from_prev_lane(v[u], 0u);  // exclusive within the step
      if (q0 + u < steps && at(q0 + u) < n) a[at(q0 + u)] = carry + ex;
      carry += (uint32_t)__builtin_amdgcn_readlane((int)v[u], kWave - 1);
    }
  }
  if (threadIdx.x == 0 && total) *total = all;
}

// Exclusive scan of a[0, n) in place; the sum of all entries into *total.
hipError_t scan_exclusive_u32(uint32_t* a, uint64_t n, uint32_t* sums, unsigned long long* total, hipStream_t s) {
  if (n <= kScanOneMax) {
    hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneWaves * kWave), 0, s, a, (uint32_t)n, total);
    return hipGetLastError();
  }
  const uint32_t sb = (uint32_t)((n + kScanTile - 1) / kScanTile);
  hipLaunchKernelGGL(k_scan_blocks, dim3(sb ? sb : 1), dim3(256), 0, s, a, n, sums);
  hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, sums, sb ? sb : 1, total);
  hipLaunchKernelGGL(k_scan_apply, dim3(sb ? sb : 1), dim3(256), 0, s, a, n, sums);
  return hipGetLastError();
}

uint64_t scan_sums_count(uint64_t n) { return (n + kScanTile - 1) / kScanTile + 1; }

// Layout of the partitioned fill's scratch for n elements over range R.
PartPlan part_plan(uint64_t n, uint64_t R) {
  PartPlan pp{};
  pp.P = (uint32_t)((R + kPartKeys - 1) / kPartKeys);
  pp.n_tiles = (uint32_t)((n + kPartTile - 1) / kPartTile);
  pp.runs = (uint64_t)(pp.P + 1) * pp.n_tiles;
  pp.part_elems = (uint64_t)pp.n_tiles * kPartTile;
  pp.usable = R > kPartKeys && pp.P <= kMaxParts && n >= (1ull << 20) && n < (1ull << 32);
  return pp;
}

// The tile-major fill: runs [n_tiles][P + 1], part [n_tiles * kPartTile].
hipError_t int_enqueue_global_array_tiles(const IntLaunch& L, const PartPlan& pp, uint32_t* runs, uint16_t* part,
                                          hipStream_t s) {
  const IntIn in{L.in, L.n, L.kv};
  hipLaunchKernelGGL(k_part_tile, dim3(pp.n_tiles), dim3(kPartThreads), part_tile_lds(pp.P), s, in, L.R, pp.P, runs, part,
                     L.flags);
  hipLaunchKernelGGL(k_part_fill_tiles, dim3(pp.P), dim3(1024), 0, s, part, runs, pp.P, pp.n_tiles, L.R, L.dcnt, L.blk);
  return hipGetLastError();
}

// Compaction of the dense arrays into the outputs; clears them when asked.
// blk_counted: the blocks' present keys are in L.blk already (partitioned fill).
hipError_t int_enqueue_dense_out(const IntLaunch& L, bool clear, bool blk_counted, hipStream_t s) {
  const uint32_t nb = (uint32_t)((L.R + kCompTile - 1) / kCompTile);
  if (!blk_counted) hipLaunchKernelGGL(k_dense_count, dim3(nb ? nb : 1), dim3(256), 0, s, L.dcnt, L.R, L.blk);
  if (nb <= kScanOneMax) hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneWaves * kWave), 0, s, L.blk, nb, L.n_out);
  else hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, L.blk, nb, L.n_out);
  switch (L.op) {
    case 0: hipLaunchKernelGGL(k_dense_write<0>, dim3(nb ? nb : 1), dim3(256), 0, s, L.dcnt, L.dval, L.R, L.blk, L.out_keys, L.out_vals, L.cap, clear); break;
    case 1: hipLaunchKernelGGL(k_dense_write<1>, dim3(nb ? nb : 1), dim3(256), 0, s, L.dcnt, L.dval, L.R, L.blk, L.out_keys, L.out_vals, L.cap, clear); break;
    case 2: hipLaunchKernelGGL(k_dense_write<2>, dim3(nb ? nb : 1), dim3(256), 0, s, L.dcnt, L.dval, L.R, L.blk, L.out_keys, L.out_vals, L.cap, clear); break;
    case 3: hipLaunchKernelGGL(k_dense_write<3>, dim3(nb ? nb : 1), dim3(256), 0, s, L.dcnt, L.dval, L.R, L.blk, L.out_keys, L.out_vals, L.cap, clear); break;
  }
  return hipGetLastError();
}

hipError_t int_enqueue_hash_map(const IntLaunch& L, hipStream_t s) {
  const IntIn in{L.in, L.n, L.kv};
  IntTable T{L.t_keys, L.t_cnt, L.t_val, L.t_cap, L.claimed, L.n_claimed, L.side_cnt, L.side_val, L.flags};
#define HASH_CASE(OP) \
  case OP: hipLaunchKernelGGL((k_int_hash<OP, 12>), dim3(L.G), dim3(kIntThreads), 0, s, in, T, L.G, L.debug_hash, L.R); break;
  switch (L.op) {
    HASH_CASE(0)
    HASH_CASE(1)
    HASH_CASE(2)
    HASH_CASE(3)
  }
#undef HASH_CASE
  return hipGetLastError();
}

// Radix sort of n records (64-bit keys and values) over the given key bits.
hipError_t radix_sort64(unsigned long long* k0, unsigned long long* v0, unsigned long long* k1, unsigned long long* v1,
                        uint64_t n, int bits, uint32_t* hist, uint32_t* scan_sums, bool* result_in_1, hipStream_t s) {
  const uint32_t n_tiles = (uint32_t)((n + kSortTile - 1) / kSortTile);
  const uint64_t hn = 256ull * n_tiles;
  const uint32_t sb = (uint32_t)((hn + kScanTile - 1) / kScanTile);
  bool in1 = false;
  for (int sh = 0; sh < bits; sh += 8) {
    unsigned long long *ki = in1 ? k1 : k0, *vi = in1 ? v1 : v0, *ko = in1 ? k0 : k1, *vo = in1 ? v0 : v1;
    if (n) {
      hipLaunchKernelGGL(k_radix_hist, dim3(n_tiles), dim3(256), 0, s, ki, n, sh, n_tiles, hist);
      if (hn <= kScanOneMax) {
        hipLaunchKernelGGL(k_scan_one, dim3(1), dim3(kScanOneWaves * kWave), 0, s, hist, (uint32_t)hn,
                           (unsigned long long*)nullptr);
      } else {
        hipLaunchKernelGGL(k_scan_blocks, dim3(sb), dim3(256), 0, s, hist, hn, scan_sums);
        hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, scan_sums, sb, (unsigned long long*)nullptr);
        hipLaunchKernelGGL(k_scan_apply, dim3(sb), dim3(256), 0, s, hist, hn, scan_sums);
      }
      hipLaunchKernelGGL(k_radix_scatter, dim3(n_tiles), dim3(256), 0, s, ki, vi, n, sh, n_tiles, hist, ko, vo);
    }
    in1 = !in1;
  }
  *result_in_1 = in1;
  return hipGetLastError();
}

hipError_t int_enqueue_hash_out(const IntLaunch& L, uint64_t n_claimed_host, hipStream_t s) {
  IntTable T{L.t_keys, L.t_cnt, L.t_val, L.t_cap, L.claimed, L.n_claimed, L.side_cnt, L.side_val, L.flags};
  const uint64_t n = n_claimed_host;
  const uint32_t g = blocks_for(n, 256, 4096);
  switch (L.op) {
    case 0: hipLaunchKernelGGL(k_int_gather<0>, dim3(g), dim3(256), 0, s, T, L.rk32, L.rv0); break;
    case 1: hipLaunchKernelGGL(k_int_gather<1>, dim3(g), dim3(256), 0, s, T, L.rk32, L.rv0); break;
    case 2: hipLaunchKernelGGL(k_int_gather<2>, dim3(g), dim3(256), 0, s, T, L.rk32, L.rv0); break;
    case 3: hipLaunchKernelGGL(k_int_gather<3>, dim3(g), dim3(256), 0, s, T, L.rk32, L.rv0); break;
  }
  return hipGetLastError();
}

__global__ void k_widen_keys(const uint32_t* __restrict__ a, unsigned long long* __restrict__ b, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) b[i] = a[i];
}

hipError_t int_enqueue_hash_sort_out(const IntLaunch& L, uint64_t n, hipStream_t s) {
  const uint32_t g = blocks_for(n, 256, 4096);
  hipLaunchKernelGGL(k_widen_keys, dim3(g), dim3(256), 0, s, L.rk32, L.rk0, n);
  bool in1 = false;
  hipError_t e = radix_sort64(L.rk0, L.rv0, L.rk1, L.rv1, n, 32, L.hist, L.scan_sums, &in1, s);
  if (e != hipSuccess) return e;
  const unsigned long long* rk = in1 ? L.rk1 : L.rk0;
  const unsigned long long* rv = in1 ? L.rv1 : L.rv0;
  hipLaunchKernelGGL(k_split_out, dim3(g), dim3(256), 0, s, rk, rv, n, L.op, L.out_keys, L.out_vals, L.cap);
  hipLaunchKernelGGL(k_side_append, dim3(1), dim3(64), 0, s, L.side_cnt, L.side_val, L.op, L.n_claimed, L.n_out,
                     L.out_keys, L.out_vals, L.cap);
  return hipGetLastError();
}

hipError_t int_enqueue_sort(const IntLaunch& L, hipStream_t s) {
  const IntIn in{L.in, L.n, L.kv};
  const uint64_t n = L.n;
  const uint32_t g = blocks_for(n, 256, 8192);
  hipLaunchKernelGGL(k_sort_records, dim3(g), dim3(256), 0, s, in, (int)L.op, L.R, L.flags, L.rk0, L.rv0);
  bool in1 = false;
  hipError_t e = radix_sort64(L.rk0, L.rv0, L.rk1, L.rv1, n, L.op >= 2 ? 64 : 32, L.hist, L.scan_sums, &in1, s);
  if (e != hipSuccess) return e;
  unsigned long long* rk = in1 ? L.rk1 : L.rk0;
  unsigned long long* rv = in1 ? L.rv1 : L.rv0;
  // heads and their exclusive scan (run index of each head)
  hipLaunchKernelGGL(k_run_heads, dim3(g), dim3(256), 0, s, rk, n, (int)L.op, L.head);
  if (n) {
    const hipError_t e2 = hipMemcpyAsync(L.pos, L.head, 4 * n, hipMemcpyDeviceToDevice, s);
    if (e2 != hipSuccess) return e2;
  }
  const uint32_t sb = (uint32_t)((n + kScanTile - 1) / kScanTile);
  if (n) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(sb), dim3(256), 0, s, L.pos, n, L.scan_sums);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, s, L.scan_sums, sb, L.n_out);
    hipLaunchKernelGGL(k_scan_apply, dim3(sb), dim3(256), 0, s, L.pos, n, L.scan_sums);
  }
  if (L.op == 1 && n) {
    const uint32_t pb = (uint32_t)((n + kPsTile - 1) / kPsTile);
    hipLaunchKernelGGL(k_ps64_blocks, dim3(pb), dim3(256), 0, s, rv, n, L.ps_sums);
    hipLaunchKernelGGL(k_ps64_scan_sums, dim3(1), dim3(64), 0, s, L.ps_sums, pb);
    hipLaunchKernelGGL(k_ps64_apply, dim3(pb), dim3(256), 0, s, rv, n, L.ps_sums);
  }
  hipLaunchKernelGGL(k_run_starts, dim3(g), dim3(256), 0, s, L.head, L.pos, n, L.n_out, L.hpos);
  hipLaunchKernelGGL(k_run_write, dim3(g), dim3(256), 0, s, rk, rv, L.hpos, L.n_out, (int)L.op, L.out_keys, L.out_vals,
                     L.cap);
  return hipGetLastError();
}

}  // namespace mr
