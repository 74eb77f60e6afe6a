// Bloom filter build on gfx950 (benchmark application "Bloom Filter": large
// array container, Section III-E "eliminating local arrays").
//
// map: every k-mer (k consecutive bases of A, C, G, T; a k-mer holding any
// other byte is skipped) emits the h bit positions of the filter; reduce: OR
// into one array of m bits.
//   code  v = 2-bit packed k-mer (A 0, C 1, G 2, T 3, first base highest)
//   x     = fmix64(v) (the 64-bit finaliser of MurmurHash3)
//   g_i   = (lo32(x) + i * (hi32(x) | 1)) mod 2^32   (double hashing, i < h)
//   pos_i = floor(g_i * m / 2^32)                     (multiply-shift into [0, m))
//
// Device atomics on a 37.5 MB array would be the bottleneck, so the array is
// filled by position ranges of 2^19 bits. A tile of 16384 k-mers counts its
// positions per range; an exclusive scan over (range, tile) gives each tile
// its segment of each range; the tile then writes its positions into those
// segments, 2048 k-mers at a time, each batch ordered by range in LDS first so
// that consecutive lanes write consecutive words; finally one workgroup per
// range ORs its segment into a 64 KB LDS bit array and writes the range's
// words once.
#include "common.h"
#include "launch.h"

namespace mr {

constexpr uint32_t kBloomRangeBits = 19;                   // positions per range: 2^19 bits = 64 KB of LDS words
constexpr uint32_t kBloomRangeMask = (1u << kBloomRangeBits) - 1;
constexpr uint32_t kBloomRangeWords = (1u << kBloomRangeBits) / 32;
constexpr uint32_t kBloomMaxRanges = 1024;                 // m up to 2^29 bits
constexpr uint32_t kBloomSub = 2048;                       // k-mers per batch of the scatter pass
constexpr uint32_t kBloomTile = 16384;                     // k-mers per tile of the count and scatter passes
constexpr uint32_t kBloomThreads = 512;
constexpr uint32_t kBloomScatterPer = kBloomSub / kBloomThreads;  // consecutive k-mers per thread in a batch
constexpr uint32_t kBloomCountPer = 8;                            // the same in the count pass
constexpr uint32_t kBloomCountSub = kBloomCountPer * kBloomThreads;
constexpr uint32_t kBloomMaxK = 32;
constexpr uint32_t kBloomMaxH = 8;                         // hashes per k-mer
constexpr uint32_t kBloomRangesPer = kBloomMaxRanges / kBloomThreads;  // ranges owned by one thread in scans
constexpr uint32_t kBloomFillThreads = 1024;
constexpr uint32_t kBloomPartPad = 8;                      // words readable past the last position

// Stages the codes of bytes [e0, e0 + span) into LDS: A 0, C 1, G 2, T 3,
// anything else (and bytes past the input) 4.
MR_DEV void bloom_stage(const uint8_t* __restrict__ in, uint64_t n_bytes, uint64_t e0, uint32_t span, uint8_t* st) {
  for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) {
    const uint64_t p = e0 + i;
    const uint32_t b = p < n_bytes ? in[p] : 0u;
    st[i] = (uint8_t)(b == 'A' ? 0u : b == 'C' ? 1u : b == 'G' ? 2u : b == 'T' ? 3u : 4u);
  }
}

// Hash halves of this thread's PER consecutive k-mers of the staged batch
// (k-mer index e0 + j): a = low32(fmix64(v)), b = high32(fmix64(v)) | 1.
// Bit j of the result is set when k-mer j exists and holds only A, C, G, T.
template <uint32_t PER>
MR_DEV uint32_t bloom_thread_hashes(const uint8_t* st, uint64_t e0, uint64_t n_kmers, uint32_t k, uint32_t (&a)[PER],
                                    uint32_t (&b)[PER]) {
  const uint32_t j0 = threadIdx.x * PER;  // a multiple of 4
  const uint64_t mask = k == 32 ? ~0ull : ((1ull << (2 * k)) - 1);
  uint64_t v = 0;
  uint32_t run = 0, valid = 0;  // run: valid bases ending at the current byte
  auto push = [&](uint32_t c) {
    run = c < 4 ? run + 1 : 0;
    v = (v << 2) | (c & 3u);
  };
  // the first k - 1 bases of k-mer j0, four codes per LDS read
  uint32_t q = 0;
  for (; q + 4 <= k - 1; q += 4) {
    const uint32_t w = *reinterpret_cast<const uint32_t*>(st + j0 + q);
    push(w & 0xff);
    push((w >> 8) & 0xff);
    push((w >> 16) & 0xff);
    push(w >> 24);
  }
  for (; q + 1 < k; ++q) push(st[j0 + q]);
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    push(st[j0 + j + k - 1]);
    v &= mask;
    const uint64_t x = fmix64(v);
    a[j] = (uint32_t)x;
    b[j] = (uint32_t)(x >> 32) | 1u;
    if (run >= k && e0 + j0 + j < n_kmers) valid |= 1u << j;
  }
  return valid;
}

// Calls f(pos) for the h positions floor((a + i b mod 2^32) m / 2^32) of each valid k-mer.
template <uint32_t PER, typename F>
MR_DEV void bloom_for_positions(const uint32_t (&a)[PER], const uint32_t (&b)[PER], uint32_t valid, uint32_t h,
                                uint64_t m, F&& f) {
#pragma unroll
  for (uint32_t j = 0; j < PER; ++j) {
    if (!(valid >> j & 1u)) continue;
    for (uint32_t i = 0; i < h; ++i) {
      const uint32_t g = a[j] + i * b[j];
      f((uint32_t)(((uint64_t)g * m) >> 32));
    }
  }
}

__global__ __launch_bounds__(kBloomThreads) void k_bloom_count(const uint8_t* __restrict__ in, uint64_t n_bytes,
                                                               uint64_t n_kmers, uint32_t k, uint32_t h, uint64_t m,
                                                               uint32_t P, uint32_t n_tiles, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[kBloomMaxRanges];
  __shared__ __align__(16) uint8_t st[kBloomCountSub + kBloomMaxK];
  for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) cnt[p] = 0;
  for (uint32_t e = 0; e < kBloomTile; e += kBloomCountSub) {
    const uint64_t e0 = (uint64_t)blockIdx.x * kBloomTile + e;
    if (e0 >= n_kmers) break;
    __syncthreads();  // the previous batch is no longer read
    bloom_stage(in, n_bytes, e0, kBloomCountSub + k - 1, st);
    __syncthreads();
    uint32_t a[kBloomCountPer], b[kBloomCountPer];
    const uint32_t valid = bloom_thread_hashes<kBloomCountPer>(st, e0, n_kmers, k, a, b);
    bloom_for_positions<kBloomCountPer>(a, b, valid, h, m,
                                        [&](uint32_t pos) { atomicAdd(&cnt[pos >> kBloomRangeBits], 1u); });
  }
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) hist[(uint64_t)p * n_tiles + blockIdx.x] = cnt[p];
}

// offs: exclusive scan of the counts, range-major (index p * n_tiles + t).
// The written words are the positions themselves: the range in bits 19 and
// up, the position within the range in bits 0..18.
__global__ __launch_bounds__(kBloomThreads) void k_bloom_scatter(const uint8_t* __restrict__ in, uint64_t n_bytes,
                                                                 uint64_t n_kmers, uint32_t k, uint32_t h, uint64_t m,
                                                                 uint32_t P, uint32_t n_tiles,
                                                                 const uint32_t* __restrict__ offs,
                                                                 uint32_t* __restrict__ part) {
  __shared__ uint32_t cnt[kBloomMaxRanges];        // batch counts, then each range's first slot
  __shared__ uint32_t delta[kBloomMaxRanges];      // output word of slot j of range p: delta[p] + j
  __shared__ uint32_t sk[kBloomSub * kBloomMaxH];  // the batch's positions, ordered by range
  __shared__ __align__(16) uint8_t st[kBloomSub + kBloomMaxK];
  __shared__ uint32_t wsum[kBloomThreads / kWave];
  const uint32_t t = blockIdx.x;
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  // next free word of each owned range's segment, and the owned ranges' counts in the previous batch
  uint32_t gb[kBloomRangesPer], prev[kBloomRangesPer];
#pragma unroll
  for (uint32_t q = 0; q < kBloomRangesPer; ++q) {
    const uint32_t p = threadIdx.x * kBloomRangesPer + q;
    prev[q] = 0;
    gb[q] = p < P ? offs[(uint64_t)p * n_tiles + t] : 0u;
  }
  for (uint32_t e = 0; e < kBloomTile; e += kBloomSub) {
    const uint64_t e0 = (uint64_t)t * kBloomTile + e;
    if (e0 >= n_kmers) break;
    __syncthreads();  // the previous batch's slots have been written out
    for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) cnt[p] = 0;
    bloom_stage(in, n_bytes, e0, kBloomSub + k - 1, st);
    __syncthreads();
    uint32_t a[kBloomScatterPer], b[kBloomScatterPer];
    const uint32_t valid = bloom_thread_hashes<kBloomScatterPer>(st, e0, n_kmers, k, a, b);
    // each position's rank among the batch's positions of its range
    uint32_t rank[kBloomScatterPer][kBloomMaxH];
#pragma unroll
    for (uint32_t j = 0; j < kBloomScatterPer; ++j) {
#pragma unroll
      for (uint32_t i = 0; i < kBloomMaxH; ++i) {
        if ((valid >> j & 1u) && i < h) {
          const uint32_t pos = (uint32_t)(((uint64_t)(a[j] + i * b[j]) * m) >> 32);
          rank[j][i] = atomicAdd(&cnt[pos >> kBloomRangeBits], 1u);
        }
      }
    }
    __syncthreads();
    // exclusive scan of the batch counts over the ranges
    uint32_t c[kBloomRangesPer], sum = 0;
#pragma unroll
    for (uint32_t q = 0; q < kBloomRangesPer; ++q) {
      const uint32_t p = threadIdx.x * kBloomRangesPer + q;
      c[q] = p < P ? cnt[p] : 0u;
      sum += c[q];
    }
    uint32_t incl = sum;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
      if (lane >= (uint32_t)o) incl += y;
    }
    if (lane == kWave - 1) wsum[wv] = incl;
    __syncthreads();
    uint32_t run = incl - sum, btot = 0;
    for (uint32_t w = 0; w < kBloomThreads / kWave; ++w) {
      if (w < wv) run += wsum[w];
      btot += wsum[w];
    }
#pragma unroll
    for (uint32_t q = 0; q < kBloomRangesPer; ++q) {
      const uint32_t p = threadIdx.x * kBloomRangesPer + q;
      gb[q] += prev[q];
      prev[q] = c[q];
      if (p < P) {
        cnt[p] = run;  // the batch's first slot of range p
        delta[p] = gb[q] - run;
      }
      run += c[q];
    }
    __syncthreads();
#pragma unroll
    for (uint32_t j = 0; j < kBloomScatterPer; ++j) {
#pragma unroll
      for (uint32_t i = 0; i < kBloomMaxH; ++i) {
        if ((valid >> j & 1u) && i < h) {
          const uint32_t pos = (uint32_t)(((uint64_t)(a[j] + i * b[j]) * m) >> 32);
          sk[cnt[pos >> kBloomRangeBits] + rank[j][i]] = pos;
        }
      }
    }
    __syncthreads();
    for (uint32_t j = threadIdx.x; j < btot; j += blockDim.x) {
      const uint32_t v = sk[j];
      part[delta[v >> kBloomRangeBits] + j] = v;
    }
  }
}

// part holds kBloomPartPad readable words past the last position.
__global__ __launch_bounds__(kBloomFillThreads) void k_bloom_fill(const uint32_t* __restrict__ part,
                                                                  const uint32_t* __restrict__ offs,
                                                                  const unsigned long long* __restrict__ total,
                                                                  uint32_t P, uint32_t n_tiles, uint64_t n_words,
                                                                  uint32_t* __restrict__ words) {
  __shared__ uint32_t bits[kBloomRangeWords];
  const uint32_t p = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kBloomRangeWords; i += blockDim.x) bits[i] = 0;
  __syncthreads();
  const uint64_t start = offs[(uint64_t)p * n_tiles];
  const uint64_t end = p + 1 < P ? offs[(uint64_t)(p + 1) * n_tiles] : *total;
  if (start < end) {
    // 16-byte loads from the aligned word below start, four per thread in
    // flight while the previous four are applied; addresses past the segment
    // are clamped to its last aligned word and their words skipped
    const uint64_t a0 = start & ~3ull, last = (end - 1) & ~3ull, stride = 4ull * blockDim.x;
    auto load4 = [&](uint64_t j, uint4 (&x)[4]) {
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        const uint64_t at = j + u * stride;
        x[u] = *reinterpret_cast<const uint4*>(part + (at < last ? at : last));
      }
    };
    auto put = [&](uint32_t v, uint64_t j) {
      if (j >= start && j < end) atomicOr(&bits[(v & kBloomRangeMask) >> 5], 1u << (v & 31));
    };
    uint64_t j = a0 + 4ull * threadIdx.x;
    uint4 cur[4], nxt[4];
    load4(j, cur);
    for (; j < end; j += 4 * stride) {
      load4(j + 4 * stride, nxt);
#pragma unroll
      for (uint32_t u = 0; u < 4; ++u) {
        const uint64_t at = j + u * stride;
        put(cur[u].x, at);
        put(cur[u].y, at + 1);
        put(cur[u].z, at + 2);
        put(cur[u].w, at + 3);
        cur[u] = nxt[u];
      }
    }
  }
  __syncthreads();
  const uint64_t w0 = (uint64_t)p * kBloomRangeWords;
  for (uint32_t i = threadIdx.x; i < kBloomRangeWords && w0 + i < n_words; i += blockDim.x) words[w0 + i] = bits[i];
}

__global__ void k_bloom_zero_words(uint32_t* __restrict__ words, uint64_t n) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) words[i] = 0u;
}

BloomPlan bloom_plan(uint64_t n_bytes, uint32_t k, uint32_t h, uint64_t m) {
  BloomPlan b{};
  b.n_kmers = n_bytes >= k ? n_bytes - k + 1 : 0;
  b.n_words = (m + 31) / 32;
  b.P = (uint32_t)((m + (1ull << kBloomRangeBits) - 1) >> kBloomRangeBits);
  b.n_tiles = (uint32_t)((b.n_kmers + kBloomTile - 1) / kBloomTile);
  b.H = (uint64_t)b.P * b.n_tiles;
  b.max_entries = b.n_kmers * h;
  b.part_words = b.max_entries + kBloomPartPad;
  b.ok = k >= 1 && k <= kBloomMaxK && h >= 1 && h <= kBloomMaxH && m >= 1 && b.P <= kBloomMaxRanges && b.max_entries < (1ull << 32);
  return b;
}

hipError_t bloom_enqueue(const uint8_t* in, uint64_t n_bytes, uint32_t k, uint32_t h, uint64_t m, const BloomPlan& b,
                         uint32_t* hist, uint32_t* scan_sums, unsigned long long* total, uint32_t* part, uint32_t* words,
                         hipStream_t s) {
  if (b.n_tiles) {
    hipLaunchKernelGGL(k_bloom_count, dim3(b.n_tiles), dim3(kBloomThreads), 0, s, in, n_bytes, b.n_kmers, k, h, m, b.P,
                       b.n_tiles, hist);
    hipError_t e = scan_exclusive_u32(hist, b.H, scan_sums, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_bloom_scatter, dim3(b.n_tiles), dim3(kBloomThreads), 0, s, in, n_bytes, b.n_kmers, k, h, m, b.P,
                       b.n_tiles, hist, part);
    hipLaunchKernelGGL(k_bloom_fill, dim3(b.P), dim3(kBloomFillThreads), 0, s, part, hist, total, b.P, b.n_tiles, b.n_words, words);
  } else {
    hipLaunchKernelGGL(k_bloom_zero_words, dim3(256), dim3(256), 0, s, words, b.n_words);
  }
  return hipGetLastError();
}

}  // namespace mr
