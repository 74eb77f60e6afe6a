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
// filled by position ranges of 2^18 bits: count each tile's positions per
// range, scan, scatter each position's low 18 bits into its range's segment
// (tile ordered by range in LDS first), then one workgroup per range ORs its
// segment into a 32 KB LDS bit array and writes the range's words once.
#include "common.h"
#include "launch.h"

namespace mr {

constexpr uint32_t kBloomRangeBits = 18;                   // positions per range: 2^18 bits = 32 KB of LDS words
constexpr uint32_t kBloomRangeWords = (1u << kBloomRangeBits) / 32;
constexpr uint32_t kBloomMaxRanges = 2048;                 // m up to 2^29 bits
constexpr uint32_t kBloomTile = 2048;                      // k-mers per tile of the count and scatter passes
constexpr uint32_t kBloomThreads = 256;
constexpr uint32_t kBloomPer = kBloomTile / kBloomThreads;  // consecutive k-mers per thread
constexpr uint32_t kBloomMaxK = 32;
constexpr uint32_t kBloomMaxH = 8;                         // hashes per k-mer

MR_DEV uint32_t base_code(uint32_t b) {
  // A 0, C 1, G 2, T 3; anything else 4
  return b == 'A' ? 0u : b == 'C' ? 1u : b == 'G' ? 2u : b == 'T' ? 3u : 4u;
}

// The tile's bytes [e0, e0 + kBloomTile + k - 1) into LDS (bytes past the
// input read as 'N').
MR_DEV void bloom_stage(const uint8_t* __restrict__ in, uint64_t n_bytes, uint64_t e0, uint32_t k, uint8_t* st) {
  const uint32_t span = kBloomTile + k - 1;
  for (uint32_t i = threadIdx.x; i < span; i += blockDim.x) {
    const uint64_t p = e0 + i;
    st[i] = p < n_bytes ? in[p] : (uint8_t)'N';
  }
}

// Calls f(pos) for every position of every valid k-mer among this thread's
// kBloomPer consecutive k-mers of the staged tile (k-mer index e0 + j).
template <typename F>
MR_DEV void bloom_thread_positions(const uint8_t* st, uint64_t e0, uint64_t n_kmers, uint32_t k, uint32_t h, uint64_t m,
                                   F&& f) {
  const uint32_t j0 = threadIdx.x * kBloomPer;
  if (e0 + j0 >= n_kmers) return;
  const uint64_t mask = k == 32 ? ~0ull : ((1ull << (2 * k)) - 1);
  uint64_t v = 0;
  uint32_t run = 0;  // valid bases ending at the current byte
  // the first k - 1 bases of k-mer j0
  for (uint32_t q = 0; q + 1 < k; ++q) {
    const uint32_t c = base_code(st[j0 + q]);
    run = c < 4 ? run + 1 : 0;
    v = ((v << 2) | (c & 3u)) & mask;
  }
  for (uint32_t j = j0; j < j0 + kBloomPer && e0 + j < n_kmers; ++j) {
    const uint32_t c = base_code(st[j + k - 1]);
    run = c < 4 ? run + 1 : 0;
    v = ((v << 2) | (c & 3u)) & mask;
    if (run < k) continue;
    const uint64_t x = fmix64(v);
    const uint32_t a = (uint32_t)x, b = (uint32_t)(x >> 32) | 1u;
    for (uint32_t i = 0; i < h; ++i) {
      const uint32_t g = a + i * b;
      f((uint32_t)(((uint64_t)g * m) >> 32));
    }
  }
}

__global__ __launch_bounds__(kBloomThreads) void k_bloom_count(const uint8_t* __restrict__ in, uint64_t n_bytes,
                                                               uint64_t n_kmers, uint32_t k, uint32_t h, uint64_t m,
                                                               uint32_t P, uint32_t n_tiles, uint32_t* __restrict__ hist) {
  __shared__ uint32_t cnt[kBloomMaxRanges];
  __shared__ uint8_t st[kBloomTile + kBloomMaxK];
  const uint64_t e0 = (uint64_t)blockIdx.x * kBloomTile;
  for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) cnt[p] = 0;
  bloom_stage(in, n_bytes, e0, k, st);
  __syncthreads();
  bloom_thread_positions(st, e0, n_kmers, k, h, m, [&](uint32_t pos) { atomicAdd(&cnt[pos >> kBloomRangeBits], 1u); });
  __syncthreads();
  for (uint32_t p = threadIdx.x; p < P; p += blockDim.x) hist[(uint64_t)p * n_tiles + blockIdx.x] = cnt[p];
}

__global__ __launch_bounds__(kBloomThreads) void k_bloom_scatter(const uint8_t* __restrict__ in, uint64_t n_bytes,
                                                                 uint64_t n_kmers, uint32_t k, uint32_t h, uint64_t m,
                                                                 uint32_t P, uint32_t n_tiles,
                                                                 const uint32_t* __restrict__ offs,
                                                                 const unsigned long long* __restrict__ total,
                                                                 uint32_t* __restrict__ part) {
  __shared__ uint32_t lbase[kBloomMaxRanges + 1];
  __shared__ uint32_t lpos[kBloomMaxRanges];
  __shared__ uint32_t sk[kBloomTile * kBloomMaxH];  // staged low bits of the positions, ordered by range
  __shared__ uint8_t st[kBloomTile + kBloomMaxK];
  __shared__ uint32_t wsum[kBloomThreads / kWave];
  const uint32_t t = blockIdx.x;
  const uint64_t e0 = (uint64_t)t * kBloomTile;
  bloom_stage(in, n_bytes, e0, k, st);
  // this tile's count of range p, from the scanned counts (range-major, tile-minor)
  auto tile_count = [&](uint32_t p) -> uint32_t {
    const uint64_t at = (uint64_t)p * n_tiles + t;
    const uint64_t next = at + 1 < (uint64_t)P * n_tiles ? (uint64_t)offs[at + 1] : *total;
    return (uint32_t)(next - offs[at]);
  };
  constexpr uint32_t kPer = kBloomMaxRanges / kBloomThreads;
  uint32_t c[kPer], sum = 0;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t p = threadIdx.x * kPer + q;
    c[q] = p < P ? tile_count(p) : 0u;
    sum += c[q];
  }
  const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
  uint32_t incl = sum;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
    if (lane >= (uint32_t)o) incl += y;
  }
  if (lane == kWave - 1) wsum[wv] = incl;
  __syncthreads();
  uint32_t pre = 0, mtot = 0;
  for (uint32_t w = 0; w < kBloomThreads / kWave; ++w) {
    if (w < wv) pre += wsum[w];
    mtot += wsum[w];
  }
  uint32_t run = pre + incl - sum;
#pragma unroll
  for (uint32_t q = 0; q < kPer; ++q) {
    const uint32_t p = threadIdx.x * kPer + q;
    if (p < P) {
      lbase[p] = run;
      lpos[p] = run;
    }
    run += c[q];
  }
  if (threadIdx.x == 0) lbase[P] = mtot;
  __syncthreads();
  bloom_thread_positions(st, e0, n_kmers, k, h, m, [&](uint32_t pos) {
    sk[atomicAdd(&lpos[pos >> kBloomRangeBits], 1u)] = pos & ((1u << kBloomRangeBits) - 1);
  });
  __syncthreads();
  for (uint32_t p = wv; p < P; p += kBloomThreads / kWave) {
    const uint32_t b0 = lbase[p], b1 = lbase[p + 1];
    uint32_t* dst = part + offs[(uint64_t)p * n_tiles + t];
    for (uint32_t j = b0 + lane; j < b1; j += kWave) dst[j - b0] = sk[j];
  }
}

__global__ __launch_bounds__(1024) void k_bloom_fill(const uint32_t* __restrict__ part, const uint32_t* __restrict__ offs,
                                                     const unsigned long long* __restrict__ total, uint32_t P,
                                                     uint32_t n_tiles, uint64_t n_words, uint32_t* __restrict__ words) {
  __shared__ uint32_t bits[kBloomRangeWords];
  const uint32_t p = blockIdx.x;
  for (uint32_t i = threadIdx.x; i < kBloomRangeWords; i += blockDim.x) bits[i] = 0;
  __syncthreads();
  const uint64_t start = offs[(uint64_t)p * n_tiles];
  const uint64_t end = p + 1 < P ? offs[(uint64_t)(p + 1) * n_tiles] : *total;
  for (uint64_t j = start + threadIdx.x; j < end; j += blockDim.x) {
    const uint32_t lo = part[j];
    atomicOr(&bits[lo >> 5], 1u << (lo & 31));
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
                       b.n_tiles, hist, total, part);
    hipLaunchKernelGGL(k_bloom_fill, dim3(b.P), dim3(1024), 0, s, part, hist, total, b.P, b.n_tiles, b.n_words, words);
  } else {
    hipLaunchKernelGGL(k_bloom_zero_words, dim3(256), dim3(256), 0, s, words, b.n_words);
  }
  return hipGetLastError();
}

}  // namespace mr
