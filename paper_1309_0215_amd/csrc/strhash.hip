// Word hashing, one character per lane per step (arXiv 1309.0215, Section
// III-C): FNV-1a 64 of every word, in input order, computed by one wavefront
// per block of consecutive words.
//   * SIMDH-Padding: rounds of `units` consecutive words, one per lane; a
//     round lasts as long as its longest word plus the terminator step, and
//     lanes with shorter words idle (masked) until it ends.
//   * SIMDH-Stream: every lane takes the next word as soon as its own ends.
//     The paper finds the lanes to refill from a mask of the lanes that met
//     a terminator and a prefix sum over it; here the mask is a wave ballot
//     and the prefix sum is mbcnt (the number of set mask bits below the
//     lane), so lanes freed together take the next words in lane order.
// A word's terminator takes a step of its own in both schemes, as in the
// paper's worked example. The per-word schedule (lane, first and last step)
// can be written out for checking.
#include "common.h"
#include "launch.h"

namespace mr {

constexpr uint64_t kFnvBasis = 0xCBF29CE484222325ULL, kFnvPrime = 0x100000001B3ULL;
constexpr uint32_t kHwChunk = 16;  // bytes per thread in the word-list passes

MR_DEV bool hw_word_start(const uint8_t* in, uint64_t i) {
  return !is_sep_byte(in[i]) && (i == 0 || is_sep_byte(in[i - 1]));
}

// Word starts per 16-byte chunk of the input.
__global__ void k_hw_count(const uint8_t* __restrict__ in, uint64_t n, uint32_t* __restrict__ counts, uint64_t n_chunks) {
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < n_chunks; c += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = (c + 1) * kHwChunk < n ? (c + 1) * kHwChunk : n;
    uint32_t k = 0;
    for (uint64_t i = c * kHwChunk; i < e; ++i) k += hw_word_start(in, i) ? 1u : 0u;
    counts[c] = k;
  }
}

// Offset and length of every word, placed by the scanned counts.
__global__ void k_hw_list(const uint8_t* __restrict__ in, uint64_t n, const uint32_t* __restrict__ first, uint64_t n_chunks,
                          uint32_t* __restrict__ off, uint32_t* __restrict__ len) {
  for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < n_chunks; c += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t e = (c + 1) * kHwChunk < n ? (c + 1) * kHwChunk : n;
    uint32_t w = first[c];
    for (uint64_t i = c * kHwChunk; i < e; ++i) {
      if (!hw_word_start(in, i)) continue;
      uint64_t j = i + 1;
      while (j < n && !is_sep_byte(in[j])) ++j;
      off[w] = (uint32_t)i;
      len[w] = (uint32_t)(j - i);
      ++w;
    }
  }
}

// One wavefront per block of `block` consecutive words; lanes below `units`
// hash. sched (optional): [word][3] = lane, first step, last step (steps
// counted from 1 within the block).
template <bool kStream>
__global__ __launch_bounds__(64) void k_hw_hash(const uint8_t* __restrict__ in, const uint32_t* __restrict__ off,
                                               const uint32_t* __restrict__ len, uint64_t n_words, uint32_t units,
                                               uint64_t block, unsigned long long* __restrict__ hashes,
                                               uint32_t* __restrict__ sched) {
  const uint32_t lane = threadIdx.x;
  const bool unit = lane < units;
  const uint64_t w0 = (uint64_t)blockIdx.x * block;
  if (w0 >= n_words) return;
  const uint64_t w1 = w0 + block < n_words ? w0 + block : n_words;
  if constexpr (kStream) {
    int64_t cur = -1;
    uint32_t pos = 0, wl = 0, o = 0, first = 0;
    uint64_t h = 0;
    uint64_t next = w0;  // uniform
    for (uint32_t step = 1;; ++step) {
      // lanes without a word take the next ones, in lane order
      const uint64_t free_m = __ballot(unit && cur < 0);
      const uint64_t idx = next + mbcnt(free_m);
      if (unit && cur < 0 && idx < w1) {
        cur = (int64_t)idx;
        pos = 0;
        wl = len[idx];
        o = off[idx];
        h = kFnvBasis;
        first = step;
      }
      const uint64_t took = popc64(free_m);
      next = next + took < w1 ? next + took : w1;
      if (__ballot(cur >= 0) == 0) break;
      if (cur >= 0) {
        if (pos == wl) {  // the terminator step
          hashes[cur] = h;
          if (sched) {
            sched[3 * cur] = lane;
            sched[3 * cur + 1] = first;
            sched[3 * cur + 2] = step;
          }
          cur = -1;
        } else {
          h = (h ^ in[(uint64_t)o + pos]) * kFnvPrime;
          ++pos;
        }
      }
    }
  } else {
    uint32_t start = 1;
    for (uint64_t r0 = w0; r0 < w1; r0 += units) {
      const uint64_t idx = r0 + lane;
      const bool has = unit && idx < w1;
      const uint32_t wl = has ? len[idx] : 0u, o = has ? off[idx] : 0u;
      // the round lasts for the longest word of the round plus its terminator
      uint32_t lmax = wl;
      for (int sh = 32; sh > 0; sh >>= 1) {
        const uint32_t y = (uint32_t)__shfl_xor((int)lmax, sh);
        lmax = y > lmax ? y : lmax;
      }
      uint64_t h = kFnvBasis;
      for (uint32_t p = 0; p <= lmax; ++p) {
        if (has && p < wl) h = (h ^ in[(uint64_t)o + p]) * kFnvPrime;
        if (has && p == wl) {
          hashes[idx] = h;
          if (sched) {
            sched[3 * idx] = lane;
            sched[3 * idx + 1] = start;
            sched[3 * idx + 2] = start + p;
          }
        }
      }
      start += lmax + 1;
    }
  }
}

hipError_t hw_enqueue_list(const uint8_t* in, uint64_t n, uint32_t* counts, uint64_t n_chunks, uint32_t* scan_sums,
                           unsigned long long* total, hipStream_t s) {
  const uint32_t g = (uint32_t)((n_chunks + 255) / 256 < 8192 ? (n_chunks + 255) / 256 : 8192);
  hipLaunchKernelGGL(k_hw_count, dim3(g ? g : 1), dim3(256), 0, s, in, n, counts, n_chunks);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return scan_exclusive_u32(counts, n_chunks, scan_sums, total, s);
}

hipError_t hw_enqueue_words(const uint8_t* in, uint64_t n, const uint32_t* first, uint64_t n_chunks, uint32_t* off,
                            uint32_t* len, hipStream_t s) {
  const uint32_t g = (uint32_t)((n_chunks + 255) / 256 < 8192 ? (n_chunks + 255) / 256 : 8192);
  hipLaunchKernelGGL(k_hw_list, dim3(g ? g : 1), dim3(256), 0, s, in, n, first, n_chunks, off, len);
  return hipGetLastError();
}

hipError_t hw_enqueue_hash(const uint8_t* in, const uint32_t* off, const uint32_t* len, uint64_t n_words, bool stream,
                           uint32_t units, uint64_t block, unsigned long long* hashes, uint32_t* sched, hipStream_t s) {
  const uint64_t nb = (n_words + block - 1) / block;
  if (nb == 0) return hipSuccess;
  if (stream)
    hipLaunchKernelGGL(k_hw_hash<true>, dim3((uint32_t)nb), dim3(64), 0, s, in, off, len, n_words, units, block, hashes, sched);
  else
    hipLaunchKernelGGL(k_hw_hash<false>, dim3((uint32_t)nb), dim3(64), 0, s, in, off, len, n_words, units, block, hashes, sched);
  return hipGetLastError();
}

}  // namespace mr
