// RGB histogram on gfx950 (benchmark application "Histogram", array container).
//
// The key range is small (3 x 256), so each workgroup keeps its own copy of
// the array in LDS (the paper's rule of Section III-E keeps per-worker arrays
// while they are small). Each workgroup streams a contiguous range of the
// input with 16-byte non-temporal loads and bumps LDS counters; lanes spread
// over R replicas of the array to cut same-address conflicts. At the end each
// workgroup writes its partial array as one row (no atomics); a second kernel
// adds groups of rows in 64-bit and merges the group sums with a few atomics.
// Merging every workgroup's array with global atomics instead would put all
// of them on the same 768 addresses.
#include "common.h"
#include "launch.h"

namespace mr {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kHistThreads = 512;
constexpr int kHistReplicas = 8;
constexpr int kHistBins = 768;
// Replica stride in words: 776 = 768 + 8 puts bin b of neighbouring replicas
// in different LDS banks (with 768 every replica's bin b shares one bank).
constexpr int kHistStride = 776;
// channel phase advance (bytes mod 3) for a step of T and 2T vectors of 16 bytes
constexpr uint32_t kPhaseT = (16u * kHistThreads) % 3u;
constexpr uint32_t kPhase2T = (32u * kHistThreads) % 3u;

MR_DEV uint32_t add_mod3(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s >= 3u ? s - 3u : s;
}

MR_DEV void count16(uint32_t* __restrict__ h, uint32_t ph, u32x4_t v) {
  // byte q of the 16 has channel (ph + q) mod 3
  const uint32_t b0 = ph * 256u, b1 = add_mod3(ph, 1u) * 256u, b2 = add_mod3(ph, 2u) * 256u;
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const uint32_t byte = (w[q >> 2] >> (8 * (q & 3))) & 0xFFu;
    const uint32_t base = (q % 3 == 0) ? b0 : ((q % 3 == 1) ? b1 : b2);
    atomicAdd(&h[base + byte], 1u);
  }
}

// Each workgroup counts bytes [lo, hi) of the input (offsets relative to in).
__global__ __launch_bounds__(kHistThreads) void k_rgb_partial(const uint8_t* __restrict__ in, uint64_t n,
                                                              uint32_t* __restrict__ partials, uint32_t G) {
  __shared__ uint32_t h[kHistReplicas * kHistStride];
  for (int i = threadIdx.x; i < kHistReplicas * kHistStride; i += kHistThreads) h[i] = 0u;
  __syncthreads();
  const uint64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  uint32_t* hr = h + (threadIdx.x % kHistReplicas) * kHistStride;
  // aligned body [a_lo, a_hi) in absolute addresses
  const uint64_t base = (uint64_t)in;
  const uint64_t a_lo = (base + lo + 15) & ~15ull;
  const uint64_t a_hi = (base + hi) & ~15ull;
  if (a_lo < a_hi) {
    const u32x4_t* p = reinterpret_cast<const u32x4_t*>(a_lo);
    const uint64_t nv = (a_hi - a_lo) / 16;
    uint64_t i = threadIdx.x;
    uint32_t ph = (uint32_t)((a_lo - base + 16 * i) % 3);  // channel of the first byte of vector i
    // two loads in flight per lane
    for (; i + kHistThreads < nv; i += 2 * kHistThreads) {
      const u32x4_t v0 = __builtin_nontemporal_load(p + i);
      const u32x4_t v1 = __builtin_nontemporal_load(p + i + kHistThreads);
      count16(hr, ph, v0);
      count16(hr, add_mod3(ph, kPhaseT), v1);
      ph = add_mod3(ph, kPhase2T);
    }
    if (i < nv) count16(hr, ph, __builtin_nontemporal_load(p + i));
  }
  // head and tail bytes outside the aligned body
  {
    const uint64_t head_end = a_lo < a_hi ? a_lo - base : hi;
    for (uint64_t o = lo + threadIdx.x; o < head_end; o += kHistThreads) atomicAdd(&hr[(o % 3) * 256 + in[o]], 1u);
    if (a_lo < a_hi)
      for (uint64_t o = (a_hi - base) + threadIdx.x; o < hi; o += kHistThreads) atomicAdd(&hr[(o % 3) * 256 + in[o]], 1u);
  }
  __syncthreads();
  // one contiguous row of 768 counts per workgroup (whole cache lines)
  for (int b = threadIdx.x; b < kHistBins; b += kHistThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kHistReplicas; ++r) s += h[r * kHistStride + b];
    partials[(uint64_t)blockIdx.x * kHistBins + b] = s;
  }
}

// Bins are zero before the partial rows are added in.
__global__ __launch_bounds__(kHistBins) void k_rgb_zero(unsigned long long* __restrict__ out) {
  out[threadIdx.x] = 0ull;
}

// Workgroup q adds rows [q G / Q, (q + 1) G / Q) of the partials (thread =
// bin, so every row is read as one contiguous block) and adds its sums into
// the output: Q atomics per bin.
constexpr uint32_t kHistReduceGroups = 64;

__global__ __launch_bounds__(kHistBins) void k_rgb_reduce(const uint32_t* __restrict__ partials, uint32_t G,
                                                          unsigned long long* __restrict__ out) {
  const uint32_t b = threadIdx.x;
  const uint64_t g0 = (uint64_t)G * blockIdx.x / gridDim.x, g1 = (uint64_t)G * (blockIdx.x + 1) / gridDim.x;
  unsigned long long s = 0;
  uint64_t g = g0;
  for (; g + 4 <= g1; g += 4) {
    const uint32_t a0 = partials[g * kHistBins + b], a1 = partials[(g + 1) * kHistBins + b];
    const uint32_t a2 = partials[(g + 2) * kHistBins + b], a3 = partials[(g + 3) * kHistBins + b];
    s += (unsigned long long)a0 + a1 + a2 + a3;
  }
  for (; g < g1; ++g) s += partials[g * kHistBins + b];
  if (s) atomicAdd(&out[b], s);
}

uint32_t rgb_grid(uint64_t n, int n_cu) {
  // 16 workgroups per CU (measured best for 512 threads and 8 replicas);
  // each must count fewer than 2^32 bytes
  uint64_t g = (uint64_t)n_cu * 16;
  while (n / g >= (1ull << 31)) g *= 2;
  if (g > n / 64 + 1) g = n / 64 + 1;
  return (uint32_t)(g ? g : 1);
}

hipError_t rgb_enqueue(const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G, unsigned long long* out,
                       hipStream_t s, hipEvent_t map0, hipEvent_t map1) {
  if (map0) (void)hipEventRecord(map0, s);
  hipLaunchKernelGGL(k_rgb_partial, dim3(G), dim3(kHistThreads), 0, s, in, n, partials, G);
  if (map1) (void)hipEventRecord(map1, s);
  hipLaunchKernelGGL(k_rgb_zero, dim3(1), dim3(kHistBins), 0, s, out);
  const uint32_t q = G < kHistReduceGroups ? G : kHistReduceGroups;
  hipLaunchKernelGGL(k_rgb_reduce, dim3(q), dim3(kHistBins), 0, s, partials, G, out);
  return hipGetLastError();
}

}  // namespace mr
