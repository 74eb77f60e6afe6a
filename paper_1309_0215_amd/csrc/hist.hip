// RGB histogram on gfx950 (benchmark application "Histogram", array container).
//
// The key range is small (3 x 256), so each workgroup keeps its own copy of
// the array in LDS (the paper's rule of Section III-E keeps per-worker arrays
// while they are small). Each workgroup streams a contiguous range of the
// input with 16-byte non-temporal loads and bumps LDS counters; lanes spread
// over R replicas of the array to cut same-address conflicts. At the end each
// workgroup writes its partial array (no atomics), and a second kernel adds
// the partials bin by bin in 64-bit. Merging partials with global atomics
// instead would put every workgroup on the same 768 addresses.
#include "common.h"
#include "launch.h"

namespace mr {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kHistThreads = 512;
constexpr int kHistReplicas = 4;
constexpr int kHistBins = 768;

MR_DEV void count16(uint32_t* __restrict__ h, uint32_t b0, uint32_t b1, uint32_t b2, u32x4_t v) {
  // byte q of the 16 has channel (phase + q) mod 3; b0, b1, b2 are the bin bases of q mod 3 = 0, 1, 2
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
  __shared__ uint32_t h[kHistReplicas * kHistBins];
  for (int i = threadIdx.x; i < kHistReplicas * kHistBins; i += blockDim.x) h[i] = 0u;
  __syncthreads();
  const uint64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  uint32_t* hr = h + (threadIdx.x % kHistReplicas) * kHistBins;
  // aligned body [a_lo, a_hi) in absolute addresses
  const uint64_t base = (uint64_t)in;
  const uint64_t a_lo = (base + lo + 15) & ~15ull;
  const uint64_t a_hi = (base + hi) & ~15ull;
  if (a_lo < a_hi) {
    const u32x4_t* p = reinterpret_cast<const u32x4_t*>(a_lo);
    const uint64_t nv = (a_hi - a_lo) / 16;
    const uint64_t o0 = a_lo - base;  // byte offset of vector 0
    uint64_t i = threadIdx.x;
    // two loads in flight per lane
    for (; i + blockDim.x < nv; i += 2 * (uint64_t)blockDim.x) {
      const u32x4_t v0 = __builtin_nontemporal_load(p + i);
      const u32x4_t v1 = __builtin_nontemporal_load(p + i + blockDim.x);
      {
        const uint32_t ph = (uint32_t)((o0 + 16 * i) % 3);
        count16(hr, ph * 256u, ((ph + 1) % 3) * 256u, ((ph + 2) % 3) * 256u, v0);
      }
      {
        const uint32_t ph = (uint32_t)((o0 + 16 * (i + blockDim.x)) % 3);
        count16(hr, ph * 256u, ((ph + 1) % 3) * 256u, ((ph + 2) % 3) * 256u, v1);
      }
    }
    for (; i < nv; i += blockDim.x) {
      const u32x4_t v0 = __builtin_nontemporal_load(p + i);
      const uint32_t ph = (uint32_t)((o0 + 16 * i) % 3);
      count16(hr, ph * 256u, ((ph + 1) % 3) * 256u, ((ph + 2) % 3) * 256u, v0);
    }
  }
  // head and tail bytes outside the aligned body
  {
    const uint64_t head_end = a_lo < a_hi ? a_lo - base : hi;
    for (uint64_t o = lo + threadIdx.x; o < head_end; o += blockDim.x) atomicAdd(&hr[(o % 3) * 256 + in[o]], 1u);
    if (a_lo < a_hi)
      for (uint64_t o = (a_hi - base) + threadIdx.x; o < hi; o += blockDim.x) atomicAdd(&hr[(o % 3) * 256 + in[o]], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kHistBins; b += blockDim.x) {
    uint32_t s = 0;
#pragma unroll
    for (int r = 0; r < kHistReplicas; ++r) s += h[r * kHistBins + b];
    partials[(uint64_t)b * G + blockIdx.x] = s;
  }
}

__global__ __launch_bounds__(256) void k_rgb_reduce(const uint32_t* __restrict__ partials, uint32_t G,
                                                    unsigned long long* __restrict__ out) {
  __shared__ unsigned long long ws[256 / kWave];
  const uint32_t b = blockIdx.x;
  unsigned long long s = 0;
  for (uint32_t g = threadIdx.x; g < G; g += blockDim.x) s += partials[(uint64_t)b * G + g];
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o);
  if (lane_id() == 0) ws[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < 256 / kWave; ++w) t += ws[w];
    out[b] = t;
  }
}

uint32_t rgb_grid(uint64_t n, int n_cu) {
  // enough workgroups to fill the chip; each must count fewer than 2^32 bytes
  uint64_t g = (uint64_t)n_cu * 4;
  while (n / g >= (1ull << 31)) g *= 2;
  if (g > n / 64 + 1) g = n / 64 + 1;
  return (uint32_t)(g ? g : 1);
}

hipError_t rgb_enqueue(const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G, unsigned long long* out,
                       hipStream_t s, hipEvent_t map0, hipEvent_t map1) {
  if (map0) (void)hipEventRecord(map0, s);
  hipLaunchKernelGGL(k_rgb_partial, dim3(G), dim3(kHistThreads), 0, s, in, n, partials, G);
  if (map1) (void)hipEventRecord(map1, s);
  hipLaunchKernelGGL(k_rgb_reduce, dim3(kHistBins), dim3(256), 0, s, partials, G, out);
  return hipGetLastError();
}

}  // namespace mr
