// RGB histogram on gfx950 (benchmark application "Histogram", array container).
//
// The key range is small (3 x 256), so each workgroup keeps its own copy of
// the array in LDS (the paper's rule of Section III-E keeps per-worker arrays
// while they are small). Each workgroup streams a contiguous range of the
// input with 16-byte non-temporal global loads, one round of loads in flight
// while the previous one is counted, and bumps LDS counters.
//
// LDS layout: every bin has kHistCols 32-bit counters, and a lane adds into
// column (lane mod kHistCols). Consecutive words of a bin fall in consecutive
// banks, so the lanes of one atomic instruction spread over the banks
// whatever byte values they hold; with one array per workgroup (or a few
// replicas) the skewed pixel values put many lanes of an instruction on the
// same bank. The count is then bound by the loads and the per-byte address
// arithmetic (two vector instructions per byte), not by LDS conflicts.
//
// At the end each workgroup writes its partial array as one row (no atomics);
// a second kernel adds groups of rows in 64-bit and merges the group sums with
// a few atomics. Merging every workgroup's array with global atomics instead
// would put all of them on the same 768 addresses.
#include "common.h"
#include "launch.h"

namespace mr {

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

constexpr int kHistThreads = 512;
constexpr int kHistBins = 768;
constexpr int kHistCols = 16;    // counters per bin (one per lane column)
constexpr int kHistUnroll = 2;   // 16-byte vectors per lane per round
// channel phase advance (bytes mod 3) for a step of kHistThreads vectors of 16 bytes
constexpr uint32_t kPhaseT = (16u * kHistThreads) % 3u;

MR_DEV uint32_t add_mod3(uint32_t a, uint32_t b) {
  const uint32_t s = a + b;
  return s >= 3u ? s - 3u : s;
}

// Word of bin (channel base cb = channel * 256 * kHistCols + column, byte v).
MR_DEV uint32_t hist_word(uint32_t cb, uint32_t v) { return cb + v * kHistCols; }

MR_DEV void count16(uint32_t* __restrict__ h, uint32_t col, uint32_t ph, u32x4_t v) {
  // byte q of the 16 has channel (ph + q) mod 3
  const uint32_t b0 = ph * 256u * kHistCols + col;
  const uint32_t b1 = add_mod3(ph, 1u) * 256u * kHistCols + col;
  const uint32_t b2 = add_mod3(ph, 2u) * 256u * kHistCols + col;
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const uint32_t byte = (w[q >> 2] >> (8 * (q & 3))) & 0xFFu;
    const uint32_t cb = (q % 3 == 0) ? b0 : ((q % 3 == 1) ? b1 : b2);
    atomicAdd(&h[hist_word(cb, byte)], 1u);
  }
}

// Each workgroup counts bytes [lo, hi) of the input (offsets relative to in).
// Workgroup 0 also clears the output bins, which the reduce kernel launched
// after this one adds into.
__global__ __launch_bounds__(kHistThreads) void k_rgb_partial(const uint8_t* __restrict__ in, uint64_t n,
                                                              uint32_t* __restrict__ partials, uint32_t G,
                                                              unsigned long long* __restrict__ out) {
  constexpr int kWords = kHistBins * kHistCols;
  __shared__ uint32_t h[kWords];
  if (blockIdx.x == 0)
    for (int b = threadIdx.x; b < kHistBins; b += kHistThreads) out[b] = 0ull;
  for (int i = threadIdx.x; i < kWords; i += kHistThreads) h[i] = 0u;
  __syncthreads();
  const uint64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  const uint32_t col = lane_id() & (kHistCols - 1);
  // aligned body [a_lo, a_hi) in absolute addresses
  const uint64_t base = (uint64_t)in;
  const uint64_t a_lo = (base + lo + 15) & ~15ull;
  const uint64_t a_hi = (base + hi) & ~15ull;
  if (a_lo < a_hi) {
    const MR_GLOBAL u32x4_t* p = reinterpret_cast<const MR_GLOBAL u32x4_t*>(a_lo);
    const uint64_t nv = (a_hi - a_lo) / 16;
    constexpr uint64_t kRound = (uint64_t)kHistUnroll * kHistThreads;  // vectors per round
    const uint64_t rounds = nv / kRound;
    uint32_t ph = (uint32_t)((a_lo - base + 16ull * threadIdx.x) % 3);  // channel of this lane's next vector
    // Two register buffers: one round's loads are in flight while the other
    // is counted. The loads inside the loop are unconditional, so the
    // compiler's wait counts let them overlap.
    u32x4_t A[kHistUnroll], B[kHistUnroll];
    auto load = [&](u32x4_t* buf, uint64_t r) {
#pragma unroll
      for (int u = 0; u < kHistUnroll; ++u) buf[u] = __builtin_nontemporal_load(p + r * kRound + threadIdx.x + u * kHistThreads);
    };
    auto count = [&](const u32x4_t* buf) {
#pragma unroll
      for (int u = 0; u < kHistUnroll; ++u) {
        count16(h, col, ph, buf[u]);
        ph = add_mod3(ph, kPhaseT);
      }
    };
    uint64_t r = 0;
    if (rounds) load(A, 0);
    for (; r + 2 < rounds; r += 2) {
      load(B, r + 1);
      count(A);
      load(A, r + 2);
      count(B);
    }
    if (r + 1 < rounds) {
      load(B, r + 1);
      count(A);
      count(B);
    } else if (r < rounds) {
      count(A);
    }
    for (uint64_t i = rounds * kRound + threadIdx.x; i < nv; i += kHistThreads) {
      count16(h, col, ph, __builtin_nontemporal_load(p + i));
      ph = add_mod3(ph, kPhaseT);
    }
  }
  // head and tail bytes outside the aligned body
  {
    const uint64_t head_end = a_lo < a_hi ? a_lo - base : hi;
    for (uint64_t o = lo + threadIdx.x; o < head_end; o += kHistThreads)
      atomicAdd(&h[hist_word((uint32_t)(o % 3) * 256u * kHistCols + col, in[o])], 1u);
    if (a_lo < a_hi)
      for (uint64_t o = (a_hi - base) + threadIdx.x; o < hi; o += kHistThreads)
        atomicAdd(&h[hist_word((uint32_t)(o % 3) * 256u * kHistCols + col, in[o])], 1u);
  }
  __syncthreads();
  // one contiguous row of 768 counts per workgroup (whole cache lines); the
  // column order is rotated per bin so that neighbouring threads read
  // different banks
  for (int b = threadIdx.x; b < kHistBins; b += kHistThreads) {
    uint32_t s = 0;
#pragma unroll
    for (int l = 0; l < kHistCols; ++l) s += h[b * kHistCols + ((l + b) & (kHistCols - 1))];
    partials[(uint64_t)blockIdx.x * kHistBins + b] = s;
  }
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
  // 4 workgroups per CU (measured best for 512 threads, 16 columns and
  // 48 KiB of LDS each); each must count fewer than 2^32 bytes
  uint64_t g = (uint64_t)n_cu * 4;
  while (n / g >= (1ull << 31)) g *= 2;
  if (g > n / 64 + 1) g = n / 64 + 1;
  return (uint32_t)(g ? g : 1);
}

hipError_t rgb_enqueue(const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G, unsigned long long* out,
                       hipStream_t s, hipEvent_t map0, hipEvent_t map1) {
  if (map0) (void)hipEventRecord(map0, s);
  hipLaunchKernelGGL(k_rgb_partial, dim3(G), dim3(kHistThreads), 0, s, in, n, partials, G, out);
  if (map1) (void)hipEventRecord(map1, s);
  const uint32_t q = G < kHistReduceGroups ? G : kHistReduceGroups;
  hipLaunchKernelGGL(k_rgb_reduce, dim3(q), dim3(kHistBins), 0, s, partials, G, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Allocation-free variant: the partial rows live in a file-scope device array
// (one copy per GPU, held until the process ends) instead of a workspace.
// Host code never passes the array's name to a kernel (on the host it only
// stands in for the symbol): its device address is looked up once per device
// with hipGetSymbolAddress and used from then on.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint32_t scratch[kRgbStaticRows * kHistBins];

namespace {
constexpr int kMaxDevices = 64;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t rgb_static_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (g_scratch_ptr[device]) return hipSuccess;
  int prev = -1;
  hipError_t e = hipGetDevice(&prev);
  if (e != hipSuccess) return e;
  if (prev != device && (e = hipSetDevice(device)) != hipSuccess) return e;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch_ptr[device] = ptr;
  if (prev != device) (void)hipSetDevice(prev);
  return e;
}

uint32_t rgb_static_rows(uint64_t n, int n_cu) {
  const uint32_t g = rgb_grid(n, n_cu);
  return g < kRgbStaticRows ? g : kRgbStaticRows;
}

hipError_t rgb_static_enqueue(int device, const uint8_t* in, uint64_t n, uint32_t G, unsigned long long* out,
                              hipStream_t s) {
  if (device < 0 || device >= kMaxDevices || !g_scratch_ptr[device]) return hipErrorNotInitialized;
  if (G == 0 || G > kRgbStaticRows) return hipErrorInvalidValue;
  return rgb_enqueue(in, n, static_cast<uint32_t*>(g_scratch_ptr[device]), G, out, s, nullptr, nullptr);
}

// The same sequence as a graph built node by node: event records around
// the whole sequence (all0, all1) and around k_rgb_partial (map0, map1, may
// be null). Built explicitly rather than by stream capture, since event
// records inside a capture are not supported by every HIP runtime.
hipError_t rgb_graph_build(hipGraph_t g, const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G,
                           unsigned long long* out, hipEvent_t all0, hipEvent_t map0, hipEvent_t map1,
                           hipEvent_t all1) {
  hipError_t e = hipSuccess;
  hipGraphNode_t prev = nullptr, node = nullptr;
  auto add_event = [&](hipEvent_t ev) -> hipError_t {
    if (!ev) return hipSuccess;
    const hipError_t r = hipGraphAddEventRecordNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, ev);
    if (r == hipSuccess) prev = node;
    return r;
  };
  auto add_kernel = [&](const void* fn, dim3 grid, dim3 block, void** args) -> hipError_t {
    hipKernelNodeParams kp{};
    kp.func = const_cast<void*>(fn);
    kp.gridDim = grid;
    kp.blockDim = block;
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    const hipError_t r = hipGraphAddKernelNode(&node, g, prev ? &prev : nullptr, prev ? 1 : 0, &kp);
    if (r == hipSuccess) prev = node;
    return r;
  };
  const uint32_t q = G < kHistReduceGroups ? G : kHistReduceGroups;
  void* a_partial[] = {&in, &n, &partials, &G, &out};
  void* a_reduce[] = {&partials, &G, &out};
  if ((e = add_event(all0)) != hipSuccess) return e;
  if ((e = add_event(map0)) != hipSuccess) return e;
  if ((e = add_kernel(reinterpret_cast<const void*>(&k_rgb_partial), dim3(G), dim3(kHistThreads), a_partial)) != hipSuccess)
    return e;
  if ((e = add_event(map1)) != hipSuccess) return e;
  if ((e = add_kernel(reinterpret_cast<const void*>(&k_rgb_reduce), dim3(q), dim3(kHistBins), a_reduce)) != hipSuccess)
    return e;
  return add_event(all1);
}

}  // namespace mr
