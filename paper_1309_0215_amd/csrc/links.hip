// Reverse Index on gfx950: the file list of every URL (benchmark
// application "Reverse Index", hash table container).
//
// The map (k_links_find, k_links_insert in words.hip) puts every URL into the
// word table, whose compaction and sample sort give the distinct URLs in
// bytewise order with their link counts, and leaves one (table slot, record)
// pair per link; the sort also records the output rank of each slot. Here the
// pairs are radix sorted by (rank, record), and the first of each run of equal
// pairs writes its record into the rank's list: the lists come out ascending
// and free of repeats, their offsets follow from the runs, and so do the link
// counts (the length of each rank's run).
#include "common.h"
#include "jobs.h"
#include "launch.h"

namespace mr {

constexpr uint32_t kLinksThreads = 256;
constexpr uint32_t kLinksRadixTile = 2048;  // elements per tile of the radix sort in ints.hip

__global__ void k_links_init(unsigned long long* total, unsigned long long* n_valid, uint32_t* flags) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *total = 0ull;
    *n_valid = 0ull;
    *flags = 0u;
  }
}

// Sort key of each pair: (output rank of its URL) * file_mod + record, which
// orders by rank and then record in fewer bits than a shifted rank when the
// record count is not a power of two; all ones for a marker that starts no
// link (those sort last: the sorted bits of a valid key are never all ones).
__global__ __launch_bounds__(kLinksThreads) void k_links_rank(LinksPost P) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < P.n; i += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t slot = P.pair_slot[i];
    unsigned long long key = ~0ull;
    if (slot != ~0u) {
      const uint32_t rank = P.slot_rank[slot];
      if (rank < P.n_keys) key = (unsigned long long)rank * P.file_mod + P.pair_file[i];
      else atomicOr(P.flags, kFlagInternal);  // every URL of the table has an output rank
    }
    P.k0[i] = key;
    P.v0[i] = 0ull;  // the sort carries values; these are not used
  }
}

// head[i] = 1 for the first of each run of equal valid keys; the last valid
// key writes the number of links (valid keys come first).
__global__ __launch_bounds__(kLinksThreads) void k_links_heads(const unsigned long long* __restrict__ k, uint64_t n,
                                                               uint32_t* __restrict__ head,
                                                               unsigned long long* __restrict__ n_valid) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const unsigned long long x = k[i];
    head[i] = (x != ~0ull && (i == 0 || x != k[i - 1])) ? 1u : 0u;
    if (x != ~0ull && (i + 1 == n || k[i + 1] == ~0ull)) *n_valid = i + 1;
  }
}

// After the exclusive scan of the heads: each head writes its record into
// the list at its position (positions past cap_ids are skipped: the host
// reports the capacity error after the launch); the first head of a rank writes the rank's list
// offset and its first index among the sorted pairs. list_off[n_keys] = the
// number of list entries, first[n_keys] = the number of links.
__global__ __launch_bounds__(kLinksThreads) void k_links_write(const unsigned long long* __restrict__ k, uint64_t n,
                                                               const uint32_t* __restrict__ pos, uint64_t file_mod,
                                                               const unsigned long long* __restrict__ total,
                                                               const unsigned long long* __restrict__ n_valid,
                                                               uint64_t n_keys, uint32_t* __restrict__ ids, uint64_t cap_ids,
                                                               uint64_t* __restrict__ list_off, uint32_t* __restrict__ first) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    list_off[n_keys] = *total;
    first[n_keys] = (uint32_t)*n_valid;
  }
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const unsigned long long x = k[i];
    if (x == ~0ull) continue;
    const unsigned long long prev = i ? k[i - 1] : ~0ull;
    if (i && x == prev) continue;
    const unsigned long long rank = x / file_mod;
    if (pos[i] < cap_ids) ids[pos[i]] = (uint32_t)(x - rank * file_mod);
    if (i == 0 || rank != prev / file_mod) {
      list_off[rank] = pos[i];
      first[rank] = (uint32_t)i;
    }
  }
}

// Links per URL: the length of its run among the sorted pairs.
__global__ __launch_bounds__(kLinksThreads) void k_links_counts(const uint32_t* __restrict__ first, uint64_t n_keys,
                                                                uint32_t* __restrict__ counts) {
  for (uint64_t r = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; r < n_keys; r += (uint64_t)gridDim.x * blockDim.x)
    counts[r] = first[r + 1] - first[r];
}

uint64_t links_hist_words(uint64_t n) { return 256ull * ((n + kLinksRadixTile - 1) / kLinksRadixTile); }

static uint32_t links_grid(uint64_t n) {
  const uint64_t g = (n + kLinksThreads - 1) / kLinksThreads;
  return (uint32_t)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

hipError_t links_enqueue_rank_sort(const LinksPost& P, bool* sorted_in_1, hipStream_t s) {
  *sorted_in_1 = false;
  hipLaunchKernelGGL(k_links_init, dim3(1), dim3(64), 0, s, P.total, P.n_valid, P.flags);
  if (!P.n) return hipGetLastError();
  hipLaunchKernelGGL(k_links_rank, dim3(links_grid(P.n)), dim3(kLinksThreads), 0, s, P);
  hipError_t e = radix_sort64(P.k0, P.v0, P.k1, P.v1, P.n, P.sort_bits, P.hist, P.scan_sums, sorted_in_1, s);
  if (e != hipSuccess) return e;
  const unsigned long long* k = *sorted_in_1 ? P.k1 : P.k0;
  hipLaunchKernelGGL(k_links_heads, dim3(links_grid(P.n)), dim3(kLinksThreads), 0, s, k, P.n, P.head, P.n_valid);
  return scan_exclusive_u32(P.head, P.n, P.scan_sums, P.total, s);
}

hipError_t links_enqueue_write(const LinksPost& P, bool sorted_in_1, uint32_t* ids, uint64_t cap_ids, uint64_t* list_off,
                               uint32_t* counts, hipStream_t s) {
  const unsigned long long* k = sorted_in_1 ? P.k1 : P.k0;
  hipLaunchKernelGGL(k_links_write, dim3(links_grid(P.n)), dim3(kLinksThreads), 0, s, k, P.n, P.head, P.file_mod,
                     P.total, P.n_valid, P.n_keys, ids, cap_ids, list_off, P.first);
  if (P.n_keys)
    hipLaunchKernelGGL(k_links_counts, dim3(links_grid(P.n_keys)), dim3(kLinksThreads), 0, s, P.first, P.n_keys, counts);
  return hipGetLastError();
}

}  // namespace mr
