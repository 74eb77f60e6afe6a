// Internal launch interfaces between the host planner (api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "jobs.h"

namespace mr {

struct WordsLaunch {
  const WordJob* jobs;        // device array [n_jobs]
  const uint64_t* tile_base;  // device array [n_jobs + 1]
  uint32_t n_jobs;
  uint64_t total_tiles;
  uint64_t total_slots;       // sum of table capacities
  uint32_t map_grid;
  uint32_t sort_grid;
  int lds_log2;
  uint32_t debug_hash;
  bool any_records;
  bool wave_combine;          // merge equal words of a wave before the LDS cache (the wave-level combiner)
  uint32_t* totals;           // device [2]: buckets, record tiles
  uint32_t* bucket_cnt;       // device [n_jobs * kMaxBuckets]
  unsigned long long* bucket_bytes;
  uint32_t* bucket_start;
  unsigned long long* bucket_bstart;
  uint32_t* bucket_fill;
  JobState* states;           // device [n_jobs]
  uint32_t n_parts;            // partitions of the two-phase reduce through partition queues (0: none)
  // Reverse Index map instead of the word map (one job)
  bool links;
  uint32_t link_grid;
  uint32_t* link_marks;       // device [link_cap] marker offsets
  unsigned long long* link_n; // device: markers found
  uint64_t link_cap;
  uint32_t* link_pair_slot;          // device [link_cap] table slot of the link's URL (all ones: no link)
  uint32_t* link_pair_file;          // device [link_cap] record of the link
};

hipError_t words_enqueue_zero_states(const WordsLaunch& L, hipStream_t s);
hipError_t words_enqueue_prep(const WordsLaunch& L, hipStream_t s);
hipError_t words_enqueue_map(const WordsLaunch& L, hipStream_t s);
hipError_t words_enqueue_reduce(const WordsLaunch& L, hipStream_t s);

// Reverse Index file lists from the pairs and the sorted URLs (links.hip)
struct LinksPost {
  const uint32_t* pair_slot;    // table slot of each link's URL (all ones: no link)
  const uint32_t* pair_file;
  uint64_t n;                   // pairs (markers)
  const uint32_t* slot_rank;    // output rank of the URL in each table slot
  uint64_t n_keys;              // distinct URLs
  uint64_t file_mod;            // sort key = rank * file_mod + record (file_mod: the record count, at least 1)
  int sort_bits;                // key bits, a multiple of 8, with 2^sort_bits > n_keys * file_mod
  unsigned long long *k0, *v0, *k1, *v1;  // [n] each: sort keys, unused values, and their second buffers
  uint32_t* hist;               // radix histogram
  uint32_t* scan_sums;
  uint32_t* head;               // [n]
  unsigned long long* total;    // device: distinct (URL, file) pairs
  unsigned long long* n_valid;  // device: links
  uint32_t* flags;              // device: internal errors
  uint32_t* first;              // [n_keys + 1] first sorted pair of each rank
};
hipError_t links_enqueue_rank_sort(const LinksPost& P, bool* sorted_in_1, hipStream_t s);
hipError_t links_enqueue_write(const LinksPost& P, bool sorted_in_1, uint32_t* ids, uint64_t cap_ids, uint64_t* list_off,
                               uint32_t* counts, hipStream_t s);
uint64_t links_hist_words(uint64_t n);
hipError_t radix_sort64(unsigned long long* k0, unsigned long long* v0, unsigned long long* k1, unsigned long long* v1,
                        uint64_t n, int bits, uint32_t* hist, uint32_t* scan_sums, bool* result_in_1, hipStream_t s);

// Allocation-free histogram: partial rows in a static device array of
// kRgbStaticRows rows (3 MiB per GPU). rgb_static_init looks up its address
// on a device (once); rgb_static_rows is the row count for an input (at most
// kRgbStaticRows); rgb_static_enqueue launches the two kernels on it.
constexpr uint32_t kRgbStaticRows = 1024;
hipError_t rgb_static_init(int device);
uint32_t rgb_static_rows(uint64_t n, int n_cu);
hipError_t rgb_static_enqueue(int device, const uint8_t* in, uint64_t n, uint32_t G, unsigned long long* out,
                              hipStream_t s);
uint32_t rgb_grid(uint64_t n, int n_cu);
// map0 / map1 (optional) are recorded around k_rgb_partial.
hipError_t rgb_enqueue(const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G, unsigned long long* out,
                       hipStream_t s, hipEvent_t map0, hipEvent_t map1);
// Adds the same sequence to an empty graph g, with event-record nodes for the
// non-null events: all0, map0, k_rgb_partial, map1, k_rgb_reduce, all1.
hipError_t rgb_graph_build(hipGraph_t g, const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G,
                           unsigned long long* out, hipEvent_t all0, hipEvent_t map0, hipEvent_t map1,
                           hipEvent_t all1);

// Integer-key jobs: one launch description shared by the four containers.
struct IntLaunch {
  const uint32_t* in;
  uint64_t n;           // elements
  uint32_t kv;          // 1 = interleaved (key, value) pairs
  uint32_t op;          // 0 COUNT, 1 SUM, 2 MIN, 3 MAX
  uint64_t R;           // declared key range (0 = none)
  uint32_t G;           // workgroups of the map kernels
  uint32_t debug_hash;
  uint32_t* flags;      // device job flags
  // array containers
  uint32_t* cnt_part;
  void* val_part;
  uint32_t* dcnt;       // dense counts [R]
  void* dval;           // dense values [R] (64-bit for SUM)
  uint32_t* blk;        // compaction block counts
  // hash container
  uint32_t* t_keys;
  uint32_t* t_cnt;
  void* t_val;
  uint64_t t_cap;
  uint32_t* claimed;
  unsigned long long* n_claimed;
  uint32_t* side_cnt;
  void* side_val;
  // sort scratch
  uint32_t* rk32;
  unsigned long long *rk0, *rv0, *rk1, *rv1;
  uint32_t* hist;
  uint32_t* scan_sums;
  uint32_t* head;
  uint32_t* pos;
  uint32_t* hpos;
  unsigned long long* ps_sums;
  // outputs
  uint32_t* out_keys;
  void* out_vals;
  uint64_t cap;
  unsigned long long* n_out;  // device: number of distinct keys
};

hipError_t int_enqueue_lds_array(const IntLaunch& L, hipStream_t s);
// device-wide exclusive scan of uint32 counts (sums: scan_sums_count(n) entries)
hipError_t scan_exclusive_u32(uint32_t* a, uint64_t n, uint32_t* sums, unsigned long long* total, hipStream_t s);
uint64_t scan_sums_count(uint64_t n);

// Bloom filter build: plan and enqueue (see bloom.hip)
struct BloomPlan {
  uint64_t n_kmers;      // k-mers of the input
  uint64_t n_words;      // uint32 words of the m-bit filter
  uint32_t P;            // position ranges of 2^18 bits
  uint32_t n_tiles;      // tiles of the count and scatter passes
  uint64_t H;            // P * n_tiles range counts
  uint64_t max_entries;  // positions emitted at most (n_kmers * h)
  uint64_t part_words;   // uint32 words of the position buffer
  bool ok;               // parameters and sizes within the kernels' limits
};
BloomPlan bloom_plan(uint64_t n_bytes, uint32_t k, uint32_t h, uint64_t m);
hipError_t bloom_enqueue(const uint8_t* in, uint64_t n_bytes, uint32_t k, uint32_t h, uint64_t m, const BloomPlan& b,
                         uint32_t* hist, uint32_t* scan_sums, unsigned long long* total, uint32_t* part, uint32_t* words,
                         hipStream_t s);
// global array filled by key-range partitions (COUNT): plan and enqueue
struct PartPlan {
  uint32_t P;        // key ranges of 2^15 keys
  uint32_t n_tiles;  // tiles of elements
  uint64_t runs;     // (P + 1) * n_tiles run starts
  uint64_t part_elems;  // n_tiles * tile size: the in-range offsets, tile by tile
  bool usable;       // range, size and element count suit this fill
};
PartPlan part_plan(uint64_t n, uint64_t R);
hipError_t int_enqueue_global_array_tiles(const IntLaunch& L, const PartPlan& pp, uint32_t* runs, uint16_t* part,
                                          hipStream_t s);
hipError_t int_enqueue_global_array(const IntLaunch& L, hipStream_t s);
hipError_t int_enqueue_dense_out(const IntLaunch& L, bool clear, bool blk_counted, hipStream_t s);
hipError_t int_enqueue_hash_map(const IntLaunch& L, hipStream_t s);
hipError_t int_enqueue_hash_out(const IntLaunch& L, uint64_t n_claimed_host, hipStream_t s);
hipError_t int_enqueue_hash_sort_out(const IntLaunch& L, uint64_t n, hipStream_t s);
hipError_t int_enqueue_sort(const IntLaunch& L, hipStream_t s);
uint32_t int_lds_array_bytes(uint64_t R, uint32_t op);

// One k-means step.
struct KmLaunch {
  const float* X;       // points [N][d]
  uint64_t N;
  const float* C;       // centroids [k][d]
  uint32_t k, d;
  float* cn;            // scratch [k]
  double* cmax;         // scratch [1]
  uint32_t G;           // workgroups of the assignment kernel
  bool mfma;            // d == 32, k == 64 and X 16-byte aligned
  int32_t* assign;      // [N]
  double* part_sum;     // [G][k][d]
  uint32_t* part_cnt;   // [G][k]
  unsigned long long* n_recheck;
  unsigned long long* tiny;  // set when a coordinate is nonzero and below 2^-100 (the step is then redone generically)
  float* sums;          // [k][d]
  uint32_t* counts;     // [k]
  float* cent;          // [k][d]
};

hipError_t km_enqueue(const KmLaunch& L, hipStream_t s, hipEvent_t map0, hipEvent_t map1);

// Selector: features of a job and the network kernels.
// Selector features: one sampling workgroup per window writes its window's
// results into the state, and a finishing workgroup merges them.
uint64_t feature_state_bytes();
hipError_t features_enqueue(const uint8_t* in, uint64_t bytes, int kind, int op, uint64_t key_range, uint32_t lds_budget,
                            float* feats, void* state, hipStream_t s);
hipError_t mlp_forward_enqueue(const float* P, const float* X, uint32_t B, float* H1, float* H2, float* Y, hipStream_t s);
hipError_t select_enqueue(const float* feats, const float* norm, const float* P, uint32_t feas, int32_t* choice,
                          hipStream_t s);
hipError_t mlp_backward_enqueue(const float* P, const float* X, const float* H1, const float* H2, const float* Y,
                                const float* T, const float* M, uint32_t B, float* dY, float* dZ1, float* dZ2, float* loss,
                                float* G, hipStream_t s);
hipError_t adam_enqueue(float* P, const float* G, float* m, float* v, uint32_t step, float lr, float b1, float b2, float eps,
                        hipStream_t s);

// Word hashing one character per lane per step (strhash.hip): word starts per
// 16-byte chunk and their exclusive scan (counts[n_chunks] in place, total
// = number of words); the word list (offsets, lengths, uint32); FNV-1a 64 of
// every word with the padding or the stream schedule, `units` lanes per
// wavefront, one wavefront per `block` words; sched optional ([word][3]).
hipError_t hw_enqueue_list(const uint8_t* in, uint64_t n, uint32_t* counts, uint64_t n_chunks, uint32_t* scan_sums,
                           unsigned long long* total, hipStream_t s);
hipError_t hw_enqueue_words(const uint8_t* in, uint64_t n, const uint32_t* first, uint64_t n_chunks, uint32_t* off,
                            uint32_t* len, hipStream_t s);
hipError_t hw_enqueue_hash(const uint8_t* in, const uint32_t* off, const uint32_t* len, uint64_t n_words, bool stream,
                           uint32_t units, uint64_t block, unsigned long long* hashes, uint32_t* sched, hipStream_t s);

}  // namespace mr
