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
  uint32_t* totals;           // device [2]
  uint32_t* bucket_cnt;       // device [n_jobs * kMaxBuckets]
  unsigned long long* bucket_bytes;
  uint32_t* bucket_start;
  unsigned long long* bucket_bstart;
  uint32_t* bucket_fill;
};

hipError_t words_enqueue_prep(const WordsLaunch& L, hipStream_t s);
hipError_t words_enqueue_map(const WordsLaunch& L, hipStream_t s);
hipError_t words_enqueue_reduce(const WordsLaunch& L, hipStream_t s);

uint32_t rgb_grid(uint64_t n, int n_cu);
hipError_t rgb_enqueue(const uint8_t* in, uint64_t n, uint32_t* partials, uint32_t G, unsigned long long* out,
                       hipStream_t s, hipEvent_t map0, hipEvent_t map1);

}  // namespace mr
