// Host/device job descriptors shared by the host planner and the kernels.
// Plain data only: the host fills them and copies them to device memory.
#pragma once
#include <stdint.h>

namespace mr {

// Flag words every job carries in device memory.
enum : uint32_t {
  kFlagTableFull = 1u,   // an insert found no free slot: the table must grow
  kFlagBadInput = 2u,    // malformed record offsets or a key outside the declared range
  kFlagSpin = 4u,        // a bounded wait expired (never expected)
  kFlagCapacity = 8u,    // an output buffer was too small (sizes still reported)
  kFlagInternal = 32u,   // an internal invariant failed (reported as MR_ERR_HIP)
};


// Per-job state the kernels update in device memory. Zeroed by the host
// before each run (one memset of the whole state array).
struct JobState {
  uint64_t valid_lo;               // first input byte inside a record
  uint64_t valid_hi;               // one past the last input byte inside a record
  unsigned long long n_recs;       // distinct keys found by the compaction
  unsigned long long key_bytes;    // total output key bytes (words)
  unsigned long long claims;       // table slots claimed by the map
  uint32_t flags;                  // kFlag* bits
  uint32_t nb;                     // sort buckets
  uint32_t bucket_base;            // first global bucket of this job
  uint32_t rtile_base;             // first record tile of this job
  uint32_t sort_spills;            // sort buckets too large for LDS (sorted in global memory)
  uint32_t pad;
};

static_assert(sizeof(JobState) % 8 == 0, "JobState is cleared as 32-bit words");

// One word-count job of a batch (a single mr_run is a batch of one).
struct WordJob {
  const uint8_t* in;         // input bytes (device)
  uint64_t n;                // input length
  const uint64_t* rec;       // record offsets [n_rec + 1] or NULL
  uint64_t n_rec;
  uint64_t chunk0;           // (address of in) / 16
  uint64_t n_chunks;         // 16-byte aligned chunks covering [in, in + n)
  uint64_t tile_base;        // first map tile of this job in the batch tile space
  unsigned long long* tw;    // global table words [cap]
  uint32_t* tc;              // global table counts [cap]
  uint64_t cap;              // global table slots (power of two)
  uint64_t slot_base;        // first slot of this job's table in the table arena
  void* recs;                // compacted records [cap]
  void* recs2;               // bucket-ordered records [cap]
  uint32_t* rec_bucket;      // bucket of each compacted record [cap]
  void* splitters;           // sort splitters [kMaxBuckets - 1]
  uint8_t* out_key_bytes;    // outputs (device), may be NULL when capacities are 0
  uint64_t* out_key_offsets;
  uint32_t* out_values;
  uint64_t cap_keys;
  uint64_t cap_key_bytes;
  JobState* st;
  uint32_t* slot_rank;       // [cap] output rank of the key in each table slot, or NULL
  // partition queues of the two-phase reduce, or NULL. Map workgroup w
  // appends the words its LDS cache cannot take, and its cache entries when
  // it flushes the cache, to its own sub-queue of the key's partition
  // (records [n_parts][mq_grid][mq_cap], positions from LDS counters, no
  // global atomics; shared by the jobs of a batch) and stores the sub-queue's
  // fill in mq_fill[p * mq_grid + w]; one workgroup per partition then sums
  // the records by key. A key's partition is its 64-bit hash >> part_shift
  // (n_parts = 2^(64 - part_shift)).
  // Records of keys of up to 8 bytes (with counts below 4096 and job
  // indices below 65536) take 16 bytes in a second set of sub-queues (sq,
  // sq_fill, sq_cap, laid out alike); the others take 32 bytes in mq.
  uint32_t mq_cap;
  uint32_t mq_grid;
  void* mq;
  uint32_t* mq_fill;
  void* sq;
  uint32_t* sq_fill;
  uint32_t sq_cap;
  uint32_t part_shift;
  // 0, or log2 of the slots of one partition's region of the global table:
  // a key of partition p then lives in slots [p << region_log2, (p + 1) <<
  // region_log2) (probing wraps inside the region), so that in the summing
  // kernel only partition p's workgroup writes region p
  uint32_t region_log2;
};

constexpr uint32_t kMaxWordParts = 256;  // partitions of the two-phase reduce (the top 8 hash bits)

// Compacted table entry of a word, ordered by (p, len) then tail bytes.
struct WRec {
  uint32_t p[4];   // first 16 key bytes as big-endian words, zero padded
  uint32_t len;    // key length in bytes
  uint32_t off;    // offset of one occurrence in the input
  uint32_t cnt;    // reduced count
  uint32_t pad;
};

constexpr uint32_t kMaxBuckets = 1024;     // sort buckets per job
constexpr uint32_t kBucketCap = 2048;      // records a bucket sorts in LDS
constexpr uint32_t kRecTile = 1024;        // records per sort work item
constexpr uint32_t kMapThreads = 1024;     // word map workgroup size
constexpr uint32_t kMapTileChunks = 992;   // 16-byte chunks a map tile owns (16 waves x 62)

}  // namespace mr
