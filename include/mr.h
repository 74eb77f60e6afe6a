/*
 * mr.h - C ABI of an MI355X (gfx950) MapReduce hot path.
 *
 * The operation is the MapReduce programming model of Section II-A of
 * "Optimizing the MapReduce Framework on Intel Xeon Phi Coprocessor"
 * (arXiv 1309.0215): a map function is applied to every element of an input
 * array and emits intermediate (key, value) pairs; a reduce function combines
 * all pairs with the same key; the resulting pairs are output, ordered.
 * Reduction goes into one of the two containers of Section III-A: a hash table
 * for arbitrary keys, or an array for integer keys in a fixed range. Large
 * arrays are updated in place with atomics instead of per-worker copies
 * (Section III-E); small ones are privatised per workgroup in LDS.
 *
 * Conventions for every entry point:
 *   - Every call returns an mr_status; no exception or abort crosses the ABI.
 *     mr_last_error() returns a thread-local text with details of the last
 *     failure on the calling thread.
 *   - "device pointer" means memory on the job's GPU (hipMalloc or a torch
 *     CUDA tensor). "host pointer" means ordinary process memory.
 *   - The caller owns every buffer it passes in. Device memory the library
 *     needs beyond the inputs and outputs comes from one of two places:
 *     a caller workspace given in mr_job_config (the library then never
 *     allocates device memory; mr_workspace_bytes says how much a call
 *     needs), or, without one, device memory the library allocates for the
 *     job (grown on demand, kept between calls, freed by mr_job_destroy).
 *     stats.device_allocs counts the allocations a call made.
 *   - Calls on one mr_job are not thread-safe; use one job per host thread.
 *   - mr_run and mr_batch_run enqueue on the job's stream and synchronise that
 *     stream before returning.
 */
#ifndef MR_H_
#define MR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mr_status;
enum {
  MR_OK = 0,
  MR_ERR_INVALID_ARG = -1, /* malformed arguments; nothing was launched */
  MR_ERR_CAPACITY = -2,    /* an output buffer is too small; required sizes are set in mr_output */
  MR_ERR_OVERFLOW = -3,    /* a reduced value does not fit its output type */
  MR_ERR_HIP = -4,         /* a HIP runtime call failed */
  MR_ERR_UNSUPPORTED = -5, /* valid but unsupported combination or size */
  MR_ERR_NO_DEVICE = -6    /* no usable gfx950 device */
};

/* Map functions built into the library (Table "Benchmark applications" and
 * the workloads built on it). */
typedef enum {
  /* Word count. Input: bytes. A word is a maximal run of bytes that are not
   * one of the six ASCII whitespace bytes 0x09-0x0D, 0x20. Optional record
   * offsets cut the input into records; a record boundary ends a word.
   * Output: distinct words in unsigned bytewise order (a proper prefix
   * first) with uint32 counts. */
  MR_MAP_WORDS = 0,
  /* Integer keys. Input: little-endian uint32 keys; each emits (key, 1).
   * Output: distinct keys ascending with uint32 counts. */
  MR_MAP_U32_KEYS = 1,
  /* Integer key-value pairs. Input: little-endian (uint32 key, uint32 value)
   * pairs. Output: distinct keys ascending; SUM gives uint64 values, MIN and
   * MAX give uint32 values, COUNT gives uint32 values. */
  MR_MAP_U32_KV = 2,
  /* RGB histogram. Input: interleaved 8-bit R,G,B pixels (length a multiple
   * of 3). Output: 768 uint64 bins, channel-major: bin c*256+v counts bytes
   * of channel c equal to v. */
  MR_MAP_RGB_HIST = 3,
  /* One k-means (Lloyd) step. Input: float32 points [n][d] row-major.
   * Output: assignments int32[n], per-cluster float32 sums [k][d], uint32
   * counts [k] and new centroids [k][d] (sum / count; an empty cluster keeps
   * its previous centroid). */
  MR_MAP_KMEANS = 4,
  /* Bloom filter build (benchmark application "Bloom Filter"). Input: DNA
   * bytes. Every k-mer (bloom_k consecutive bytes, all of them A, C, G or T;
   * a k-mer holding any other byte emits nothing) is packed two bits per
   * base (A 0, C 1, G 2, T 3, first base in the highest bits) into v, and
   * x = fmix64(v), the 64-bit finaliser of MurmurHash3. It sets the
   * bloom_hashes bits g_i * m / 2^32 (integer division), i = 0, 1, ...,
   * where g_i = (low32(x) + i * (high32(x) | 1)) mod 2^32 and m = key_range,
   * the filter size in bits (1 <= m <= 2^29). Reduce: bitwise OR (op must be
   * MR_REDUCE_COUNT, the only op accepted). Output: values = uint32
   * words[ceil(m / 32)], bit b of the filter in bit b % 32 of word b / 32;
   * cap_keys is the capacity in words and n_keys the words written. */
  MR_MAP_BLOOM = 5,
  /* Reverse Index (benchmark application "Reverse Index"). Input: bytes cut
   * into files by the record offsets (without offsets, one file); file i is
   * record i. A link is the nine bytes <a href=" followed by a URL of 1 to
   * 4095 bytes other than a double quote and then a double quote, all inside
   * one file; every start position is tried, so links may overlap (a quote
   * can close one URL and end the next marker). Matching is exact: case and
   * spacing included. Output: distinct URLs in unsigned bytewise order (a
   * proper prefix first) in key_bytes / key_offsets as for MR_MAP_WORDS;
   * values[i] = number of links to URL i (uint32); list_ids[list_offsets[i]
   * .. list_offsets[i + 1]) = the distinct files linking to URL i,
   * ascending (uint32). op must be MR_REDUCE_COUNT. */
  MR_MAP_LINKS = 6
} mr_map_kind;

typedef enum { MR_REDUCE_COUNT = 0, MR_REDUCE_SUM = 1, MR_REDUCE_MIN = 2, MR_REDUCE_MAX = 3 } mr_reduce_op;

/* Reduce container strategy. RULE applies the paper's rule (Section III-E:
 * keep per-worker arrays only while each is small, otherwise one shared
 * array with atomics; hash table for keys without a fixed range). LEARNED
 * uses the trained selector when weights are loaded, otherwise RULE. The
 * other four force a container; forcing one that is infeasible for the job
 * (an array without a declared key range) returns MR_ERR_UNSUPPORTED. */
typedef enum {
  MR_STRAT_RULE = 0,
  MR_STRAT_LEARNED = 1,
  MR_STRAT_LDS_ARRAY = 2,    /* per-workgroup LDS array, partials merged without atomics */
  MR_STRAT_GLOBAL_ARRAY = 3, /* one global array updated with atomics */
  MR_STRAT_HASH = 4,         /* LDS hash cache per workgroup in front of a global open-addressing table */
  MR_STRAT_SORT = 5          /* radix sort of all pairs, then a segmented reduce */
} mr_strategy;

typedef struct mr_job mr_job;

typedef struct {
  int32_t device;          /* HIP device ordinal */
  void* stream;            /* hipStream_t to enqueue on; NULL = the null stream */
  mr_strategy strategy;    /* reduce container choice for integer-key jobs */
  uint32_t lds_slots;      /* slots of the per-workgroup LDS hash cache (power of two, 0 = default) */
  uint32_t max_load_pct;   /* global hash table load-factor limit in percent (0 = default 50) */
  uint32_t tile_bytes;     /* input bytes per work item for the word map (0 = default) */
  uint32_t debug_hash;     /* 0 = normal; 1 = force all keys to collide (tests only) */
  uint64_t table_slots;    /* initial global hash table slots (power of two, 0 = planned) */
  uint32_t timing;         /* 1 = also time the map kernel alone with HIP events (stats.map_ms) */
  /* k-means only: dimensions, clusters and the initial centroids (device, float32 [k][d]) */
  uint32_t km_d;
  uint32_t km_k;
  const float* km_centroids;
  /* Bloom filter only: k-mer length (1..32, 0 = 20) and hash count (1..8, 0 = 7) */
  uint32_t bloom_k;
  uint32_t bloom_hashes;
  /* Word count: 1 = each wave merges equal words among the 64 it holds
   * (four leader rounds) before the LDS cache insert, so repeated words take
   * one atomic (Section II-A combiner at wave level); 0 = off (default:
   * measured slower on the Zipf text, see the design notes). Outputs do not
   * depend on it. */
  uint32_t wave_combine;
  /* Caller workspace: device memory (256-byte aligned) of workspace_bytes
   * bytes that the job uses for all its device buffers instead of allocating
   * (NULL = the library allocates). It stays the caller's: it must outlive
   * the job and must not be used for anything else meanwhile, since the job
   * keeps state in it between calls (clean tables, graphs, uploaded
   * weights). A call that needs more fails with MR_ERR_CAPACITY and sets
   * stats.workspace_needed; create a job with a larger workspace then. */
  void* workspace;
  uint64_t workspace_bytes;
} mr_job_config;

typedef struct {
  uint32_t strategy_used;  /* mr_strategy actually run */
  uint32_t retries;        /* hash-table regrowths */
  uint64_t table_slots;    /* final global hash table slots */
  uint64_t n_items;        /* number of map elements (words, keys, pixels, points) */
  float gpu_ms;            /* device time of the job's kernels (HIP events) */
  float map_ms;            /* device time of the map (dominant) kernel alone; needs cfg.timing */
  uint32_t km_rechecked;   /* k-means: points whose float32 decision was re-made in float64 */
  uint32_t selector_used;  /* 1 when the learned selector chose the strategy */
  uint32_t device_allocs;  /* device allocations (hipMalloc) the library made during this call;
                              always 0 with a caller workspace */
  uint32_t sort_spills;    /* words: sort buckets too large for LDS, sorted in global memory instead */
  uint64_t workspace_needed; /* with a caller workspace that was too small (MR_ERR_CAPACITY): the
                                bytes the call had reached; 0 otherwise */
} mr_stats;

/* Output buffers (device pointers, caller-allocated) and their capacities.
 * Which fields are used depends on the map kind:
 *   WORDS:    key_bytes[cap_key_bytes], key_offsets[cap_keys + 1] (uint64),
 *             values[cap_keys] (uint32 counts)
 *   U32_*:    keys[cap_keys] (uint32), values[cap_keys] (uint32, or uint64 for SUM)
 *   RGB_HIST: values[768] (uint64)
 *   KMEANS:   assign[n] (int32), sums[k*d] (float32), counts[k] (uint32),
 *             centroids[k*d] (float32)
 *   BLOOM:    values[cap_keys] (uint32 filter words)
 *   LINKS:    as WORDS, plus list_offsets[cap_keys + 1] (uint64, required)
 *             and list_ids[cap_list_ids] (uint32)
 * On return n_keys and key_bytes_used hold the result sizes. When they
 * exceed the capacities the call returns MR_ERR_CAPACITY, leaves the output
 * buffers unspecified and keeps the required sizes here, so the caller can
 * grow its buffers and call again. For LINKS, n_list_ids is the exact list
 * size once the URL outputs fit, and an upper bound (the number of links)
 * when they do not. */
typedef struct {
  void* keys;
  uint8_t* key_bytes;
  uint64_t* key_offsets;
  void* values;
  int32_t* assign;
  float* sums;
  uint32_t* counts;
  float* centroids;
  uint64_t cap_keys;
  uint64_t cap_key_bytes;
  uint64_t n_keys;
  uint64_t key_bytes_used;
  mr_status status; /* per-item status for mr_batch_run */
  mr_stats stats;
  /* LINKS only */
  uint64_t* list_offsets;
  uint32_t* list_ids;
  uint64_t cap_list_ids;
  uint64_t n_list_ids;
} mr_output;

/* Status text ("MR_OK", ...). Never NULL. */
const char* mr_status_str(mr_status s);

/* Details of the last failure on this thread ("" if none). Never NULL. */
const char* mr_last_error(void);

/* Create a job bound to cfg->device and cfg->stream. cfg is copied; for
 * k-means the initial centroids are copied from device memory at creation.
 * Errors: MR_ERR_INVALID_ARG (NULL pointers, bad sizes), MR_ERR_NO_DEVICE. */
mr_status mr_job_create(const mr_job_config* cfg, mr_job** out);

/* Free the job and the device memory the library allocated for it (a caller
 * workspace is left alone). NULL is accepted. */
mr_status mr_job_destroy(mr_job* job);

/* Workspace bytes an mr_run of `kind` needs for inputs of up to
 * max_input_bytes bytes (and, for integer keys, declared key range
 * key_range, 0 = undeclared; for MR_MAP_BLOOM the filter bits), with the
 * job settings of *cfg (device, strategy, table and tuning fields; its
 * workspace fields are ignored). A pure host computation: the caller then
 * allocates that much and passes it in mr_job_config.workspace.
 * The figure covers the call as planned from the input size (Section II-A:
 * input array in, ordered pairs out). What the data decides beyond the plan
 * is not covered: a word or integer hash table that must grow past its
 * planned size (more distinct keys than one per 64 input bytes, or than the
 * integer range), a Reverse Index with more than one link per 512 bytes.
 * Such a call fails with MR_ERR_CAPACITY and stats.workspace_needed. For
 * mr_batch_run, plan with the batch's total size per job kind, or use the
 * figure a failed call reports. The entry points of the selector need
 * 24 KiB plus, for mr_mlp_loss_backward, 528 bytes per example.
 * Errors: MR_ERR_INVALID_ARG (NULL pointers, unknown kind, invalid cfg),
 * MR_ERR_NO_DEVICE. */
mr_status mr_workspace_bytes(const mr_job_config* cfg, mr_map_kind kind, uint64_t max_input_bytes, uint64_t key_range,
                             uint64_t* out_bytes);

/* Run one MapReduce job over d_input (device pointer, input_bytes bytes,
 * read only). d_record_offsets (device pointer, uint64[n_records + 1],
 * non-decreasing, last <= input_bytes) is only valid for MR_MAP_WORDS and
 * MR_MAP_LINKS; pass NULL for one record. Results go to *out (see mr_output).
 * Errors: MR_ERR_INVALID_ARG (bad pointers, input length not a multiple of
 * the element size, malformed record offsets, unsupported kind/op pair),
 * MR_ERR_CAPACITY, MR_ERR_UNSUPPORTED (word inputs of 4 GiB or more; integer
 * inputs of 2^32 or more elements; a forced array strategy without a key
 * range; a Bloom filter of more than 2^29 bits or with more than 2^32
 * positions), MR_ERR_HIP. key_range (0 = undeclared) declares that every uint32
 * key is < key_range, which makes the array containers feasible. Keys at or
 * above a declared range make the call fail with MR_ERR_INVALID_ARG. For
 * MR_MAP_BLOOM, key_range is the filter size m in bits (required). */
mr_status mr_run(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input, uint64_t input_bytes,
                 const uint64_t* d_record_offsets, uint64_t n_records, uint64_t key_range, mr_output* out);

/* RGB histogram (MR_MAP_RGB_HIST with MR_REDUCE_COUNT) for callers that
 * cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation. Same result as mr_run: d_bins
 * (device, uint64[768], channel-major) receives the 768 bins, overwritten.
 * It allocates nothing, sets no memory with memset calls and does not
 * synchronise: the two kernels are enqueued on the job's stream and the bins
 * are ready when that stream reaches this point.
 * Scratch: the per-workgroup partial rows go to a library-owned static device
 * array of 1024 x 768 uint32 (3 MiB), one per GPU, kept until the process
 * ends. Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other jobs, other host threads) race and give wrong
 * bins; serialise them. Errors: MR_ERR_INVALID_ARG (NULL pointers, length not
 * a multiple of 3), MR_ERR_UNSUPPORTED (inputs of 2^41 bytes or more, which
 * the 1024 rows of 32-bit counters cannot hold), MR_ERR_HIP. */
mr_status mr_rgb_hist_static(mr_job* job, const void* d_input, uint64_t input_bytes, uint64_t* d_bins);

/* FNV-1a 64 (basis 0xcbf29ce484222325, prime 0x100000001b3) of every word of
 * d_input (words as for MR_MAP_WORDS, one record), in input order, hashed one
 * character per lane per step as the string hashes of Section III-C:
 * mode 0 = SIMDH-Padding (rounds of `units` consecutive words; a round lasts
 * for its longest word, shorter ones padded), mode 1 = SIMDH-Stream (a lane
 * takes the next word as soon as its own ends; lanes freed together take the
 * next words in lane order, found from a ballot of the freed lanes and its
 * prefix count). One wavefront of which `units` (1..64) lanes hash takes
 * each block of `block` consecutive words (0 = 4096). A word's terminator
 * takes a step of its own. Outputs (device): d_hashes uint64[cap_words];
 * d_sched (optional, NULL = not written) uint32[cap_words][3] = lane, first
 * and last step of each word, steps counted from 1 within its block; on
 * return *n_words holds the number of words and *hash_ms (optional, host)
 * the device time of the hashing kernel. Errors: MR_ERR_INVALID_ARG,
 * MR_ERR_CAPACITY (more words than cap_words; *n_words is set),
 * MR_ERR_UNSUPPORTED (inputs of 4 GiB or more), MR_ERR_HIP. */
mr_status mr_hash_words(mr_job* job, const void* d_input, uint64_t input_bytes, uint32_t mode, uint32_t units,
                        uint32_t block, uint64_t* d_hashes, uint32_t* d_sched, uint64_t cap_words, uint64_t* n_words,
                        float* hash_ms);

/* One item of a batch (device pointers as in mr_run). */
typedef struct {
  mr_map_kind kind;
  mr_reduce_op op;
  const void* d_input;
  uint64_t input_bytes;
  const uint64_t* d_record_offsets;
  uint64_t n_records;
  uint64_t key_range;
} mr_batch_item;

/* Run many independent jobs in one call (the start-up cost of many small
 * jobs is what the paper's worker pool amortises, Section IV): word-count
 * items (MR_MAP_WORDS, MR_REDUCE_COUNT) and integer-key items
 * (MR_MAP_U32_KEYS, MR_MAP_U32_KV with any reduce op), in any mix.
 * Word items: one persistent map launch over a device work list of
 * (job, tile) items, then batched compaction, sort and output, captured in a
 * HIP graph that is replayed while the batch layout is unchanged.
 * Integer items: the container of each is decided first, for all of them at
 * once: with MR_STRAT_LEARNED and weights loaded, the features and the
 * network of every item run in one captured HIP graph (replayed while the
 * items' inputs stay the same) and the choices are read back once; otherwise
 * the rule or the forced container. Their containers then run one after
 * another on the job's stream in regions sized for the largest item, and
 * their states are read back once at the end.
 * outs[i] receives item i's result exactly as mr_run would produce it, and
 * outs[i].status its status. Returns MR_OK, or the first failing status. */
mr_status mr_batch_run(mr_job* job, const mr_batch_item* items, uint32_t n_items, mr_output* outs);

/* --------------------------------------------------------------------------
 * Reduce-strategy selector. Features of a job are computed on the GPU from a
 * sample of its input (mr_job_features). A 12-64-64-4 ReLU network predicts
 * the standardised log time of each of the four containers; the feasible
 * container with the lowest prediction is chosen.
 * -------------------------------------------------------------------------- */

#define MR_N_FEATURES 12
#define MR_N_STRATS 4
#define MR_MLP_PARAMS 5252

/* Compute the 12 selector features of a job into feats (host float[12]). */
mr_status mr_job_features(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input, uint64_t input_bytes,
                          uint64_t key_range, float* feats);

/* Load trained selector weights: params (host float[5252]: W1[64][12], b1[64],
 * W2[64][64], b2[64], W3[4][64], b3[4]), feature mean and scale (host
 * float[12] each; the network sees (f - mean) / scale), and the feature
 * range seen in training (host float[12] lo and hi; outside it the rule is
 * used). Passing params = NULL unloads the selector. */
mr_status mr_selector_set(mr_job* job, const float* params, const float* feat_mean, const float* feat_scale,
                          const float* feat_lo, const float* feat_hi);

/* Load trained selector weights from a JSON file (path on the host): an
 * object whose members "params" (5252 numbers), "feat_mean", "feat_scale",
 * "feat_lo" and "feat_hi" (12 numbers each) are as in mr_selector_set;
 * other members are ignored. The file the training driver writes
 * (selector_weights.json) has this form. Errors: MR_ERR_INVALID_ARG (file
 * missing or unreadable, malformed JSON, a member missing or of the wrong
 * length, a scale not positive); the job then keeps what it had loaded
 * before (without weights, MR_STRAT_LEARNED runs the rule). */
mr_status mr_selector_load(mr_job* job, const char* weights_json);

/* Training settings (zero fields take the defaults in brackets). */
typedef struct {
  uint32_t epochs; /* passes over the jobs [500] */
  uint32_t batch;  /* jobs per Adam step, at most 4096 [64] */
  float lr;        /* Adam step size [1e-3] */
  float beta1;     /* [0.9] */
  float beta2;     /* [0.999] */
  float eps;       /* [1e-8] */
  uint64_t seed;   /* initialisation and shuffling (SplitMix64) */
} mr_train_config;

/* Train the selector on measured timings and load the result into the job.
 * feats: host float[n][12], each job's mr_job_features; times: host
 * float[n][4], each container's device time in any unit (read only where
 * feasible, and positive there); feasible: host uint8[n][4] (nonzero =
 * the container can run the job). The network learns the standardised log
 * time of every feasible container (one mean and scale over all of them;
 * masked mean squared error), from He-uniform initial weights, with
 * bias-corrected Adam over shuffled batches; forward, backward and Adam run
 * on the GPU in the kernels mr_mlp_* expose. Features are standardised
 * (mean, standard deviation; a constant feature keeps scale 1) and the
 * range seen, widened by a tenth, becomes feat_lo / feat_hi. loss_out (host
 * float[epochs] or NULL) receives each epoch's mean loss; out_json (path or
 * NULL) receives the weights in the form mr_selector_load reads. Device
 * memory for the call: about 80 bytes per job, 1.1 KiB per batch example
 * and 84 KiB (a workspace region, or a library allocation freed before the
 * call returns). Errors: MR_ERR_INVALID_ARG (NULL
 * pointers, n = 0, no feasible container, a feasible time not positive,
 * batch above 4096, a beta not below 1, out_json not writable),
 * MR_ERR_CAPACITY (caller workspace too small), MR_ERR_HIP. */
mr_status mr_selector_train(mr_job* job, const float* feats, const float* times, const uint8_t* feasible, uint32_t n,
                            const mr_train_config* cfg, float* loss_out, const char* out_json);

/* Predicted standardised log times (host float[4]) for host features feats. */
mr_status mr_selector_predict(mr_job* job, const float* feats, float* pred);

/* Device kernels of the selector network, exposed for training on the GPU.
 * All pointers are device pointers to float32.
 *   mr_mlp_forward: X[B][12] -> Y[B][4]; H1 and H2 ([B][64] each) receive the
 *     post-ReLU activations for the backward pass.
 *   mr_mlp_loss_backward: masked mean squared error of Y against T with mask
 *     M ([B][4] each); writes loss[1] and the gradient grad[5252] (same
 *     layout as params).
 *   mr_mlp_adam: one bias-corrected Adam step (step = 1, 2, ...) on params
 *     with first and second moments m, v ([5252] each). */
mr_status mr_mlp_forward(mr_job* job, const float* params, const float* X, uint32_t B, float* H1, float* H2, float* Y);
mr_status mr_mlp_loss_backward(mr_job* job, const float* params, const float* X, const float* H1, const float* H2,
                               const float* Y, const float* T, const float* M, uint32_t B, float* loss, float* grad);
mr_status mr_mlp_adam(mr_job* job, float* params, const float* grad, float* m, float* v, uint32_t step, float lr,
                      float beta1, float beta2, float eps);

/* --------------------------------------------------------------------------
 * Tuned launch parameters (the batched workload's tile, load-factor and
 * privatisation thresholds). An entry covers the jobs of one map kind whose
 * input size lies in [bytes_lo, bytes_hi); the first matching entry is used.
 * Word jobs look entries up by the bytes one launch covers: a batch by its
 * total, for every parameter (the setting the tuner timed on whole
 * batches), and a single job by its own size. A nonzero field of
 * mr_job_config still wins over an entry, and an entry's zero field keeps
 * the built-in default. The project's autotuner times candidate settings
 * with this runtime and keeps the fastest per size bucket; outputs do not
 * depend on these parameters.
 * -------------------------------------------------------------------------- */
typedef struct {
  mr_map_kind kind;         /* MR_MAP_WORDS, MR_MAP_U32_KEYS or MR_MAP_U32_KV */
  uint64_t bytes_lo;        /* input sizes [bytes_lo, bytes_hi) */
  uint64_t bytes_hi;
  uint32_t lds_slots;       /* word map: LDS hash cache slots per workgroup (256, 1024, 2048 or 4096) */
  uint32_t max_load_pct;    /* global hash table load limit in percent (1..95) */
  uint32_t map_grid_pct;    /* word map: workgroups as a percentage of the CUs (1..100); fewer workgroups
                               take more 16 KiB tiles each and flush fewer LDS caches */
  uint32_t lds_array_bytes; /* uint32 jobs under the rule: LDS bytes a key range may take as
                               per-workgroup arrays (1..65536); larger ranges use the global array */
} mr_tune_entry;

/* Replace the job's tuned entries with entries[0, n) (copied). n = 0 clears
 * them. Errors: MR_ERR_INVALID_ARG for an unsupported kind, an empty size
 * range or a field outside its range (nothing is changed then). */
mr_status mr_tune_set(mr_job* job, const mr_tune_entry* entries, uint32_t n);

#ifdef __cplusplus
}
#endif
#endif /* MR_H_ */
