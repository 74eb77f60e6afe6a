// Host side of the C ABI declared in include/mr.h: argument checks, planning,
// workspace management, kernel enqueue, retries and status reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/mr.h"
#include "jobs.h"
#include "launch.h"

using namespace mr;

namespace {

thread_local std::string g_last_error;

mr_status fail(mr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define MR_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(MR_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

uint64_t sel_floats();  // floats of the selector region

uint64_t next_pow2(uint64_t x) {
  uint64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint64_t align_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

}  // namespace

// ----------------------------------------------------------------------------
// job object
// ----------------------------------------------------------------------------

struct mr_job {
  mr_job_config cfg{};
  hipStream_t stream = nullptr;
  int device = 0;
  int n_cu = 256;
  // one device workspace, grown on demand; the table region must be all zero between runs
  uint8_t* ws = nullptr;
  uint64_t ws_bytes = 0;
  uint64_t table_clean_bytes = 0;  // [0, table_clean_bytes) of ws is known to be all zero
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr;
  // selector
  bool sel_loaded = false;
  std::vector<float> sel_params, sel_mean, sel_scale, sel_lo, sel_hi;
  // k-means centroids (device; a host copy re-fills them when a caller
  // workspace region holding them was overwritten)
  float* km_c = nullptr;
  uint64_t km_c_bytes = 0;
  std::vector<float> km_host;
  // batched graph cache: valid while nothing else has written the workspace
  hipGraphExec_t graph = nullptr;
  // selection graph of a batch's integer items (features and network per item)
  hipGraphExec_t sel_graph = nullptr;
  uint64_t sel_graph_key = 0;
  hipEvent_t ev_int0 = nullptr, ev_int1 = nullptr;  // around a batch's integer items
  uint64_t graph_key = 0;
  bool graph_valid = false;
  uint64_t plain_key = 0;  // launch-sequence identity of the last plain word pass
  // RGB histogram graph: a repeated call (same input, size, output, workspace) replays it
  hipGraphExec_t rgb_graph = nullptr;
  uint64_t rgb_graph_key = 0;
  uint64_t rgb_plain_key = 0;
  bool rgb_graph_off = false;  // the runtime refused to build or run the graph: plain launches only
  // the graph's own timing events: whole sequence, then the partial kernel
  hipEvent_t rgb_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // final table size of the last single word job and the input it ran on
  // final table size of recent word jobs by input (address, length): a job
  // over the same input starts at the size it grew to, in a batch too
  std::unordered_map<uint64_t, uint64_t> table_hint;
  hipStream_t gstream = nullptr;  // non-blocking stream for graph capture (the job's may be the null stream)
  // pinned host staging for job states
  JobState* h_states = nullptr;
  uint32_t h_states_cap = 0;
  // integer-key containers: persistent and kept clean between runs
  void* int_dense = nullptr;     // dense counts [R] then values [R] (64-bit)
  uint64_t int_dense_R = 0;      // R of the dense layout
  uint64_t int_dense_bytes = 0;
  void* int_table = nullptr;     // keys [cap], counts [cap], values [cap] (64-bit), claimed [cap]
  uint64_t int_table_bytes = 0;  // (int_table_cap: the cap of the layout)
  uint64_t int_table_cap = 0;
  void* int_small = nullptr;     // flags, counters, side slot
  uint64_t int_small_bytes = 0;
  void* int_scratch = nullptr;   // partials, sort records, scans
  uint64_t int_scratch_bytes = 0;
  uint64_t int_last_distinct = 0;
  // selector scratch (device): features, inputs, outputs, parameters; MLP training scratch
  void* sel_dev = nullptr;
  uint64_t sel_dev_bytes = 0;
  void* mlp_dev = nullptr;
  uint64_t mlp_dev_bytes = 0;
  // Reverse Index: marker list and pairs (sized by link_cap), then the sort scratch
  void* link_dev = nullptr;
  uint64_t link_dev_bytes = 0;
  uint64_t link_cap = 0;
  // tuned launch parameters by map kind and input size
  std::vector<mr_tune_entry> tune;
  // device memory accounting: hipMalloc calls during the current call and in total
  uint32_t call_allocs = 0;
  uint64_t total_allocs = 0;
  // caller-owned workspace (cfg.workspace): every device buffer of a call is a
  // region of it, carved in request order from offset 0 (so a call repeating
  // the previous call's requests finds its regions where they were); the
  // library then never allocates device memory
  uint8_t* cws = nullptr;
  uint64_t cws_bytes = 0;
  uint64_t cws_off = 0;    // end of the current call's regions
  uint64_t cws_need = 0;   // bytes the current call needed when it ran out (0: it fit)
  int cws_family = -1;     // which entry point family the last call was
  bool cws_prefix = true;  // every region of this call so far matches the last call's
  struct Region {
    int id;
    uint64_t off, bytes;
    bool operator==(const Region& o) const { return id == o.id && off == o.off && bytes == o.bytes; }
  };
  std::vector<Region> cws_prev, cws_cur;
  bool sel_uploaded = false;  // the selector weights are in the device region
};

namespace {

// Every entry point selects the job's device and starts from a clear HIP
// error state, so that an error left behind by other code in the process is
// not reported as a failure of this call (kernel launches are checked with
// hipGetLastError).
struct ScopedDevice {
  int prev = -1;
  hipError_t stale = hipSuccess;
  explicit ScopedDevice(int d) {
    stale = hipGetLastError();
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != d) (void)hipSetDevice(d);
  }
  ~ScopedDevice() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

// Workspace layout carved for one run: offsets from ws.
struct Carve {
  uint64_t off = 0;
  uint64_t take(uint64_t bytes, uint64_t align = 256) {
    off = align_up(off, align);
    const uint64_t o = off;
    off += bytes;
    return o;
  }
};

// Device regions of a job and the entry-point families that use them.
enum RegionId {
  kRegWs = 1, kRegKmC, kRegSmall, kRegDense, kRegTable, kRegScratch, kRegSel, kRegMlp, kRegLink, kRegTrain, kRegHashList
};
enum Family {
  kFamWords = 1, kFamRgb, kFamKmeans, kFamBloom, kFamU32, kFamLinks, kFamFeatures, kFamPredict, kFamMlp, kFamTrain, kFamBatch,
  kFamHash
};

// Start of a call of `family`. With a caller workspace the call carves its
// regions from offset 0; a region keeps its contents from the last call only
// when that call was of the same family and every region requested up to it
// had the same place and size (then no other region overlapped it since).
void arena_begin(mr_job* job, int family) {
  job->call_allocs = 0;
  job->cws_need = 0;
  if (!job->cws) return;
  job->cws_prev.clear();
  if (family == job->cws_family) job->cws_prev.swap(job->cws_cur);
  job->cws_cur.clear();
  job->cws_off = 0;
  job->cws_prefix = true;
  if (family != job->cws_family) {
    // the workspace was used by another kind of call: nothing in it is known
    job->table_clean_bytes = 0;
    job->graph_valid = false;
    job->sel_uploaded = false;
  }
  job->cws_family = family;
}

// Device memory of region `id`, at least `want` bytes, at *p (size in *have).
// Library memory: a buffer already large enough is kept (*fresh = false);
// otherwise it is replaced by `alloc` >= want new bytes (*fresh = true:
// contents undefined; the old buffer is freed after the job's streams are
// synchronised). Caller workspace: the next `want` bytes of the workspace
// (256-byte aligned). A region requested again in the same call is the same
// one when it is large enough (*fresh = false: contents as this call left
// them), is extended in place when it is the last one, and is otherwise
// taken anew after the others. For a first request *fresh tells whether the
// contents are those the last call left there. A workspace
// too small fails with MR_ERR_CAPACITY and the bytes needed in cws_need.
mr_status dev_region(mr_job* job, int id, void** p, uint64_t* have, uint64_t want, uint64_t alloc, bool* fresh) {
  if (!job->cws) {
    if (*p && *have >= want) {
      *fresh = false;
      return MR_OK;
    }
    if (*p) {
      MR_HIP(hipStreamSynchronize(job->stream));
      if (job->gstream) MR_HIP(hipStreamSynchronize(job->gstream));
      MR_HIP(hipFree(*p));
      *p = nullptr;
      *have = 0;
    }
    alloc = std::max(alloc, want);
    hipError_t e = hipMalloc(p, alloc);
    if (e != hipSuccess) return fail(MR_ERR_HIP, "hipMalloc(%llu) failed: %s", (unsigned long long)alloc, hipGetErrorString(e));
    ++job->call_allocs;
    ++job->total_allocs;
    *have = alloc;
    *fresh = true;
    return MR_OK;
  }
  auto& cur = job->cws_cur;
  for (size_t i = cur.size(); i-- > 0;) {
    // a region this call already carved and large enough: the same one again
    if (cur[i].id == id && cur[i].bytes >= want) {
      *p = job->cws + cur[i].off;
      *have = cur[i].bytes;
      *fresh = false;
      return MR_OK;
    }
    if (cur[i].id == id) break;
  }
  if (!cur.empty() && cur.back().id == id) {
    // the last region again: extend it in place
    mr_job::Region& r = cur.back();
    if (r.off + want > job->cws_bytes) {
      job->cws_need = r.off + want;
      return fail(MR_ERR_CAPACITY, "the workspace (%llu bytes) is too small: this call needs %llu bytes",
                  (unsigned long long)job->cws_bytes, (unsigned long long)job->cws_need);
    }
    if (want > r.bytes) {
      r.bytes = want;
      job->cws_prefix = false;
    }
    job->cws_off = r.off + r.bytes;
    *p = job->cws + r.off;
    *have = r.bytes;
    *fresh = !job->cws_prefix;
    return MR_OK;
  }
  const uint64_t o = align_up(job->cws_off, 256);
  if (o + want > job->cws_bytes) {
    job->cws_need = o + want;
    return fail(MR_ERR_CAPACITY, "the workspace (%llu bytes) is too small: this call needs %llu bytes",
                (unsigned long long)job->cws_bytes, (unsigned long long)job->cws_need);
  }
  const mr_job::Region r{id, o, want};
  const size_t i = cur.size();
  if (!(job->cws_prefix && i < job->cws_prev.size() && job->cws_prev[i] == r)) job->cws_prefix = false;
  cur.push_back(r);
  job->cws_off = o + want;
  *p = job->cws + o;
  *have = want;
  *fresh = !job->cws_prefix;
  return MR_OK;
}

mr_status ensure_ws(mr_job* job, uint64_t bytes) {
  void* p = job->ws;
  bool fresh = false;
  mr_status st = dev_region(job, kRegWs, &p, &job->ws_bytes, bytes, std::max<uint64_t>(bytes, job->ws_bytes + job->ws_bytes / 2),
                            &fresh);
  if (st != MR_OK) return st;
  job->ws = static_cast<uint8_t*>(p);
  if (fresh) {
    job->table_clean_bytes = 0;
    job->graph_valid = false;
  }
  return MR_OK;
}

mr_status ensure_host_states(mr_job* job, uint32_t n) {
  if (n <= job->h_states_cap) return MR_OK;
  if (job->h_states) (void)hipHostFree(job->h_states);
  job->h_states = nullptr;
  MR_HIP(hipHostMalloc(&job->h_states, sizeof(JobState) * n, hipHostMallocDefault));
  job->h_states_cap = n;
  return MR_OK;
}

// The tuned entry for a job of this kind and input size, or NULL.
const mr_tune_entry* tune_for(const mr_job* job, mr_map_kind kind, uint64_t bytes) {
  for (const mr_tune_entry& e : job->tune)
    if (e.kind == kind && bytes >= e.bytes_lo && bytes < e.bytes_hi) return &e;
  return nullptr;
}

// Effective parameters: the job's explicit setting, else the tuned one, else the default.
uint32_t eff_load_pct(const mr_job* job, mr_map_kind kind, uint64_t bytes) {
  if (job->cfg.max_load_pct) return job->cfg.max_load_pct;
  const mr_tune_entry* t = tune_for(job, kind, bytes);
  return t && t->max_load_pct ? t->max_load_pct : 50u;
}

uint32_t eff_lds_slots(const mr_job* job, uint64_t bytes) {
  if (job->cfg.lds_slots) return job->cfg.lds_slots;
  const mr_tune_entry* t = tune_for(job, MR_MAP_WORDS, bytes);
  return t && t->lds_slots ? t->lds_slots : 4096u;
}

uint32_t eff_grid_pct(const mr_job* job, uint64_t bytes) {
  const mr_tune_entry* t = tune_for(job, MR_MAP_WORDS, bytes);
  return t && t->map_grid_pct ? t->map_grid_pct : 100u;
}

}  // namespace

// ----------------------------------------------------------------------------
// status helpers
// ----------------------------------------------------------------------------

extern "C" const char* mr_status_str(mr_status s) {
  switch (s) {
    case MR_OK: return "MR_OK";
    case MR_ERR_INVALID_ARG: return "MR_ERR_INVALID_ARG";
    case MR_ERR_CAPACITY: return "MR_ERR_CAPACITY";
    case MR_ERR_OVERFLOW: return "MR_ERR_OVERFLOW";
    case MR_ERR_HIP: return "MR_ERR_HIP";
    case MR_ERR_UNSUPPORTED: return "MR_ERR_UNSUPPORTED";
    case MR_ERR_NO_DEVICE: return "MR_ERR_NO_DEVICE";
    default: return "MR_ERR_UNKNOWN";
  }
}

extern "C" const char* mr_last_error(void) { return g_last_error.c_str(); }

extern "C" mr_status mr_job_create(const mr_job_config* cfg, mr_job** out) {
  if (!cfg || !out) return fail(MR_ERR_INVALID_ARG, "mr_job_create: NULL argument");
  *out = nullptr;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev <= 0) return fail(MR_ERR_NO_DEVICE, "no HIP device");
  if (cfg->device < 0 || cfg->device >= n_dev) return fail(MR_ERR_INVALID_ARG, "device %d out of range", cfg->device);
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, cfg->device) != hipSuccess) return fail(MR_ERR_NO_DEVICE, "device query failed");
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return fail(MR_ERR_NO_DEVICE, "device %d is %s, this library is built for gfx950", cfg->device, prop.gcnArchName);
  if (cfg->lds_slots && (cfg->lds_slots & (cfg->lds_slots - 1)))
    return fail(MR_ERR_INVALID_ARG, "lds_slots must be a power of two");
  if (cfg->table_slots && (cfg->table_slots & (cfg->table_slots - 1)))
    return fail(MR_ERR_INVALID_ARG, "table_slots must be a power of two");
  if (cfg->max_load_pct > 95) return fail(MR_ERR_INVALID_ARG, "max_load_pct above 95");
  if ((cfg->workspace_bytes && !cfg->workspace) || (cfg->workspace && (uintptr_t)cfg->workspace % 256))
    return fail(MR_ERR_INVALID_ARG, "the workspace must be a 256-byte aligned device pointer with its size");
  mr_job* job = new (std::nothrow) mr_job();
  if (!job) return fail(MR_ERR_INVALID_ARG, "out of host memory");
  job->cfg = *cfg;
  job->device = cfg->device;
  job->stream = static_cast<hipStream_t>(cfg->stream);
  job->n_cu = prop.multiProcessorCount;
  job->cws = static_cast<uint8_t*>(cfg->workspace);
  job->cws_bytes = cfg->workspace ? cfg->workspace_bytes : 0;
  ScopedDevice sd(job->device);
  if (hipEventCreate(&job->ev0) != hipSuccess || hipEventCreate(&job->ev1) != hipSuccess ||
      hipEventCreate(&job->ev2) != hipSuccess || hipEventCreate(&job->ev3) != hipSuccess ||
      hipStreamCreateWithFlags(&job->gstream, hipStreamNonBlocking) != hipSuccess) {
    delete job;
    return fail(MR_ERR_HIP, "hipEventCreate failed");
  }
  // the allocation-free histogram's static scratch: its address on this device, looked up once
  if (rgb_static_init(job->device) != hipSuccess) {
    mr_job_destroy(job);
    return fail(MR_ERR_HIP, "looking up the static histogram scratch on device %d failed", cfg->device);
  }
  if (cfg->km_k) {
    if (!cfg->km_centroids || cfg->km_d == 0 || cfg->km_d > 256 || cfg->km_k > 1024) {
      mr_job_destroy(job);
      return fail(MR_ERR_INVALID_ARG, "k-means needs centroids, 1 <= d <= 256 and 1 <= k <= 1024");
    }
    // kept on the host; each run places them in a device region
    job->km_host.resize((size_t)cfg->km_d * cfg->km_k);
    if (hipMemcpyAsync(job->km_host.data(), cfg->km_centroids, sizeof(float) * job->km_host.size(), hipMemcpyDeviceToHost,
                       job->stream) != hipSuccess ||
        hipStreamSynchronize(job->stream) != hipSuccess) {
      mr_job_destroy(job);
      return fail(MR_ERR_HIP, "copying the initial centroids failed");
    }
  }
  *out = job;
  return MR_OK;
}

extern "C" mr_status mr_job_destroy(mr_job* job) {
  if (!job) return MR_OK;
  ScopedDevice sd(job->device);
  if (job->stream) (void)hipStreamSynchronize(job->stream);
  if (job->graph) (void)hipGraphExecDestroy(job->graph);
  if (job->rgb_graph) (void)hipGraphExecDestroy(job->rgb_graph);
  if (job->sel_graph) (void)hipGraphExecDestroy(job->sel_graph);
  if (job->ev_int0) (void)hipEventDestroy(job->ev_int0);
  if (job->ev_int1) (void)hipEventDestroy(job->ev_int1);
  for (hipEvent_t e : job->rgb_ev)
    if (e) (void)hipEventDestroy(e);
  if (job->gstream) (void)hipStreamSynchronize(job->gstream);
  if (job->gstream) (void)hipStreamDestroy(job->gstream);
  if (job->h_states) (void)hipHostFree(job->h_states);
  if (!job->cws) {  // regions of a caller workspace belong to the caller
    for (void* p : {(void*)job->ws, (void*)job->km_c, job->int_dense, job->int_table, job->int_small, job->int_scratch,
                    job->sel_dev, job->mlp_dev, job->link_dev})
      if (p) (void)hipFree(p);
  }
  if (job->ev0) (void)hipEventDestroy(job->ev0);
  if (job->ev1) (void)hipEventDestroy(job->ev1);
  if (job->ev2) (void)hipEventDestroy(job->ev2);
  if (job->ev3) (void)hipEventDestroy(job->ev3);
  delete job;
  return MR_OK;
}

// ----------------------------------------------------------------------------
// word count (one job or a batch)
// ----------------------------------------------------------------------------

namespace {

// Device buffers of the Reverse Index map (one job).
struct LinkBufs {
  uint32_t* marks;
  unsigned long long* n_marks;
  uint64_t cap;
  uint32_t* pair_slot;
  uint32_t* pair_file;
  uint32_t* slot_rank;  // set by the pass: output rank of each table slot
  unsigned long long h_n_marks;  // set by the pass: markers found (read back with the job states)
};

struct WordItem {
  const uint8_t* in;
  uint64_t n;
  const uint64_t* rec;
  uint64_t n_rec;
  mr_output* out;
  uint64_t cap;  // planned table slots
};

// Initial table capacity for an input of n bytes: words <= (n + 1) / 2 and
// distinct words <= words; start from a sixteenth of the bytes and let a full
// table trigger regrowth.
// size_key: the input size the tuned load limit is looked up by.
uint64_t initial_slots(const mr_job* job, uint64_t n, uint64_t size_key) {
  // (at least 4096 slots: the compaction takes 4096-slot pieces of one table)
  if (job->cfg.table_slots) return std::max<uint64_t>(4096, job->cfg.table_slots);
  const double lf = eff_load_pct(job, MR_MAP_WORDS, size_key) / 100.0;
  const uint64_t words_ub = (n + 1) / 2;
  uint64_t est = std::min<uint64_t>(words_ub, std::max<uint64_t>(2048, n / 64));
  uint64_t slots = next_pow2((uint64_t)std::ceil(est / lf));
  return std::max<uint64_t>(4096, std::min<uint64_t>(slots, 1ull << 21));
}

struct WordsPlan {
  Carve c;
  uint64_t o_jobs, o_tile_base, o_states, o_totals, o_bucket_cnt, o_bucket_bytes, o_bucket_start, o_bucket_bstart,
      o_bucket_fill, o_tw, o_tc, o_recs, o_recs2, o_rbucket, o_spl, o_slot_rank = 0;
  uint32_t n_parts = 0;  // partitions of the two-phase reduce (0: none)
  uint64_t o_mq = 0, o_mqfill = 0, o_sq = 0, o_sqfill = 0;
  uint32_t mq_cap = 0, sq_cap = 0, grid = 1;  // records per 32-byte and 16-byte sub-queue; map workgroups
  uint64_t total_slots = 0, total_tiles = 0;
  std::vector<uint64_t> slot_base, tile_base;
};

// Partitions of the two-phase reduce: 256. More partitions would let the
// distinct keys of a partition fit one summing workgroup's LDS table on
// high-cardinality inputs, but each map workgroup keeps one partly written
// line open per partition, and with 4096 partitions those lines no longer
// fit the L2 (measured on 512 MiB of text: map 575 -> 754 us).
uint32_t word_parts(uint64_t) { return 256u; }

// Records per sub-queue of each kind (one per map workgroup and partition,
// shared by the jobs of a batch): room for half the words of an input of mean
// word length 8 missing the LDS caches, spread evenly, plus the entries of the
// caches the workgroup flushes (3/4 of 4096 slots, once per job it meets: at
// most n_jobs + grid flushes in all), with half again as slack; either kind
// can take all of them. A full sub-queue sends its overflow to the global
// table directly.
uint32_t miss_queue_cap(uint64_t n, uint32_t grid, uint32_t parts, uint64_t n_jobs) {
  const uint64_t misses = n / (16ull * grid * parts);
  const uint64_t flushed = 3072ull * (n_jobs + grid) / ((uint64_t)grid * parts);
  const uint64_t want = misses + flushed + 1;
  return (uint32_t)std::min<uint64_t>(6144, std::max<uint64_t>(16, want + want / 2));
}

WordsPlan plan_words(const std::vector<WordItem>& items, bool slot_ranks, bool queues, uint64_t grid_cap) {
  WordsPlan p;
  const uint32_t n = (uint32_t)items.size();
  p.slot_base.resize(n);
  p.tile_base.resize(n + 1);
  for (uint32_t j = 0; j < n; ++j) {
    p.slot_base[j] = p.total_slots;
    p.total_slots += items[j].cap;
    p.tile_base[j] = p.total_tiles;
    const uint64_t a = (uint64_t)items[j].in;
    const uint64_t n_chunks = items[j].n ? ((a + items[j].n + 15) / 16 - a / 16) : 0;
    p.total_tiles += (n_chunks + kMapTileChunks - 1) / kMapTileChunks;
  }
  p.tile_base[n] = p.total_tiles;
  // (the summing kernel of the partition queues takes at most 1024 map workgroups)
  p.grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(std::min<uint64_t>(p.total_tiles, grid_cap), 1024));
  // the table arena comes first so that its clean prefix survives layout changes
  p.o_tw = p.c.take(p.total_slots * 8);
  p.o_tc = p.c.take(p.total_slots * 4);
  p.o_jobs = p.c.take(sizeof(WordJob) * n);
  p.o_tile_base = p.c.take(8 * (n + 1));
  p.o_states = p.c.take(sizeof(JobState) * n);
  p.o_totals = p.c.take(16);
  p.o_bucket_cnt = p.c.take(4ull * n * kMaxBuckets);
  p.o_bucket_bytes = p.c.take(8ull * n * kMaxBuckets);
  p.o_bucket_start = p.c.take(4ull * n * kMaxBuckets);
  p.o_bucket_bstart = p.c.take(8ull * n * kMaxBuckets);
  p.o_bucket_fill = p.c.take(4ull * n * kMaxBuckets);
  p.o_recs = p.c.take(sizeof(WRec) * p.total_slots);
  p.o_recs2 = p.c.take(sizeof(WRec) * p.total_slots);
  p.o_rbucket = p.c.take(4 * p.total_slots);
  p.o_spl = p.c.take(sizeof(WRec) * (kMaxBuckets - 1) * (uint64_t)n);
  if (slot_ranks) p.o_slot_rank = p.c.take(4 * p.total_slots);
  if (queues) {
    uint64_t total_n = 0;
    for (const WordItem& it : items) total_n += it.n;
    p.n_parts = word_parts(total_n);
    p.mq_cap = p.sq_cap = miss_queue_cap(total_n, p.grid, p.n_parts, n);
    p.o_mq = p.c.take(32ull * p.n_parts * p.grid * p.mq_cap);
    p.o_mqfill = p.c.take(4ull * p.n_parts * p.grid);
    p.o_sq = p.c.take(16ull * p.n_parts * p.grid * p.sq_cap);
    p.o_sqfill = p.c.take(4ull * p.n_parts * p.grid);
  }
  return p;
}

mr_status zero_device(hipStream_t s, void* p, uint64_t bytes) {
  if (!bytes) return MR_OK;
  if (bytes % 4 == 0 && (uintptr_t)p % 4 == 0) {
    MR_HIP(hipMemsetD32Async((hipDeviceptr_t)p, 0, bytes / 4, s));
  } else {
    MR_HIP(hipMemsetAsync(p, 0, bytes, s));
  }
  return MR_OK;
}

// How a word pass is launched: plain launches, a HIP graph (captured once
// per launch-sequence identity and replayed), or plain on first sight and a
// graph when the same sequence comes again.
enum class GraphMode { kNever, kAlways, kOnRepeat };

// Runs a batch of word-count items once; fills states[] (host). The caller
// handles regrowth and results.
uint64_t fnv_mix(uint64_t h, uint64_t v) {
  for (int i = 0; i < 8; ++i) {
    h ^= (v >> (8 * i)) & 0xFF;
    h *= 0x100000001B3ull;
  }
  return h;
}

// Identity of a job's input for the table-size hints.
uint64_t input_key(const uint8_t* in, uint64_t n) { return fnv_mix(fnv_mix(0xCBF29CE484222325ull, (uint64_t)in), n); }

mr_status words_pass(mr_job* job, std::vector<WordItem>& items, std::vector<JobState>& states, float* gpu_ms,
                     float* map_ms, GraphMode mode, LinkBufs* lb) {
  const uint32_t n = (uint32_t)items.size();
  // word jobs send their cache misses and flushed cache entries through
  // partition queues (shared by the jobs of a batch), summed per partition
  const bool queues = lb == nullptr;
  // tuned map parameters, looked up by the bytes this launch covers (a
  // batch by its total; each job's table load factor by its own size)
  uint64_t size_key = 0;
  for (const WordItem& it : items) size_key += it.n;
  const uint32_t lds_slots = eff_lds_slots(job, size_key);
  int lds_log2 = 0;
  while ((1u << lds_log2) < lds_slots) ++lds_log2;
  if (lds_log2 != 8 && lds_log2 != 10 && lds_log2 != 11 && lds_log2 != 12)
    return fail(MR_ERR_INVALID_ARG, "lds_slots must be 256, 1024, 2048 or 4096");
  const uint64_t grid_cap = std::max<uint64_t>(1, (uint64_t)job->n_cu * eff_grid_pct(job, size_key) / 100);
  WordsPlan p = plan_words(items, lb != nullptr, queues, grid_cap);
  mr_status st = ensure_ws(job, p.c.off);
  if (st != MR_OK) return st;
  uint8_t* ws = job->ws;
  // identity of the launch sequence: a captured graph replays only for the same one
  uint64_t key = 0xCBF29CE484222325ull;
  key = fnv_mix(key, (uint64_t)ws);
  key = fnv_mix(key, n);
  key = fnv_mix(key, (uint64_t)lds_log2);
  key = fnv_mix(key, grid_cap);
  key = fnv_mix(key, job->cfg.debug_hash);
  key = fnv_mix(key, job->cfg.wave_combine);
  key = fnv_mix(key, lb ? (uint64_t)lb->marks ^ lb->cap : 0ull);
  for (const WordItem& it : items) {
    key = fnv_mix(key, (uint64_t)it.in);
    key = fnv_mix(key, it.n);
    key = fnv_mix(key, (uint64_t)it.rec);
    key = fnv_mix(key, it.n_rec);
    key = fnv_mix(key, it.cap);
    key = fnv_mix(key, (uint64_t)it.out->key_bytes);
    key = fnv_mix(key, (uint64_t)it.out->key_offsets);
    key = fnv_mix(key, (uint64_t)it.out->values);
    key = fnv_mix(key, it.out->cap_keys);
    key = fnv_mix(key, it.out->cap_key_bytes);
  }
  // A repeated call with the same layout is captured once and then replayed
  // (per-kernel timing needs plain launches).
  const bool use_graph = mode == GraphMode::kAlways || (mode == GraphMode::kOnRepeat && !job->cfg.timing &&
                                                       (key == job->plain_key || key == job->graph_key));
  job->plain_key = use_graph ? 0 : key;
  // Everything runs on the job's stream; a graph is only captured on the
  // capture stream (the job's stream may be the null stream, which cannot
  // be captured) and is launched on the job's stream, which orders it after
  // the work before it without an event.
  const hipStream_t s = job->stream;
  const uint64_t table_bytes_g = p.o_tc + p.total_slots * 4;
  if (use_graph && job->graph && job->graph_valid && job->graph_key == key && job->table_clean_bytes >= table_bytes_g) {
    // replay: descriptors, tile bases and the clean table are still in place
    job->table_clean_bytes = 0;
    MR_HIP(hipEventRecord(job->ev0, s));
    MR_HIP(hipGraphLaunch(job->graph, s));
    MR_HIP(hipEventRecord(job->ev1, s));
    st = ensure_host_states(job, n);
    if (st != MR_OK) return st;
    MR_HIP(hipMemcpyAsync(job->h_states, ws + p.o_states, sizeof(JobState) * n, hipMemcpyDeviceToHost, s));
    MR_HIP(hipStreamSynchronize(s));
    states.assign(job->h_states, job->h_states + n);
    float ms = 0.f;
    MR_HIP(hipEventElapsedTime(&ms, job->ev0, job->ev1));
    *gpu_ms = ms;
    *map_ms = 0.f;
    bool dirty = false;
    for (auto& s : states) dirty |= (s.flags & kFlagTableFull) != 0;
    job->table_clean_bytes = dirty ? 0 : table_bytes_g;
    if (dirty) job->graph_valid = false;
    return MR_OK;
  }
  job->graph_valid = false;  // this pass rewrites the descriptors
  // the table arena must start all zero
  const uint64_t table_bytes = p.o_tc + p.total_slots * 4;
  if (job->table_clean_bytes < table_bytes) {
    st = zero_device(s, ws + job->table_clean_bytes, table_bytes - job->table_clean_bytes);
    if (st != MR_OK) return st;
  }
  job->table_clean_bytes = 0;  // until this pass completes
  std::vector<WordJob> hj(n);
  bool any_rec = false;
  for (uint32_t j = 0; j < n; ++j) {
    WordJob& J = hj[j];
    const WordItem& it = items[j];
    J.in = it.in;
    J.n = it.n;
    J.rec = it.rec;
    J.n_rec = it.n_rec;
    const uint64_t a = (uint64_t)it.in;
    J.chunk0 = a / 16;
    J.n_chunks = it.n ? ((a + it.n + 15) / 16 - a / 16) : 0;
    J.tile_base = p.tile_base[j];
    J.tw = reinterpret_cast<unsigned long long*>(ws + p.o_tw) + p.slot_base[j];
    J.tc = reinterpret_cast<uint32_t*>(ws + p.o_tc) + p.slot_base[j];
    J.cap = it.cap;
    J.slot_base = p.slot_base[j];
    J.recs = reinterpret_cast<WRec*>(ws + p.o_recs) + p.slot_base[j];
    J.recs2 = reinterpret_cast<WRec*>(ws + p.o_recs2) + p.slot_base[j];
    J.rec_bucket = reinterpret_cast<uint32_t*>(ws + p.o_rbucket) + p.slot_base[j];
    J.splitters = reinterpret_cast<WRec*>(ws + p.o_spl) + (uint64_t)j * (kMaxBuckets - 1);
    J.out_key_bytes = it.out->key_bytes;
    J.out_key_offsets = it.out->key_offsets;
    J.out_values = static_cast<uint32_t*>(it.out->values);
    J.cap_keys = it.out->cap_keys;
    J.cap_key_bytes = it.out->cap_key_bytes;
    J.st = reinterpret_cast<JobState*>(ws + p.o_states) + j;
    J.slot_rank = lb ? reinterpret_cast<uint32_t*>(ws + p.o_slot_rank) + p.slot_base[j] : nullptr;
    J.mq_cap = p.mq_cap;
    J.mq_grid = p.grid;
    J.mq = p.n_parts ? ws + p.o_mq : nullptr;
    J.mq_fill = p.n_parts ? reinterpret_cast<uint32_t*>(ws + p.o_mqfill) : nullptr;
    J.sq_cap = p.sq_cap;
    J.sq = p.n_parts ? ws + p.o_sq : nullptr;
    J.sq_fill = p.n_parts ? reinterpret_cast<uint32_t*>(ws + p.o_sqfill) : nullptr;
    J.part_shift = p.n_parts ? 64u - (uint32_t)__builtin_ctz(p.n_parts) : 64u;
    // large tables are split into one region per partition (not with forced
    // hash collisions, which put every key of a length into one region)
    J.region_log2 = (p.n_parts && !job->cfg.debug_hash && it.cap >= 256ull * p.n_parts)
                        ? (uint32_t)__builtin_ctzll(it.cap) - (uint32_t)__builtin_ctz(p.n_parts)
                        : 0u;
    any_rec |= it.rec != nullptr;
  }
  MR_HIP(hipMemcpyAsync(ws + p.o_jobs, hj.data(), sizeof(WordJob) * n, hipMemcpyHostToDevice, s));
  MR_HIP(hipMemcpyAsync(ws + p.o_tile_base, p.tile_base.data(), 8 * (n + 1), hipMemcpyHostToDevice, s));

  WordsLaunch L{};
  L.jobs = reinterpret_cast<const WordJob*>(ws + p.o_jobs);
  L.tile_base = reinterpret_cast<const uint64_t*>(ws + p.o_tile_base);
  L.n_jobs = n;
  L.total_tiles = p.total_tiles;
  L.total_slots = p.total_slots;
  L.map_grid = p.grid;
  L.sort_grid = (uint32_t)std::max(1, job->n_cu * 2);
  L.lds_log2 = lds_log2;
  L.n_parts = p.n_parts;
  L.debug_hash = job->cfg.debug_hash;
  L.any_records = any_rec;
  L.wave_combine = job->cfg.wave_combine != 0;
  L.totals = reinterpret_cast<uint32_t*>(ws + p.o_totals);
  L.bucket_cnt = reinterpret_cast<uint32_t*>(ws + p.o_bucket_cnt);
  L.bucket_bytes = reinterpret_cast<unsigned long long*>(ws + p.o_bucket_bytes);
  L.bucket_start = reinterpret_cast<uint32_t*>(ws + p.o_bucket_start);
  L.bucket_bstart = reinterpret_cast<unsigned long long*>(ws + p.o_bucket_bstart);
  L.bucket_fill = reinterpret_cast<uint32_t*>(ws + p.o_bucket_fill);

  L.states = reinterpret_cast<JobState*>(ws + p.o_states);
  if (lb) {
    L.links = true;
    L.link_grid = (uint32_t)std::max(1, job->n_cu * 8);
    L.link_marks = lb->marks;
    L.link_n = lb->n_marks;
    L.link_cap = lb->cap;
    L.link_pair_slot = lb->pair_slot;
    L.link_pair_file = lb->pair_file;
    lb->slot_rank = reinterpret_cast<uint32_t*>(ws + p.o_slot_rank);
  }
  if (use_graph) {
    // capture the whole sequence (no memset nodes: states are cleared by a kernel)
    if (job->graph) {
      MR_HIP(hipGraphExecDestroy(job->graph));
      job->graph = nullptr;
    }
    hipGraph_t g = nullptr;
    const hipStream_t cs = job->gstream;
    MR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = words_enqueue_zero_states(L, cs);
    if (e == hipSuccess) e = words_enqueue_prep(L, cs);
    if (e == hipSuccess) e = words_enqueue_map(L, cs);
    if (e == hipSuccess) e = words_enqueue_reduce(L, cs);
    const hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(MR_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&job->graph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(MR_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    job->graph_key = key;
    MR_HIP(hipEventRecord(job->ev0, s));
    MR_HIP(hipGraphLaunch(job->graph, s));
    MR_HIP(hipEventRecord(job->ev1, s));
  } else {
    MR_HIP(hipEventRecord(job->ev0, s));
    MR_HIP(words_enqueue_zero_states(L, s));
    MR_HIP(words_enqueue_prep(L, s));
    if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev2, s));
    MR_HIP(words_enqueue_map(L, s));
    if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev3, s));
    MR_HIP(words_enqueue_reduce(L, s));
    MR_HIP(hipEventRecord(job->ev1, s));
  }
  // (with markers, their count comes back in the same round trip, in the
  // pinned buffer's entry past the states)
  st = ensure_host_states(job, n + (lb ? 1u : 0u));
  if (st != MR_OK) return st;
  MR_HIP(hipMemcpyAsync(job->h_states, ws + p.o_states, sizeof(JobState) * n, hipMemcpyDeviceToHost, s));
  if (lb) MR_HIP(hipMemcpyAsync(&job->h_states[n], lb->n_marks, 8, hipMemcpyDeviceToHost, s));
  MR_HIP(hipStreamSynchronize(s));
  states.assign(job->h_states, job->h_states + n);
  if (lb) std::memcpy(&lb->h_n_marks, &job->h_states[n], 8);
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, job->ev0, job->ev1));
  *gpu_ms = ms;
  *map_ms = 0.f;
  // (a graph replays the whole sequence: the map is timed with plain launches only)
  if (job->cfg.timing && !use_graph) MR_HIP(hipEventElapsedTime(map_ms, job->ev2, job->ev3));
  // The compaction zeroes every slot it reads, so after a complete pass the
  // table region [0, table_bytes) is zero again. Everything past it was just
  // used for descriptors, records and buckets and is not. A pass that stopped
  // on a full table leaves slots behind.
  bool dirty = false;
  for (auto& s : states) dirty |= (s.flags & kFlagTableFull) != 0;
  job->table_clean_bytes = dirty ? 0 : table_bytes;
  job->graph_valid = use_graph && !dirty;
  return MR_OK;
}

mr_status check_words_item(const WordItem& it) {
  if (!it.out) return fail(MR_ERR_INVALID_ARG, "NULL output");
  if (it.n && !it.in) return fail(MR_ERR_INVALID_ARG, "NULL input with nonzero length");
  if (it.n >= (1ull << 32)) return fail(MR_ERR_UNSUPPORTED, "word inputs must be below 4 GiB");
  if (it.rec && it.n_rec == 0) return fail(MR_ERR_INVALID_ARG, "record offsets need n_records >= 1");
  if ((it.out->cap_keys && (!it.out->key_offsets || !it.out->values)) || (it.out->cap_key_bytes && !it.out->key_bytes))
    return fail(MR_ERR_INVALID_ARG, "output capacity given without buffers");
  if (!it.out->key_offsets) return fail(MR_ERR_INVALID_ARG, "key_offsets is required (at least one entry)");
  return MR_OK;
}

mr_status run_words(mr_job* job, std::vector<WordItem>& items, std::vector<mr_status>* per_item, GraphMode use_graph,
                    LinkBufs* lb = nullptr) {
  // a batch takes its tuned parameters, the load limit included, from the
  // entry for its total size (the setting the tuner timed on whole batches);
  // a single job from the entry for its own size
  uint64_t total = 0;
  for (const auto& it : items) total += it.n;
  for (auto& it : items) {
    mr_status s = check_words_item(it);
    if (s != MR_OK) return s;
    it.cap = initial_slots(job, it.n, items.size() > 1 ? total : it.n);
    // a job over an input seen before starts at the size its table grew to
    if (!job->cfg.table_slots) {
      const auto h = job->table_hint.find(input_key(it.in, it.n));
      if (h != job->table_hint.end()) it.cap = std::max(it.cap, h->second);
    }
  }
  std::vector<JobState> states;
  uint32_t retries = 0;
  float total_ms = 0.f, map_ms = 0.f;
  for (;;) {
    float ms = 0.f;
    mr_status s = words_pass(job, items, states, &ms, &map_ms, use_graph, lb);
    if (s != MR_OK) return s;
    total_ms += ms;
    bool regrow = false;
    for (size_t j = 0; j < items.size(); ++j) {
      if (states[j].flags & kFlagTableFull) {
        if (items[j].cap >= (1ull << 31)) return fail(MR_ERR_CAPACITY, "hash table cannot grow beyond 2^31 slots");
        // the first estimate was off by an unknown factor: grow fast
        items[j].cap = std::min<uint64_t>(items[j].cap * 4, 1ull << 31);
        regrow = true;
      }
    }
    if (!regrow) break;
    if (++retries > 24) return fail(MR_ERR_CAPACITY, "hash table regrowth did not converge");
  }
  if (job->table_hint.size() > 65536) job->table_hint.clear();
  for (const WordItem& it : items) job->table_hint[input_key(it.in, it.n)] = it.cap;
  mr_status first = MR_OK;
  for (size_t j = 0; j < items.size(); ++j) {
    mr_output* o = items[j].out;
    const JobState& s = states[j];
    o->n_keys = s.n_recs;
    o->key_bytes_used = s.key_bytes;
    o->stats.strategy_used = MR_STRAT_HASH;
    o->stats.retries = retries;
    o->stats.table_slots = items[j].cap;
    o->stats.gpu_ms = total_ms;
    o->stats.map_ms = map_ms;
    o->stats.n_items = 0;
    o->stats.sort_spills = s.sort_spills;
    mr_status r = MR_OK;
    if (s.flags & kFlagBadInput) r = fail(MR_ERR_INVALID_ARG, "malformed record offsets (item %zu)", j);
    else if (s.flags & kFlagSpin) r = fail(MR_ERR_HIP, "bounded wait expired (item %zu)", j);
    else if (s.flags & kFlagInternal) r = fail(MR_ERR_HIP, "internal table invariant failed (item %zu)", j);
    else if (s.flags & kFlagCapacity)
      r = fail(MR_ERR_CAPACITY, "output needs %llu keys and %llu key bytes (item %zu)", (unsigned long long)s.n_recs,
               (unsigned long long)s.key_bytes, j);
    o->status = r;
    if (per_item) (*per_item)[j] = r;
    if (first == MR_OK && r != MR_OK) first = r;
  }
  return first;
}

// ----------------------------------------------------------------------------
// Reverse Index: the word pass with the link map, then the file lists
// ----------------------------------------------------------------------------

uint32_t bits_for(uint64_t n) {  // smallest b with 2^b >= n
  uint32_t b = 0;
  while (b < 64 && (1ull << b) < n) ++b;
  return b;
}

mr_status ensure_link_dev(mr_job* job, uint64_t bytes) {
  bool fresh = false;
  return dev_region(job, kRegLink, &job->link_dev, &job->link_dev_bytes, bytes, bytes, &fresh);
}

mr_status run_links(mr_job* job, mr_reduce_op op, const void* d_input, uint64_t bytes, const uint64_t* rec, uint64_t n_rec,
                    mr_output* out) {
  if (op != MR_REDUCE_COUNT) return fail(MR_ERR_UNSUPPORTED, "the Reverse Index takes MR_REDUCE_COUNT");
  if (!out->list_offsets) return fail(MR_ERR_INVALID_ARG, "list_offsets is required (at least one entry)");
  if (out->cap_list_ids && !out->list_ids) return fail(MR_ERR_INVALID_ARG, "cap_list_ids given without list_ids");
  if (rec && n_rec >= (1ull << 32)) return fail(MR_ERR_UNSUPPORTED, "at most 2^32 - 1 files");
  // marker list: one per 512 input bytes to start with, grown to the count found
  uint64_t cap = std::max<uint64_t>(4096, std::max<uint64_t>(job->link_cap, bytes / 512));
  std::vector<WordItem> items(1);
  mr_status st = MR_OK;
  unsigned long long n_marks = 0;
  Carve c;
  uint64_t o_marks = 0, o_n = 0, o_slot = 0, o_file = 0;
  LinkBufs lb{};
  for (int attempt = 0;; ++attempt) {
    c = Carve{};
    o_n = c.take(8);
    o_marks = c.take(4 * cap);
    o_slot = c.take(4 * cap);
    o_file = c.take(4 * cap);
    st = ensure_link_dev(job, c.off);
    if (st != MR_OK) return st;
    uint8_t* d = static_cast<uint8_t*>(job->link_dev);
    lb = LinkBufs{reinterpret_cast<uint32_t*>(d + o_marks), reinterpret_cast<unsigned long long*>(d + o_n), cap,
                  reinterpret_cast<uint32_t*>(d + o_slot), reinterpret_cast<uint32_t*>(d + o_file), nullptr, 0ull};
    items[0] = WordItem{static_cast<const uint8_t*>(d_input), bytes, rec, n_rec, out, 0};
    st = run_words(job, items, nullptr, GraphMode::kNever, &lb);
    if (st != MR_OK && st != MR_ERR_CAPACITY) return st;
    n_marks = lb.h_n_marks;
    if (n_marks <= cap) break;
    if (attempt >= 2) return fail(MR_ERR_HIP, "marker list did not converge");
    cap = next_pow2(n_marks);
  }
  job->link_cap = cap;
  out->stats.n_items = 0;
  if (st == MR_ERR_CAPACITY) {  // the URL outputs did not fit: report an upper bound of the list size
    out->n_list_ids = n_marks;
    return st;
  }
  // file lists
  const uint64_t n = n_marks, nk = out->n_keys;
  // key = rank * F + record, below n_keys * F; all ones in the sorted bits marks no link
  const uint64_t F = rec ? std::max<uint64_t>(n_rec, 1) : 1;
  const uint32_t kb = bits_for(nk * F + 1);
  const int sort_bits = (int)std::max<uint32_t>(8, (kb + 7) / 8 * 8);
  const uint64_t hw = links_hist_words(n);
  Carve c2 = c;
  const uint64_t o_k0 = c2.take(8 * n), o_v0 = c2.take(8 * n), o_k1 = c2.take(8 * n), o_v1 = c2.take(8 * n);
  const uint64_t o_hist = c2.take(4 * std::max<uint64_t>(hw, 1));
  const uint64_t o_sums = c2.take(4 * std::max(scan_sums_count(hw), scan_sums_count(n)));
  const uint64_t o_head = c2.take(4 * std::max<uint64_t>(n, 1)), o_tot = c2.take(8), o_val = c2.take(8), o_fl = c2.take(8);
  const uint64_t o_first = c2.take(4 * (nk + 1));
  if (c2.off > job->link_dev_bytes) {
    // keep the pairs: grow into a new buffer (library memory) or a new region
    // after the others (caller workspace) and copy the map's part across
    void* nd = nullptr;
    uint64_t nh = 0;
    bool fresh = false;
    st = dev_region(job, kRegLink, &nd, &nh, c2.off, c2.off, &fresh);
    if (st != MR_OK) return st;
    MR_HIP(hipMemcpyAsync(nd, job->link_dev, c.off, hipMemcpyDeviceToDevice, job->stream));
    MR_HIP(hipStreamSynchronize(job->stream));
    if (!job->cws) MR_HIP(hipFree(job->link_dev));
    job->link_dev = nd;
    job->link_dev_bytes = nh;
  }
  uint8_t* d = static_cast<uint8_t*>(job->link_dev);
  LinksPost P{};
  P.pair_slot = reinterpret_cast<const uint32_t*>(d + o_slot);
  P.pair_file = reinterpret_cast<const uint32_t*>(d + o_file);
  P.n = n;
  P.slot_rank = lb.slot_rank;
  P.n_keys = nk;
  P.file_mod = F;
  P.sort_bits = sort_bits;
  P.k0 = reinterpret_cast<unsigned long long*>(d + o_k0);
  P.v0 = reinterpret_cast<unsigned long long*>(d + o_v0);
  P.k1 = reinterpret_cast<unsigned long long*>(d + o_k1);
  P.v1 = reinterpret_cast<unsigned long long*>(d + o_v1);
  P.hist = reinterpret_cast<uint32_t*>(d + o_hist);
  P.scan_sums = reinterpret_cast<uint32_t*>(d + o_sums);
  P.head = reinterpret_cast<uint32_t*>(d + o_head);
  P.total = reinterpret_cast<unsigned long long*>(d + o_tot);
  P.n_valid = reinterpret_cast<unsigned long long*>(d + o_val);
  P.flags = reinterpret_cast<uint32_t*>(d + o_fl);
  P.first = reinterpret_cast<uint32_t*>(d + o_first);
  MR_HIP(hipEventRecord(job->ev0, job->stream));
  bool in1 = false;
  MR_HIP(links_enqueue_rank_sort(P, &in1, job->stream));
  // the lists are written at once (entries past the capacity are skipped);
  // their size and the error flag are checked after the one synchronisation
  MR_HIP(links_enqueue_write(P, in1, out->list_ids, out->cap_list_ids, out->list_offsets,
                             static_cast<uint32_t*>(out->values), job->stream));
  unsigned long long tv[2] = {0, 0};
  uint32_t flags = 0;
  MR_HIP(hipMemcpyAsync(&tv[0], P.total, 8, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipMemcpyAsync(&tv[1], P.n_valid, 8, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipMemcpyAsync(&flags, P.flags, 4, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipEventRecord(job->ev1, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  if (flags) return fail(MR_ERR_HIP, "internal error: a link's URL is missing from the sorted URLs");
  out->n_list_ids = tv[0];
  out->stats.n_items = tv[1];
  if (tv[0] > out->cap_list_ids)
    return fail(MR_ERR_CAPACITY, "the file lists need %llu entries", (unsigned long long)tv[0]);
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, job->ev0, job->ev1));
  out->stats.gpu_ms += ms;
  return MR_OK;
}

}  // namespace

// ----------------------------------------------------------------------------
// RGB histogram
// ----------------------------------------------------------------------------

namespace {

mr_status run_rgb(mr_job* job, const void* d_input, uint64_t bytes, mr_output* out) {
  if (bytes % 3) return fail(MR_ERR_INVALID_ARG, "RGB input length %llu is not a multiple of 3", (unsigned long long)bytes);
  if (!out->values) return fail(MR_ERR_INVALID_ARG, "RGB output needs values[768]");
  const uint32_t G = rgb_grid(bytes, job->n_cu);
  Carve c;
  const uint64_t o_part = c.take(4ull * 768 * G);
  mr_status st = ensure_ws(job, c.off);
  if (st != MR_OK) return st;
  job->table_clean_bytes = std::min(job->table_clean_bytes, o_part);  // scratch overwrites the table region
  job->graph_valid = false;
  uint32_t* partials = reinterpret_cast<uint32_t*>(job->ws + o_part);
  unsigned long long* bins = static_cast<unsigned long long*>(out->values);
  // The second call with the same launch sequence builds it as a graph and
  // later ones replay it: one submission, so the events around the kernels
  // are not spread apart by host launch latency. The partial rows live in the
  // workspace, whose address is part of the identity. A runtime that refuses
  // the graph leaves the job on plain launches.
  uint64_t key = input_key(static_cast<const uint8_t*>(d_input), bytes);
  key = fnv_mix(key, (uint64_t)bins);
  key = fnv_mix(key, (uint64_t)partials);
  key = fnv_mix(key, ((uint64_t)G << 1) | (job->cfg.timing ? 1u : 0u));
  bool use_graph = !job->rgb_graph_off && (key == job->rgb_plain_key || (job->rgb_graph && key == job->rgb_graph_key));
  job->rgb_plain_key = use_graph ? 0 : key;
  hipEvent_t e_all0 = job->ev0, e_all1 = job->ev1, e_map0 = job->ev2, e_map1 = job->ev3;
  hipStream_t s = job->stream;
  if (use_graph && (!job->rgb_graph || job->rgb_graph_key != key)) {
    if (job->rgb_graph) {
      MR_HIP(hipGraphExecDestroy(job->rgb_graph));
      job->rgb_graph = nullptr;
    }
    for (hipEvent_t& e : job->rgb_ev)
      if (!e) MR_HIP(hipEventCreate(&e));
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e == hipSuccess)
      e = rgb_graph_build(g, static_cast<const uint8_t*>(d_input), bytes, partials, G, bins, job->rgb_ev[0],
                          job->cfg.timing ? job->rgb_ev[2] : nullptr, job->cfg.timing ? job->rgb_ev[3] : nullptr,
                          job->rgb_ev[1]);
    if (e == hipSuccess) e = hipGraphInstantiate(&job->rgb_graph, g, nullptr, nullptr, 0);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      // keep the job working with plain launches
      (void)hipGetLastError();
      job->rgb_graph = nullptr;
      job->rgb_graph_off = true;
      use_graph = false;
    } else {
      job->rgb_graph_key = key;
    }
  }
  if (use_graph) {
    e_all0 = job->rgb_ev[0];
    e_all1 = job->rgb_ev[1];
    e_map0 = job->rgb_ev[2];
    e_map1 = job->rgb_ev[3];
    MR_HIP(hipGraphLaunch(job->rgb_graph, s));
  } else {
    MR_HIP(hipEventRecord(e_all0, s));
    MR_HIP(rgb_enqueue(static_cast<const uint8_t*>(d_input), bytes, partials, G, bins, s,
                       job->cfg.timing ? e_map0 : nullptr, job->cfg.timing ? e_map1 : nullptr));
    MR_HIP(hipEventRecord(e_all1, s));
  }
  MR_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, e_all0, e_all1));
  if (job->cfg.timing) MR_HIP(hipEventElapsedTime(&out->stats.map_ms, e_map0, e_map1));
  out->n_keys = 768;
  out->key_bytes_used = 0;
  out->stats.strategy_used = MR_STRAT_LDS_ARRAY;
  out->stats.n_items = bytes / 3;
  out->stats.gpu_ms = ms;
  return MR_OK;
}

// ---------------------------------------------------------------------------
// integer keys
// ---------------------------------------------------------------------------

constexpr uint64_t kLdsArrayBudget = 64 * 1024;   // LDS bytes a workgroup may give to a private array
constexpr uint64_t kIntSlotBytes = 4 + 4 + 8 + 4;  // integer hash table: key, count, value, claimed list
constexpr uint64_t kGlobalArrayMax = 1ull << 27;  // largest declared range for the global array

// Small per-run state block (device): flags, counters, side slot.
struct IntSmall {
  uint32_t flags;
  uint32_t side_cnt;
  unsigned long long side_val;
  unsigned long long n_claimed;
  unsigned long long n_out;
  int32_t choice;  // learned container choice (-1: use the rule)
  int32_t pad;
};

// Region `id` of at least `bytes` bytes; a new one is filled with the byte
// `fill` when fill >= 0. *fresh (optional) tells whether it is new.
mr_status int_ensure(mr_job* job, int id, void** p, uint64_t* have, uint64_t bytes, int fill, bool* fresh_out = nullptr) {
  bool fresh = false;
  mr_status st = dev_region(job, id, p, have, bytes, bytes, &fresh);
  if (st != MR_OK) return st;
  if (fresh && fill >= 0) MR_HIP(hipMemsetAsync(*p, fill, bytes, job->stream));
  if (fresh_out) *fresh_out = fresh;
  return MR_OK;
}

// The LDS budget of the rule's per-workgroup arrays: the tuned one, at most the default.
uint64_t eff_lds_array_bytes(const mr_job* job, mr_map_kind kind, uint64_t bytes) {
  const mr_tune_entry* t = tune_for(job, kind, bytes);
  return t && t->lds_array_bytes ? std::min<uint64_t>(t->lds_array_bytes, kLdsArrayBudget) : kLdsArrayBudget;
}

bool int_feasible(mr_strategy s, uint64_t R, uint32_t op, uint64_t lds_budget = kLdsArrayBudget) {
  switch (s) {
    case MR_STRAT_LDS_ARRAY: return R > 0 && int_lds_array_bytes(R, op) <= lds_budget;
    case MR_STRAT_GLOBAL_ARRAY: return R > 0 && R <= kGlobalArrayMax;
    case MR_STRAT_HASH:
    case MR_STRAT_SORT: return true;
    default: return false;
  }
}

// The paper's rule (Section III-E) for integer keys: keep per-worker arrays
// while each fits the local memory budget, otherwise one shared array with
// atomics; keys without a fixed range use the hash table. It never picks SORT.
mr_strategy rule_strategy(uint64_t R, uint32_t op, uint64_t lds_budget) {
  if (int_feasible(MR_STRAT_LDS_ARRAY, R, op, lds_budget)) return MR_STRAT_LDS_ARRAY;
  if (int_feasible(MR_STRAT_GLOBAL_ARRAY, R, op)) return MR_STRAT_GLOBAL_ARRAY;
  return MR_STRAT_HASH;
}

mr_status learned_strategy(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input, uint64_t bytes,
                           uint64_t R, mr_strategy* s, bool* used);

// Result sizes and status of an integer job from its state block.
mr_status u32_finish(mr_job* job, mr_output* out, const IntSmall& hs) {
  out->n_keys = hs.n_out;
  out->key_bytes_used = 0;
  job->int_last_distinct = hs.n_out;
  if (hs.flags & kFlagBadInput) return fail(MR_ERR_INVALID_ARG, "a key is outside the declared key_range");
  if (hs.n_out > out->cap_keys) return fail(MR_ERR_CAPACITY, "output needs %llu keys", (unsigned long long)hs.n_out);
  return MR_OK;
}

// Scratch layouts of the integer-key containers (offsets in the scratch region).
struct DenseCarve {  // LDS or global array over n elements and range R, G workgroups
  uint64_t o_blk = 0, o_cp = 0, o_vp = 0, o_ph = 0, o_pk = 0, bytes = 0;
  bool parts = false;  // a large COUNT array filled by key-range partitions
  PartPlan pp;
};
DenseCarve dense_carve(mr_strategy strat, uint64_t n, uint64_t R, uint32_t op, uint32_t G) {
  DenseCarve d;
  Carve c;
  const uint64_t nb = (R + 2047) / 2048;
  d.o_blk = c.take(4 * (nb + 1));
  if (strat == MR_STRAT_LDS_ARRAY) {
    d.o_cp = c.take(4ull * G * R);
    d.o_vp = c.take((op == MR_REDUCE_SUM ? 8ull : 4ull) * G * R);
  }
  // a large array counted by key-range partitions instead of atomics
  d.pp = part_plan(n, R);
  d.parts = strat == MR_STRAT_GLOBAL_ARRAY && op == MR_REDUCE_COUNT && d.pp.usable;
  if (d.parts) {
    d.o_ph = c.take(4 * d.pp.runs);
    d.o_pk = c.take(2 * d.pp.part_elems);
  }
  d.bytes = c.off;
  return d;
}
struct HashCarve {  // output records and radix sort of nc claimed keys
  uint64_t o_rk32, o_rk0, o_rv0, o_rk1, o_rv1, o_hist, o_ss, bytes;
};
HashCarve hash_carve(uint64_t nc) {
  HashCarve h;
  Carve c;
  const uint64_t hn = 256 * std::max<uint64_t>((nc + 2047) / 2048, 1);
  h.o_rk32 = c.take(4 * (nc + 1));
  h.o_rk0 = c.take(8 * (nc + 1));
  h.o_rv0 = c.take(8 * (nc + 1));
  h.o_rk1 = c.take(8 * (nc + 1));
  h.o_rv1 = c.take(8 * (nc + 1));
  h.o_hist = c.take(4 * hn);
  h.o_ss = c.take(4 * (hn / 4096 + 2));
  h.bytes = c.off;
  return h;
}
struct SortCarve {  // radix sort of all n pairs and the segmented reduce
  uint64_t o_rk0, o_rv0, o_rk1, o_rv1, o_hist, o_ss, o_head, o_pos, o_hpos, o_ps, bytes;
};
SortCarve sort_carve(uint64_t n) {
  SortCarve s;
  Carve c;
  const uint64_t hn = 256 * std::max<uint64_t>((n + 2047) / 2048, 1);
  s.o_rk0 = c.take(8 * (n + 1));
  s.o_rv0 = c.take(8 * (n + 1));
  s.o_rk1 = c.take(8 * (n + 1));
  s.o_rv1 = c.take(8 * (n + 1));
  s.o_hist = c.take(4 * hn);
  s.o_ss = c.take(4 * (std::max(hn, n) / 4096 + 2));
  s.o_head = c.take(4 * (n + 1));
  s.o_pos = c.take(4 * (n + 1));
  s.o_hpos = c.take(4 * (n + 2));
  s.o_ps = c.take(8 * (n / 4096 + 2));
  s.bytes = c.off;
  return s;
}
// Initial slots of the integer hash table for n elements and range R.
uint64_t int_table_slots(const mr_job* job, mr_map_kind kind, uint64_t bytes, uint64_t n, uint64_t R) {
  if (job->cfg.table_slots) return job->cfg.table_slots;
  const uint64_t bound = std::max<uint64_t>(1, R ? std::min<uint64_t>(n, R) : n);
  const double lf = eff_load_pct(job, kind, bytes) / 100.0;
  return std::max<uint64_t>(4096, next_pow2((uint64_t)std::ceil(std::min<uint64_t>(bound, 1ull << 24) / lf)));
}

// A batched integer item: the batch decides the container, gives the item
// its own state slot and reads the states back once for all items.
struct U32Ctx {
  mr_strategy strat;   // the container to run
  bool sel_used;       // the learned selector chose it
  IntSmall* sm;        // this item's state (device)
};

mr_status run_u32(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input, uint64_t bytes, uint64_t key_range,
                  mr_output* out, const U32Ctx* ctx = nullptr) {
  const uint32_t esz = kind == MR_MAP_U32_KV ? 8 : 4;
  if (bytes % esz) return fail(MR_ERR_INVALID_ARG, "input length %llu is not a multiple of %u", (unsigned long long)bytes, esz);
  if (kind == MR_MAP_U32_KEYS && op != MR_REDUCE_COUNT) return fail(MR_ERR_UNSUPPORTED, "plain keys support COUNT only");
  if (op < MR_REDUCE_COUNT || op > MR_REDUCE_MAX) return fail(MR_ERR_INVALID_ARG, "unknown reduce op");
  const uint64_t n = bytes / esz;
  if (n >= (1ull << 32)) return fail(MR_ERR_UNSUPPORTED, "integer inputs must have fewer than 2^32 elements");
  if (key_range > (1ull << 32)) return fail(MR_ERR_INVALID_ARG, "key_range above 2^32");
  if (out->cap_keys && (!out->keys || !out->values)) return fail(MR_ERR_INVALID_ARG, "output capacity given without buffers");
  if ((uintptr_t)d_input % 4) return fail(MR_ERR_INVALID_ARG, "integer input must be 4-byte aligned");
  const uint32_t o = (uint32_t)op;

  mr_strategy strat = ctx ? ctx->strat : job->cfg.strategy;
  bool sel_used = ctx ? ctx->sel_used : false;
  if (strat == MR_STRAT_LEARNED) {
    mr_status st = learned_strategy(job, kind, op, d_input, bytes, key_range, &strat, &sel_used);
    if (st != MR_OK) return st;
  }
  if (strat == MR_STRAT_RULE) strat = rule_strategy(key_range, o, eff_lds_array_bytes(job, kind, bytes));
  if (!int_feasible(strat, key_range, o))
    return fail(MR_ERR_UNSUPPORTED, "strategy %d is infeasible for this job (key_range %llu)", (int)strat,
                (unsigned long long)key_range);

  mr_status st = MR_OK;
  IntSmall* sm = ctx ? ctx->sm : nullptr;
  if (!sm) {
    st = int_ensure(job, kRegSmall, &job->int_small, &job->int_small_bytes, sizeof(IntSmall), 0);
    if (st != MR_OK) return st;
    sm = static_cast<IntSmall*>(job->int_small);
  }

  IntLaunch L{};
  L.in = static_cast<const uint32_t*>(d_input);
  L.n = n;
  L.kv = kind == MR_MAP_U32_KV;
  L.op = o;
  L.R = key_range;
  L.debug_hash = job->cfg.debug_hash;
  L.flags = &sm->flags;
  L.n_claimed = &sm->n_claimed;
  L.n_out = &sm->n_out;
  L.side_cnt = &sm->side_cnt;
  L.side_val = &sm->side_val;
  L.out_keys = static_cast<uint32_t*>(out->keys);
  L.out_vals = out->values;
  L.cap = out->cap_keys;
  L.G = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)job->n_cu * 2, (n + 1023) / 1024));

  auto scratch = [&](uint64_t bytes_needed) -> mr_status {
    return int_ensure(job, kRegScratch, &job->int_scratch, &job->int_scratch_bytes, bytes_needed, -1);
  };
  uint32_t retries = 0;
  uint64_t table_cap = 0;
  {
    const hipError_t e = hipMemsetAsync(sm, 0, sizeof(IntSmall), job->stream);
    if (e != hipSuccess) {
      hipPointerAttribute_t at{};
      const hipError_t ea = hipPointerGetAttributes(&at, sm);
      return fail(MR_ERR_HIP, "hipMemsetAsync(state %p, %zu) on stream %p: %s (pointer query: %s, type %d)", (void*)sm,
                  sizeof(IntSmall), (void*)job->stream, hipGetErrorString(e), hipGetErrorString(ea), (int)at.type);
    }
  }
  if (!ctx) MR_HIP(hipEventRecord(job->ev0, job->stream));

  if (strat == MR_STRAT_LDS_ARRAY || strat == MR_STRAT_GLOBAL_ARRAY) {
    // counts [R] then, 8-byte aligned, values [R]: 12 bytes per key plus alignment
    // a new region (or a larger R) starts all zero; the output pass clears what it reads
    bool dense_fresh = false;
    st = int_ensure(job, kRegDense, &job->int_dense, &job->int_dense_bytes, key_range * 12 + 8, 0, &dense_fresh);
    if (st != MR_OK) return st;
    // the layout's R: a kept region was laid out for an R at least this large
    if (dense_fresh) job->int_dense_R = key_range;
    L.dcnt = static_cast<uint32_t*>(job->int_dense);
    L.dval = static_cast<uint8_t*>(job->int_dense) + ((4 * job->int_dense_R + 7) & ~7ull);
    const DenseCarve dc = dense_carve(strat, n, key_range, o, L.G);
    const PartPlan& pp = dc.pp;
    const bool parts = dc.parts;
    const uint64_t o_blk = dc.o_blk, o_cp = dc.o_cp, o_vp = dc.o_vp, o_ph = dc.o_ph, o_pk = dc.o_pk;
    st = scratch(dc.bytes);
    if (st != MR_OK) return st;
    uint8_t* sc = static_cast<uint8_t*>(job->int_scratch);
    L.blk = reinterpret_cast<uint32_t*>(sc + o_blk);
    if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev2, job->stream));
    if (strat == MR_STRAT_LDS_ARRAY) {
      L.cnt_part = reinterpret_cast<uint32_t*>(sc + o_cp);
      L.val_part = sc + o_vp;
      MR_HIP(int_enqueue_lds_array(L, job->stream));
    } else if (parts) {
      MR_HIP(int_enqueue_global_array_tiles(L, pp, reinterpret_cast<uint32_t*>(sc + o_ph), reinterpret_cast<uint16_t*>(sc + o_pk),
                                            job->stream));
    } else {
      MR_HIP(int_enqueue_global_array(L, job->stream));
    }
    if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev3, job->stream));
    MR_HIP(int_enqueue_dense_out(L, true, parts, job->stream));
  } else if (strat == MR_STRAT_HASH) {
    // capacity: distinct <= min(n, range); start from the last job's distinct count when larger inputs repeat
    table_cap = int_table_slots(job, kind, bytes, n, key_range);
    for (;;) {
      {
        // a new table region is laid out for table_cap slots: keys start as
        // 0xFFFFFFFF, counts and values as 0 (a kept one is clean as a whole)
        bool fresh = false;
        st = dev_region(job, kRegTable, &job->int_table, &job->int_table_bytes, table_cap * kIntSlotBytes,
                        table_cap * kIntSlotBytes, &fresh);
        if (st != MR_OK) return st;
        if (fresh) {
          job->int_table_cap = table_cap;
          MR_HIP(hipMemsetAsync(job->int_table, 0xFF, table_cap * 4, job->stream));
          MR_HIP(hipMemsetAsync(static_cast<uint8_t*>(job->int_table) + table_cap * 4, 0, table_cap * 16, job->stream));
        }
      }
      uint8_t* tb = static_cast<uint8_t*>(job->int_table);
      const uint64_t C = job->int_table_cap;
      L.t_keys = reinterpret_cast<uint32_t*>(tb);
      L.t_cnt = reinterpret_cast<uint32_t*>(tb + 4 * C);
      L.t_val = tb + 8 * C;
      L.claimed = reinterpret_cast<uint32_t*>(tb + 16 * C);
      L.t_cap = table_cap;  // use a prefix of the allocation (kept clean as a whole)
      if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev2, job->stream));
      MR_HIP(int_enqueue_hash_map(L, job->stream));
      if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev3, job->stream));
      IntSmall hs;
      MR_HIP(hipMemcpyAsync(&hs, sm, sizeof hs, hipMemcpyDeviceToHost, job->stream));
      MR_HIP(hipStreamSynchronize(job->stream));
      const uint64_t nc = hs.n_claimed;
      // records and sort scratch for nc keys
      const HashCarve hc = hash_carve(nc);
      const uint64_t o_rk32 = hc.o_rk32, o_rk0 = hc.o_rk0, o_rv0 = hc.o_rv0, o_rk1 = hc.o_rk1, o_rv1 = hc.o_rv1,
                     o_hist = hc.o_hist, o_ss = hc.o_ss;
      st = scratch(hc.bytes);
      if (st != MR_OK) return st;
      uint8_t* sc = static_cast<uint8_t*>(job->int_scratch);
      L.rk32 = reinterpret_cast<uint32_t*>(sc + o_rk32);
      L.rk0 = reinterpret_cast<unsigned long long*>(sc + o_rk0);
      L.rv0 = reinterpret_cast<unsigned long long*>(sc + o_rv0);
      L.rk1 = reinterpret_cast<unsigned long long*>(sc + o_rk1);
      L.rv1 = reinterpret_cast<unsigned long long*>(sc + o_rv1);
      L.hist = reinterpret_cast<uint32_t*>(sc + o_hist);
      L.scan_sums = reinterpret_cast<uint32_t*>(sc + o_ss);
      MR_HIP(int_enqueue_hash_out(L, nc, job->stream));  // gathers and clears the claimed slots
      if (hs.flags & kFlagTableFull) {
        if (++retries > 24 || table_cap >= (1ull << 31)) return fail(MR_ERR_CAPACITY, "hash table cannot grow further");
        table_cap *= 2;
        MR_HIP(hipMemsetAsync(sm, 0, sizeof(IntSmall), job->stream));
        continue;
      }
      MR_HIP(int_enqueue_hash_sort_out(L, nc, job->stream));
      break;
    }
  } else {  // SORT
    const SortCarve sc_ = sort_carve(n);
    const uint64_t o_rk0 = sc_.o_rk0, o_rv0 = sc_.o_rv0, o_rk1 = sc_.o_rk1, o_rv1 = sc_.o_rv1, o_hist = sc_.o_hist,
                   o_ss = sc_.o_ss, o_head = sc_.o_head, o_pos = sc_.o_pos, o_hpos = sc_.o_hpos, o_ps = sc_.o_ps;
    st = scratch(sc_.bytes);
    if (st != MR_OK) return st;
    uint8_t* sc = static_cast<uint8_t*>(job->int_scratch);
    L.rk0 = reinterpret_cast<unsigned long long*>(sc + o_rk0);
    L.rv0 = reinterpret_cast<unsigned long long*>(sc + o_rv0);
    L.rk1 = reinterpret_cast<unsigned long long*>(sc + o_rk1);
    L.rv1 = reinterpret_cast<unsigned long long*>(sc + o_rv1);
    L.hist = reinterpret_cast<uint32_t*>(sc + o_hist);
    L.scan_sums = reinterpret_cast<uint32_t*>(sc + o_ss);
    L.head = reinterpret_cast<uint32_t*>(sc + o_head);
    L.pos = reinterpret_cast<uint32_t*>(sc + o_pos);
    L.hpos = reinterpret_cast<uint32_t*>(sc + o_hpos);
    L.ps_sums = reinterpret_cast<unsigned long long*>(sc + o_ps);
    if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev2, job->stream));
    MR_HIP(int_enqueue_sort(L, job->stream));
    if (job->cfg.timing) MR_HIP(hipEventRecord(job->ev3, job->stream));
  }
  out->stats.strategy_used = strat;
  out->stats.selector_used = sel_used ? 1u : 0u;
  out->stats.retries = retries;
  out->stats.table_slots = table_cap;
  out->stats.n_items = n;
  if (ctx) return MR_OK;  // the batch reads the state back
  MR_HIP(hipEventRecord(job->ev1, job->stream));
  IntSmall hs;
  MR_HIP(hipMemcpyAsync(&hs, sm, sizeof hs, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, job->ev0, job->ev1));
  out->stats.gpu_ms = ms;
  if (job->cfg.timing) MR_HIP(hipEventElapsedTime(&out->stats.map_ms, job->ev2, job->ev3));
  return u32_finish(job, out, hs);
}


// k-means scratch: centroid norms, the float64 re-check bound, the re-check
// and tiny-coordinate counters, per-workgroup float64 sums and counts.
struct KmCarve {
  uint64_t o_cn, o_cmax, o_nr, o_ps, o_pc, bytes;
};
KmCarve km_carve(uint32_t k, uint32_t d, uint32_t G) {
  KmCarve r;
  Carve c;
  r.o_cn = c.take(4ull * k);
  r.o_cmax = c.take(8);
  r.o_nr = c.take(16);
  r.o_ps = c.take(8ull * G * k * d);
  r.o_pc = c.take(4ull * G * k);
  r.bytes = c.off;
  return r;
}
uint32_t km_grid(uint64_t N, int n_cu, bool mfma) {
  return mfma ? (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)n_cu * 3, (N + 127) / 128)) : 1u;
}

mr_status run_kmeans(mr_job* job, const void* d_input, uint64_t bytes, mr_output* out) {
  const uint32_t k = job->cfg.km_k, d = job->cfg.km_d;
  if (job->km_host.empty() || !k || !d) return fail(MR_ERR_INVALID_ARG, "the job was created without k-means centroids");
  if (bytes % (4ull * d)) return fail(MR_ERR_INVALID_ARG, "input length is not a multiple of 4 * d");
  const uint64_t N = bytes / (4ull * d);
  if (N >= (1ull << 31)) return fail(MR_ERR_UNSUPPORTED, "k-means inputs must have fewer than 2^31 points");
  if ((N && !out->assign) || !out->sums || !out->counts || !out->centroids)
    return fail(MR_ERR_INVALID_ARG, "k-means needs assign, sums, counts and centroids outputs");
  if ((uintptr_t)d_input % 4) return fail(MR_ERR_INVALID_ARG, "points must be 4-byte aligned");
  {
    bool fresh = false;
    void* p = job->km_c;
    const uint64_t cb = sizeof(float) * job->km_host.size();
    mr_status st = dev_region(job, kRegKmC, &p, &job->km_c_bytes, cb, cb, &fresh);
    if (st != MR_OK) return st;
    job->km_c = static_cast<float*>(p);
    if (fresh) MR_HIP(hipMemcpyAsync(job->km_c, job->km_host.data(), cb, hipMemcpyHostToDevice, job->stream));
  }
  KmLaunch L{};
  L.X = static_cast<const float*>(d_input);
  L.N = N;
  L.C = job->km_c;
  L.k = k;
  L.d = d;
  L.mfma = d == 32 && k == 64 && (uintptr_t)d_input % 16 == 0;
  L.G = km_grid(N, job->n_cu, L.mfma);
  const KmCarve kc = km_carve(k, d, L.G);
  const uint64_t o_cn = kc.o_cn, o_cmax = kc.o_cmax, o_nr = kc.o_nr, o_ps = kc.o_ps, o_pc = kc.o_pc;
  mr_status st = ensure_ws(job, kc.bytes);
  if (st != MR_OK) return st;
  job->table_clean_bytes = 0;  // this scratch overwrites the word table region
  job->graph_valid = false;
  uint8_t* ws = job->ws;
  L.cn = reinterpret_cast<float*>(ws + o_cn);
  L.cmax = reinterpret_cast<double*>(ws + o_cmax);
  L.n_recheck = reinterpret_cast<unsigned long long*>(ws + o_nr);
  L.tiny = L.n_recheck + 1;
  L.part_sum = reinterpret_cast<double*>(ws + o_ps);
  L.part_cnt = reinterpret_cast<uint32_t*>(ws + o_pc);
  L.assign = out->assign;
  L.sums = out->sums;
  L.counts = out->counts;
  L.cent = out->centroids;
  unsigned long long flags[2] = {0, 0};  // rechecks, tiny
  for (int pass = 0; pass < 2; ++pass) {
    MR_HIP(hipMemsetAsync(L.n_recheck, 0, 16, job->stream));
    MR_HIP(hipEventRecord(job->ev0, job->stream));
    MR_HIP(km_enqueue(L, job->stream, job->cfg.timing ? job->ev2 : nullptr, job->cfg.timing ? job->ev3 : nullptr));
    MR_HIP(hipEventRecord(job->ev1, job->stream));
    MR_HIP(hipMemcpyAsync(flags, L.n_recheck, 16, hipMemcpyDeviceToHost, job->stream));
    MR_HIP(hipStreamSynchronize(job->stream));
    // coordinates too small for the matrix-core path's exact split: the
    // generic kernel redoes the step (it writes every output again)
    if (!L.mfma || !flags[1]) break;
    L.mfma = false;
    L.G = 1;
  }
  const unsigned long long nr = flags[0];
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, job->ev0, job->ev1));
  out->stats.gpu_ms = ms;
  if (job->cfg.timing) MR_HIP(hipEventElapsedTime(&out->stats.map_ms, job->ev2, job->ev3));
  out->stats.n_items = N;
  out->stats.km_rechecked = (uint32_t)nr;
  out->stats.strategy_used = L.mfma ? 1u : 0u;
  out->n_keys = k;
  return MR_OK;
}

// Bloom filter scratch: per (range, tile) counts, their scan, the total, the positions.
struct BloomCarve {
  uint64_t o_hist, o_sums, o_tot, o_part, bytes;
};
BloomCarve bloom_carve(const BloomPlan& b) {
  BloomCarve r;
  Carve c;
  r.o_hist = c.take(4ull * std::max<uint64_t>(b.H, 1));
  r.o_sums = c.take(4ull * scan_sums_count(b.H));
  r.o_tot = c.take(8);
  r.o_part = c.take(4ull * b.part_words);
  r.bytes = c.off;
  return r;
}

mr_status run_bloom(mr_job* job, mr_reduce_op op, const void* d_input, uint64_t bytes, uint64_t m, mr_output* out) {
  if (op != MR_REDUCE_COUNT) return fail(MR_ERR_UNSUPPORTED, "the Bloom filter takes MR_REDUCE_COUNT (bitwise OR)");
  const uint32_t k = job->cfg.bloom_k ? job->cfg.bloom_k : 20u;
  const uint32_t h = job->cfg.bloom_hashes ? job->cfg.bloom_hashes : 7u;
  if (k > 32 || h > 8) return fail(MR_ERR_INVALID_ARG, "Bloom filter k-mer length %u (1..32) or hash count %u (1..8)", k, h);
  if (m == 0) return fail(MR_ERR_INVALID_ARG, "the Bloom filter needs its size in bits as key_range");
  if (m > (1ull << 29)) return fail(MR_ERR_UNSUPPORTED, "Bloom filters of more than 2^29 bits are not supported");
  const BloomPlan b = bloom_plan(bytes, k, h, m);
  if (!b.ok) return fail(MR_ERR_UNSUPPORTED, "Bloom filter input too large (%llu positions)", (unsigned long long)b.max_entries);
  out->n_keys = b.n_words;
  out->key_bytes_used = 0;
  if (!out->values) return fail(MR_ERR_INVALID_ARG, "the Bloom filter needs values (uint32 words)");
  if (out->cap_keys < b.n_words)
    return fail(MR_ERR_CAPACITY, "the Bloom filter needs %llu words", (unsigned long long)b.n_words);
  const BloomCarve bc = bloom_carve(b);
  const uint64_t o_hist = bc.o_hist, o_sums = bc.o_sums, o_tot = bc.o_tot, o_part = bc.o_part;
  mr_status st = ensure_ws(job, bc.bytes);
  if (st != MR_OK) return st;
  job->table_clean_bytes = 0;  // this scratch overwrites the word table region
  job->graph_valid = false;
  uint8_t* ws = job->ws;
  MR_HIP(hipEventRecord(job->ev0, job->stream));
  MR_HIP(bloom_enqueue(static_cast<const uint8_t*>(d_input), bytes, k, h, m, b, reinterpret_cast<uint32_t*>(ws + o_hist),
                       reinterpret_cast<uint32_t*>(ws + o_sums), reinterpret_cast<unsigned long long*>(ws + o_tot),
                       reinterpret_cast<uint32_t*>(ws + o_part), static_cast<uint32_t*>(out->values), job->stream));
  MR_HIP(hipEventRecord(job->ev1, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, job->ev0, job->ev1));
  out->stats.gpu_ms = ms;
  out->stats.n_items = b.n_kmers;
  out->stats.strategy_used = MR_STRAT_GLOBAL_ARRAY;
  return MR_OK;
}

}  // namespace

// ----------------------------------------------------------------------------
// entry points
// ----------------------------------------------------------------------------

extern "C" mr_status mr_run(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input, uint64_t input_bytes,
                            const uint64_t* d_record_offsets, uint64_t n_records, uint64_t key_range, mr_output* out) {
  if (!job || !out) return fail(MR_ERR_INVALID_ARG, "NULL job or output");
  if (input_bytes && !d_input) return fail(MR_ERR_INVALID_ARG, "NULL input");
  if (d_record_offsets && kind != MR_MAP_WORDS && kind != MR_MAP_LINKS)
    return fail(MR_ERR_INVALID_ARG, "record offsets are only meaningful for words and links");
  ScopedDevice sd(job->device);
  out->stats = mr_stats{};
  out->status = MR_OK;
  switch (kind) {
    case MR_MAP_WORDS: arena_begin(job, kFamWords); break;
    case MR_MAP_RGB_HIST: arena_begin(job, kFamRgb); break;
    case MR_MAP_KMEANS: arena_begin(job, kFamKmeans); break;
    case MR_MAP_BLOOM: arena_begin(job, kFamBloom); break;
    case MR_MAP_LINKS: arena_begin(job, kFamLinks); break;
    default: arena_begin(job, kFamU32); break;
  }
  mr_status s;
  switch (kind) {
    case MR_MAP_WORDS: {
      if (op != MR_REDUCE_COUNT) return fail(MR_ERR_UNSUPPORTED, "words support COUNT only");
      std::vector<WordItem> items(1);
      items[0] = WordItem{static_cast<const uint8_t*>(d_input), input_bytes, d_record_offsets, n_records, out, 0};
      s = run_words(job, items, nullptr, GraphMode::kOnRepeat);
      break;
    }
    case MR_MAP_RGB_HIST:
      if (op != MR_REDUCE_COUNT) return fail(MR_ERR_UNSUPPORTED, "the histogram supports COUNT only");
      s = run_rgb(job, d_input, input_bytes, out);
      break;
    case MR_MAP_U32_KEYS:
    case MR_MAP_U32_KV:
      s = run_u32(job, kind, op, d_input, input_bytes, key_range, out);
      break;
    case MR_MAP_KMEANS:
      s = run_kmeans(job, d_input, input_bytes, out);
      break;
    case MR_MAP_BLOOM:
      s = run_bloom(job, op, d_input, input_bytes, key_range, out);
      break;
    case MR_MAP_LINKS:
      s = run_links(job, op, d_input, input_bytes, d_record_offsets, n_records, out);
      break;
    default:
      return fail(MR_ERR_INVALID_ARG, "unknown map kind %d", (int)kind);
  }
  out->stats.device_allocs = job->call_allocs;
  out->stats.workspace_needed = job->cws_need;
  out->status = s;
  return s;
}

extern "C" mr_status mr_rgb_hist_static(mr_job* job, const void* d_input, uint64_t input_bytes, uint64_t* d_bins) {
  if (!job || !d_bins || (input_bytes && !d_input)) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  if (input_bytes % 3)
    return fail(MR_ERR_INVALID_ARG, "RGB input length %llu is not a multiple of 3", (unsigned long long)input_bytes);
  const uint32_t G = rgb_static_rows(input_bytes, job->n_cu);
  // each partial row counts fewer than 2^31 bytes in 32-bit counters
  if (input_bytes / G >= (1ull << 31))
    return fail(MR_ERR_UNSUPPORTED, "input of %llu bytes exceeds the static scratch (%u rows of 2^31 bytes)",
                (unsigned long long)input_bytes, kRgbStaticRows);
  ScopedDevice sd(job->device);
  const hipError_t e = rgb_static_enqueue(job->device, static_cast<const uint8_t*>(d_input), input_bytes, G,
                                          reinterpret_cast<unsigned long long*>(d_bins), job->stream);
  if (e != hipSuccess) return fail(MR_ERR_HIP, "mr_rgb_hist_static: %s", hipGetErrorString(e));
  return MR_OK;
}

namespace {

// Bytes of a sequence of regions carved as dev_region carves a caller workspace.
struct RegionSum {
  uint64_t off = 0;
  void add(uint64_t bytes) { off = align_up(off, 256) + bytes; }
};

}  // namespace

extern "C" mr_status mr_workspace_bytes(const mr_job_config* cfg, mr_map_kind kind, uint64_t n, uint64_t key_range,
                                        uint64_t* out_bytes) {
  if (!cfg || !out_bytes) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess || n_dev <= 0) return fail(MR_ERR_NO_DEVICE, "no HIP device");
  if (cfg->device < 0 || cfg->device >= n_dev) return fail(MR_ERR_INVALID_ARG, "device %d out of range", cfg->device);
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, cfg->device) != hipSuccess || n_cu <= 0)
    return fail(MR_ERR_NO_DEVICE, "device query failed");
  // a job with these settings (no device state) for the planning functions
  mr_job tmp;
  tmp.cfg = *cfg;
  tmp.n_cu = n_cu;
  RegionSum r;
  switch (kind) {
    case MR_MAP_WORDS: {
      // the input's alignment may add a 16-byte chunk: plan at the worst one
      std::vector<WordItem> items(1);
      items[0] = WordItem{reinterpret_cast<const uint8_t*>(15), n, nullptr, 0, nullptr, initial_slots(&tmp, n, n)};
      const uint64_t grid_cap = std::max<uint64_t>(1, (uint64_t)n_cu * eff_grid_pct(&tmp, n) / 100);
      r.add(plan_words(items, false, true, grid_cap).c.off);
      break;
    }
    case MR_MAP_RGB_HIST:
      r.add(4ull * 768 * rgb_grid(n, n_cu));
      break;
    case MR_MAP_KMEANS: {
      if (!cfg->km_k || !cfg->km_d) return fail(MR_ERR_INVALID_ARG, "k-means needs km_k and km_d");
      const uint64_t N = n / (4ull * cfg->km_d);
      r.add(4ull * cfg->km_k * cfg->km_d);
      r.add(km_carve(cfg->km_k, cfg->km_d, km_grid(N, n_cu, cfg->km_d == 32 && cfg->km_k == 64)).bytes);
      break;
    }
    case MR_MAP_BLOOM: {
      const uint32_t k = cfg->bloom_k ? cfg->bloom_k : 20u, h = cfg->bloom_hashes ? cfg->bloom_hashes : 7u;
      if (!key_range || key_range > (1ull << 29) || k > 32 || h > 8)
        return fail(MR_ERR_INVALID_ARG, "the Bloom filter needs 1 <= key_range <= 2^29 bits, k <= 32, hashes <= 8");
      const BloomPlan b = bloom_plan(n, k, h, key_range);
      r.add(bloom_carve(b).bytes);
      break;
    }
    case MR_MAP_U32_KEYS:
    case MR_MAP_U32_KV: {
      const uint32_t esz = kind == MR_MAP_U32_KV ? 8 : 4;
      const uint64_t ne = n / esz;
      // pairs are planned for SUM (the widest values), keys for COUNT
      const uint32_t op = kind == MR_MAP_U32_KV ? (uint32_t)MR_REDUCE_SUM : (uint32_t)MR_REDUCE_COUNT;
      const uint32_t G = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)n_cu * 2, (ne + 1023) / 1024));
      r.add(sizeof(IntSmall));
      std::vector<mr_strategy> cand;
      if (cfg->strategy == MR_STRAT_LEARNED) {
        r.add(4 * sel_floats());
        for (mr_strategy c : {MR_STRAT_LDS_ARRAY, MR_STRAT_GLOBAL_ARRAY, MR_STRAT_HASH, MR_STRAT_SORT})
          if (int_feasible(c, key_range, op)) cand.push_back(c);
      } else if (cfg->strategy == MR_STRAT_RULE) {
        cand.push_back(rule_strategy(key_range, op, eff_lds_array_bytes(&tmp, kind, n)));
      } else {
        cand.push_back(cfg->strategy);
      }
      uint64_t worst = 0;
      for (mr_strategy c : cand) {
        RegionSum t = r;
        if (c == MR_STRAT_LDS_ARRAY || c == MR_STRAT_GLOBAL_ARRAY) {
          t.add(key_range * 12 + 8);
          t.add(dense_carve(c, ne, key_range, op, G).bytes);
        } else if (c == MR_STRAT_HASH) {
          t.add(int_table_slots(&tmp, kind, n, ne, key_range) * kIntSlotBytes);
          t.add(hash_carve(key_range ? std::min(ne, key_range) : ne).bytes);
        } else {
          t.add(sort_carve(ne).bytes);
        }
        worst = std::max(worst, t.off);
      }
      r.off = worst;
      break;
    }
    case MR_MAP_LINKS: {
      const uint64_t cap = std::max<uint64_t>(4096, n / 512);
      Carve c;
      c.take(8);
      c.take(4 * cap);
      c.take(4 * cap);
      c.take(4 * cap);
      r.add(c.off);
      std::vector<WordItem> items(1);
      items[0] = WordItem{reinterpret_cast<const uint8_t*>(15), n, nullptr, 0, nullptr, initial_slots(&tmp, n, n)};
      const uint64_t grid_cap = std::max<uint64_t>(1, (uint64_t)n_cu * eff_grid_pct(&tmp, n) / 100);
      r.add(plan_words(items, true, false, grid_cap).c.off);
      // the file-list pass: at most one pair and one URL per marker
      const uint64_t hw = links_hist_words(cap);
      c.take(8 * cap);
      c.take(8 * cap);
      c.take(8 * cap);
      c.take(8 * cap);
      c.take(4 * std::max<uint64_t>(hw, 1));
      c.take(4 * std::max(scan_sums_count(hw), scan_sums_count(cap)));
      c.take(4 * cap);
      c.take(8);
      c.take(8);
      c.take(8);
      c.take(4 * (cap + 1));
      r.add(c.off);
      break;
    }
    default:
      return fail(MR_ERR_INVALID_ARG, "unknown map kind %d", (int)kind);
  }
  *out_bytes = r.off;
  return MR_OK;
}

extern "C" mr_status mr_tune_set(mr_job* job, const mr_tune_entry* entries, uint32_t n) {
  if (!job || (n && !entries)) return fail(MR_ERR_INVALID_ARG, "NULL job or entries");
  for (uint32_t i = 0; i < n; ++i) {
    const mr_tune_entry& e = entries[i];
    const bool kind_ok = e.kind == MR_MAP_WORDS || e.kind == MR_MAP_U32_KEYS || e.kind == MR_MAP_U32_KV;
    const bool lds_ok = e.lds_slots == 0 || e.lds_slots == 256 || e.lds_slots == 1024 || e.lds_slots == 2048 || e.lds_slots == 4096;
    if (!kind_ok || e.bytes_lo >= e.bytes_hi || !lds_ok || e.max_load_pct > 95 || e.map_grid_pct > 100 ||
        e.lds_array_bytes > kLdsArrayBudget)
      return fail(MR_ERR_INVALID_ARG, "tune entry %u is malformed", i);
  }
  job->tune.assign(entries, entries + n);
  job->graph_valid = false;
  return MR_OK;
}

namespace {
mr_status batch_ints_enqueue(mr_job* job, const mr_batch_item* items, const std::vector<uint32_t>& ii, mr_output* outs,
                             std::vector<mr_status>& per);
mr_status batch_ints_finish(mr_job* job, const std::vector<uint32_t>& ii, mr_output* outs, std::vector<mr_status>& per);
}  // namespace

extern "C" mr_status mr_batch_run(mr_job* job, const mr_batch_item* items, uint32_t n_items, mr_output* outs) {
  if (!job || (!items && n_items) || (!outs && n_items)) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  if (n_items == 0) return MR_OK;
  ScopedDevice sd(job->device);
  std::vector<WordItem> w;
  std::vector<uint32_t> wi, ii;
  for (uint32_t i = 0; i < n_items; ++i) {
    const mr_batch_item& it = items[i];
    if (it.kind == MR_MAP_WORDS && it.op == MR_REDUCE_COUNT) {
      wi.push_back(i);
    } else if (it.kind == MR_MAP_U32_KEYS || it.kind == MR_MAP_U32_KV) {
      if (it.d_record_offsets) return fail(MR_ERR_INVALID_ARG, "record offsets are only meaningful for words (item %u)", i);
      ii.push_back(i);
    } else {
      return fail(MR_ERR_UNSUPPORTED, "mr_batch_run takes word-count and integer-key items (item %u)", i);
    }
    outs[i].stats = mr_stats{};
    outs[i].status = MR_OK;
  }
  for (uint32_t i : wi)
    w.push_back(WordItem{static_cast<const uint8_t*>(items[i].d_input), items[i].input_bytes, items[i].d_record_offsets,
                         items[i].n_records, &outs[i], 0});
  std::vector<mr_status> per(n_items, MR_OK);
  arena_begin(job, ii.empty() ? kFamWords : kFamBatch);
  mr_status first = MR_OK;
  // integer items first: the selection graph, then their containers on the
  // stream; the word pass after them synchronises the stream once
  if (!ii.empty()) {
    first = batch_ints_enqueue(job, items, ii, outs, per);
    if (first != MR_OK) return first;
  }
  if (!w.empty()) {
    std::vector<mr_status> wper(w.size(), MR_OK);
    const mr_status st = run_words(job, w, &wper, GraphMode::kAlways);
    for (size_t k = 0; k < w.size(); ++k) per[wi[k]] = wper[k];
    if (st != MR_OK && st != MR_ERR_CAPACITY && st != MR_ERR_INVALID_ARG) return st;
  }
  if (!ii.empty()) {
    const mr_status st = batch_ints_finish(job, ii, outs, per);
    if (st != MR_OK) return st;
  }
  for (uint32_t i = 0; i < n_items; ++i) {
    outs[i].status = per[i];
    outs[i].stats.device_allocs = job->call_allocs;
    outs[i].stats.workspace_needed = job->cws_need;
    if (first == MR_OK && per[i] != MR_OK) first = per[i];
  }
  return first;
}

// ----------------------------------------------------------------------------
// reduce-strategy selector
// ----------------------------------------------------------------------------

namespace {

// Selector scratch (device floats): [0, 16) features, [16, 32) network input,
// [32, 48) network output, [64, 128) normalisation (mean, scale, lo, hi at
// +0, +16, +32, +48), [128, 128 + 5252) parameters.
constexpr uint64_t kSelNorm = 64;
constexpr uint64_t kSelParams = 128;
constexpr uint64_t kSelState = (kSelParams + MR_MLP_PARAMS + 63) / 64 * 64;  // feature sampling state (floats offset)

uint64_t sel_floats() { return kSelState + (feature_state_bytes() + 3) / 4; }

mr_status sel_scratch(mr_job* job, uint64_t floats) {
  bool fresh = false;
  mr_status st = int_ensure(job, kRegSel, &job->sel_dev, &job->sel_dev_bytes, 4 * floats, -1, &fresh);
  if (st != MR_OK) return st;
  if (fresh) job->sel_uploaded = false;
  return MR_OK;
}

// The selector region, with the loaded weights and normalisation in it.
mr_status sel_upload(mr_job* job) {
  mr_status st = sel_scratch(job, sel_floats());
  if (st != MR_OK) return st;
  if (!job->sel_loaded || job->sel_uploaded) return MR_OK;
  float* dv = static_cast<float*>(job->sel_dev);
  MR_HIP(hipMemcpyAsync(dv + kSelParams, job->sel_params.data(), 4 * MR_MLP_PARAMS, hipMemcpyHostToDevice, job->stream));
  MR_HIP(hipMemcpyAsync(dv + kSelNorm, job->sel_mean.data(), 4 * MR_N_FEATURES, hipMemcpyHostToDevice, job->stream));
  MR_HIP(hipMemcpyAsync(dv + kSelNorm + 16, job->sel_scale.data(), 4 * MR_N_FEATURES, hipMemcpyHostToDevice, job->stream));
  MR_HIP(hipMemcpyAsync(dv + kSelNorm + 32, job->sel_lo.data(), 4 * MR_N_FEATURES, hipMemcpyHostToDevice, job->stream));
  MR_HIP(hipMemcpyAsync(dv + kSelNorm + 48, job->sel_hi.data(), 4 * MR_N_FEATURES, hipMemcpyHostToDevice, job->stream));
  // the host vectors stay unchanged until the copies are done: the next
  // change of them (mr_selector_set) synchronises the stream first
  job->sel_uploaded = true;
  return MR_OK;
}

int feature_kind(mr_map_kind kind) {
  switch (kind) {
    case MR_MAP_WORDS: return 0;
    case MR_MAP_U32_KEYS: return 1;
    case MR_MAP_U32_KV: return 2;
    default: return -1;
  }
}

}  // namespace

extern "C" mr_status mr_job_features(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input,
                                     uint64_t input_bytes, uint64_t key_range, float* feats) {
  if (!job || !feats || (input_bytes && !d_input)) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  const int fk = feature_kind(kind);
  if (fk < 0) return fail(MR_ERR_UNSUPPORTED, "features exist for word and integer-key jobs");
  if (fk > 0 && (uintptr_t)d_input % 4) return fail(MR_ERR_INVALID_ARG, "integer input must be 4-byte aligned");
  ScopedDevice sd(job->device);
  arena_begin(job, kFamFeatures);
  mr_status st = sel_scratch(job, sel_floats());
  if (st != MR_OK) return st;
  float* d = static_cast<float*>(job->sel_dev);
  MR_HIP(features_enqueue(static_cast<const uint8_t*>(d_input), input_bytes, fk, (int)op, key_range,
                          (uint32_t)kLdsArrayBudget, d, d + kSelState, job->stream));
  MR_HIP(hipMemcpyAsync(feats, d, 4 * MR_N_FEATURES, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  return MR_OK;
}

extern "C" mr_status mr_selector_set(mr_job* job, const float* params, const float* feat_mean, const float* feat_scale,
                                     const float* feat_lo, const float* feat_hi) {
  if (!job) return fail(MR_ERR_INVALID_ARG, "NULL job");
  if (!params) {
    job->sel_loaded = false;
    return MR_OK;
  }
  if (!feat_mean || !feat_scale || !feat_lo || !feat_hi) return fail(MR_ERR_INVALID_ARG, "NULL normalisation");
  for (int i = 0; i < MR_N_FEATURES; ++i)
    if (!(feat_scale[i] > 0.f)) return fail(MR_ERR_INVALID_ARG, "feature scale %d must be positive", i);
  ScopedDevice sd(job->device);
  MR_HIP(hipStreamSynchronize(job->stream));  // no copy of the previous weights is still reading them
  job->sel_params.assign(params, params + MR_MLP_PARAMS);
  job->sel_mean.assign(feat_mean, feat_mean + MR_N_FEATURES);
  job->sel_scale.assign(feat_scale, feat_scale + MR_N_FEATURES);
  job->sel_lo.assign(feat_lo, feat_lo + MR_N_FEATURES);
  job->sel_hi.assign(feat_hi, feat_hi + MR_N_FEATURES);
  job->sel_loaded = true;
  job->sel_uploaded = false;  // copied to the device by the first call that uses them
  return MR_OK;
}

namespace {

// Top-level members of a JSON object whose values are numbers or arrays of
// numbers (other members are parsed and skipped). Enough for the selector
// weights file; returns false on malformed text.
struct JsonNumbers {
  const char* p;
  const char* end;
  std::unordered_map<std::string, std::vector<double>> arrays;
  void ws() {
    while (p < end && (*p == ' ' || *p == '\n' || *p == '\r' || *p == '\t')) ++p;
  }
  bool str(std::string* out) {
    if (p >= end || *p != '"') return false;
    ++p;
    while (p < end && *p != '"') {
      if (*p == '\\') {
        if (++p >= end) return false;
      }
      if (out) out->push_back(*p);
      ++p;
    }
    if (p >= end) return false;
    ++p;
    return true;
  }
  bool number(double* v) {
    char* e = nullptr;
    const double x = std::strtod(p, &e);
    if (e == p || e > end) return false;
    p = e;
    if (v) *v = x;
    return true;
  }
  bool value(std::vector<double>* nums, int depth) {
    ws();
    if (p >= end || depth > 64) return false;
    if (*p == '{') {
      ++p;
      ws();
      if (p < end && *p == '}') return ++p, true;
      for (;;) {
        ws();
        std::string key;
        if (!str(&key)) return false;
        ws();
        if (p >= end || *p != ':') return false;
        ++p;
        std::vector<double> v;
        const bool top = depth == 0;
        if (!value(top ? &v : nullptr, depth + 1)) return false;
        if (top && !v.empty()) arrays[key] = std::move(v);
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == '}') return ++p, true;
        return false;
      }
    }
    if (*p == '[') {
      ++p;
      ws();
      if (p < end && *p == ']') return ++p, true;
      for (;;) {
        ws();
        if (p < end && (*p == '-' || (*p >= '0' && *p <= '9'))) {
          double x;
          if (!number(&x)) return false;
          if (nums) nums->push_back(x);
        } else if (!value(nullptr, depth + 1)) {
          return false;
        } else if (nums) {
          nums = nullptr;  // not an array of numbers: not kept
        }
        ws();
        if (p < end && *p == ',') { ++p; continue; }
        if (p < end && *p == ']') return ++p, true;
        return false;
      }
    }
    if (*p == '"') return str(nullptr);
    if (*p == '-' || (*p >= '0' && *p <= '9')) {
      double x;
      if (!number(&x)) return false;
      if (nums) nums->push_back(x);
      return true;
    }
    for (const char* w : {"true", "false", "null"}) {
      const size_t n = std::strlen(w);
      if ((size_t)(end - p) >= n && std::strncmp(p, w, n) == 0) return p += n, true;
    }
    return false;
  }
};

}  // namespace

extern "C" mr_status mr_selector_load(mr_job* job, const char* path) {
  if (!job || !path) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(MR_ERR_INVALID_ARG, "cannot open selector weights %s", path);
  std::string text;
  char buf[65536];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
  std::fclose(f);
  JsonNumbers j{text.c_str(), text.c_str() + text.size(), {}};
  if (!j.value(nullptr, 0)) return fail(MR_ERR_INVALID_ARG, "selector weights %s: malformed JSON", path);
  struct Need {
    const char* key;
    size_t n;
  };
  const Need need[] = {{"params", MR_MLP_PARAMS}, {"feat_mean", MR_N_FEATURES}, {"feat_scale", MR_N_FEATURES},
                       {"feat_lo", MR_N_FEATURES}, {"feat_hi", MR_N_FEATURES}};
  std::vector<float> a[5];
  for (int i = 0; i < 5; ++i) {
    auto it = j.arrays.find(need[i].key);
    if (it == j.arrays.end() || it->second.size() != need[i].n)
      return fail(MR_ERR_INVALID_ARG, "selector weights %s: \"%s\" must be %zu numbers", path, need[i].key, need[i].n);
    a[i].assign(it->second.begin(), it->second.end());
  }
  return mr_selector_set(job, a[0].data(), a[1].data(), a[2].data(), a[3].data(), a[4].data());
}

// Network output for host features, computed by the forward kernel (batch of one).
extern "C" mr_status mr_selector_predict(mr_job* job, const float* feats, float* pred) {
  if (!job || !feats || !pred) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  if (!job->sel_loaded) return fail(MR_ERR_INVALID_ARG, "no selector weights are loaded");
  ScopedDevice sd(job->device);
  arena_begin(job, kFamPredict);
  mr_status st = sel_upload(job);
  if (st != MR_OK) return st;
  float x[16];
  for (int i = 0; i < MR_N_FEATURES; ++i) x[i] = (feats[i] - job->sel_mean[i]) / job->sel_scale[i];
  float* d = static_cast<float*>(job->sel_dev);
  MR_HIP(hipMemcpyAsync(d + 16, x, 4 * MR_N_FEATURES, hipMemcpyHostToDevice, job->stream));
  MR_HIP(mlp_forward_enqueue(d + kSelParams, d + 16, 1, nullptr, nullptr, d + 32, job->stream));
  MR_HIP(hipMemcpyAsync(pred, d + 32, 4 * MR_N_STRATS, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  return MR_OK;
}

namespace {

// Features, normalisation, network and argmin over the feasible containers
// all run on the device; the choice comes back in the job's small state block.
mr_status learned_strategy(mr_job* job, mr_map_kind kind, mr_reduce_op op, const void* d_input, uint64_t bytes,
                           uint64_t R, mr_strategy* s, bool* used) {
  *s = MR_STRAT_RULE;
  *used = false;
  if (!job->sel_loaded) return MR_OK;  // no weights: the rule decides
  const int fk = feature_kind(kind);
  if (fk < 0) return MR_OK;
  static const mr_strategy order[MR_N_STRATS] = {MR_STRAT_LDS_ARRAY, MR_STRAT_GLOBAL_ARRAY, MR_STRAT_HASH, MR_STRAT_SORT};
  uint32_t feas = 0;
  for (int i = 0; i < MR_N_STRATS; ++i)
    if (int_feasible(order[i], R, (uint32_t)op)) feas |= 1u << i;
  mr_status st = int_ensure(job, kRegSmall, &job->int_small, &job->int_small_bytes, sizeof(IntSmall), 0);
  if (st != MR_OK) return st;
  IntSmall* sm = static_cast<IntSmall*>(job->int_small);
  st = sel_upload(job);
  if (st != MR_OK) return st;
  float* d = static_cast<float*>(job->sel_dev);
  MR_HIP(features_enqueue(static_cast<const uint8_t*>(d_input), bytes, fk, (int)op, R, (uint32_t)kLdsArrayBudget, d,
                          d + kSelState, job->stream));
  MR_HIP(select_enqueue(d, d + kSelNorm, d + kSelParams, feas, reinterpret_cast<int32_t*>(&sm->choice), job->stream));
  IntSmall hs;
  MR_HIP(hipMemcpyAsync(&hs, sm, sizeof hs, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  if (hs.choice >= 0 && hs.choice < MR_N_STRATS) {
    *s = order[hs.choice];
    *used = true;
  }
  return MR_OK;
}

// A batch's integer items. The containers are decided first: by the learned
// selector for all items at once (features and network of every item in one
// captured graph, replayed while the batch's inputs stay the same, then one
// read-back of the choices), otherwise by the rule or the job's forced
// container. The regions are then sized for the largest item and the items'
// containers are enqueued one after another on the job's stream, each with
// its own state block (hash-table items still read their key count back);
// batch_ints_finish reads all states back once.
mr_status batch_ints_enqueue(mr_job* job, const mr_batch_item* items, const std::vector<uint32_t>& ii, mr_output* outs,
                             std::vector<mr_status>& per) {
  const uint32_t ni = (uint32_t)ii.size();
  const hipStream_t s = job->stream;
  mr_status st = int_ensure(job, kRegSmall, &job->int_small, &job->int_small_bytes, sizeof(IntSmall) * ni, -1);
  if (st != MR_OK) return st;
  IntSmall* sm = static_cast<IntSmall*>(job->int_small);
  MR_HIP(hipMemsetAsync(sm, 0, sizeof(IntSmall) * ni, s));
  std::vector<mr_strategy> strat(ni, MR_STRAT_RULE);
  std::vector<uint8_t> chosen(ni, 0);
  for (uint32_t q = 0; q < ni; ++q) {
    const mr_batch_item& it = items[ii[q]];
    const uint32_t esz = it.kind == MR_MAP_U32_KV ? 8 : 4;
    if (it.input_bytes % esz || (it.input_bytes && !it.d_input) || (uintptr_t)it.d_input % 4 ||
        (it.kind == MR_MAP_U32_KEYS && it.op != MR_REDUCE_COUNT) || it.op > MR_REDUCE_MAX || it.key_range > (1ull << 32))
      return fail(MR_ERR_INVALID_ARG, "integer item %u is malformed", ii[q]);
  }
  static const mr_strategy order[MR_N_STRATS] = {MR_STRAT_LDS_ARRAY, MR_STRAT_GLOBAL_ARRAY, MR_STRAT_HASH, MR_STRAT_SORT};
  if (job->cfg.strategy == MR_STRAT_LEARNED && job->sel_loaded) {
    // the selector region with one feature row per item after its own fields
    st = sel_scratch(job, sel_floats() + 16ull * ni);
    if (st != MR_OK) return st;
    st = sel_upload(job);
    if (st != MR_OK) return st;
    float* d = static_cast<float*>(job->sel_dev);
    float* rows = d + sel_floats();
    uint64_t key = fnv_mix(fnv_mix(0xCBF29CE484222325ull, (uint64_t)d), (uint64_t)sm);
    std::vector<uint32_t> feas(ni, 0);
    for (uint32_t q = 0; q < ni; ++q) {
      const mr_batch_item& it = items[ii[q]];
      for (int k = 0; k < MR_N_STRATS; ++k)
        if (int_feasible(order[k], it.key_range, (uint32_t)it.op)) feas[q] |= 1u << k;
      for (uint64_t v : {(uint64_t)it.d_input, it.input_bytes, (uint64_t)it.kind, (uint64_t)it.op, it.key_range,
                         (uint64_t)feas[q]})
        key = fnv_mix(key, v);
    }
    if (!job->sel_graph || job->sel_graph_key != key) {
      if (job->sel_graph) {
        MR_HIP(hipGraphExecDestroy(job->sel_graph));
        job->sel_graph = nullptr;
      }
      hipGraph_t g = nullptr;
      const hipStream_t cs = job->gstream;
      MR_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipError_t e = hipSuccess;
      for (uint32_t q = 0; q < ni && e == hipSuccess; ++q) {
        const mr_batch_item& it = items[ii[q]];
        e = features_enqueue(static_cast<const uint8_t*>(it.d_input), it.input_bytes, feature_kind(it.kind), (int)it.op,
                             it.key_range, (uint32_t)kLdsArrayBudget, rows + 16ull * q, d + kSelState, cs);
        if (e == hipSuccess) e = select_enqueue(rows + 16ull * q, d + kSelNorm, d + kSelParams, feas[q], &sm[q].choice, cs);
      }
      const hipError_t e2 = hipStreamEndCapture(cs, &g);
      if (e == hipSuccess && e2 == hipSuccess) e = hipGraphInstantiate(&job->sel_graph, g, nullptr, nullptr, 0);
      if (g) (void)hipGraphDestroy(g);
      if (e != hipSuccess || e2 != hipSuccess)
        return fail(MR_ERR_HIP, "selection graph: %s", hipGetErrorString(e != hipSuccess ? e : e2));
      job->sel_graph_key = key;
    }
    MR_HIP(hipGraphLaunch(job->sel_graph, s));
    std::vector<IntSmall> hs(ni);
    MR_HIP(hipMemcpyAsync(hs.data(), sm, sizeof(IntSmall) * ni, hipMemcpyDeviceToHost, s));
    MR_HIP(hipStreamSynchronize(s));
    for (uint32_t q = 0; q < ni; ++q)
      if (hs[q].choice >= 0 && hs[q].choice < MR_N_STRATS) {
        strat[q] = order[hs[q].choice];
        chosen[q] = 1;
      }
  } else if (job->cfg.strategy != MR_STRAT_LEARNED) {
    for (uint32_t q = 0; q < ni; ++q) strat[q] = job->cfg.strategy;
  }
  // the rule for the items the selector left to it; the regions for the largest item
  uint64_t dense_b = 0, dense_r = 0, table_s = 0, scratch_b = 0;
  for (uint32_t q = 0; q < ni; ++q) {
    const mr_batch_item& it = items[ii[q]];
    const uint32_t op = (uint32_t)it.op;
    const uint64_t n = it.input_bytes / (it.kind == MR_MAP_U32_KV ? 8 : 4);
    if (strat[q] == MR_STRAT_RULE || strat[q] == MR_STRAT_LEARNED)
      strat[q] = rule_strategy(it.key_range, op, eff_lds_array_bytes(job, it.kind, it.input_bytes));
    if (!int_feasible(strat[q], it.key_range, op)) {
      per[ii[q]] = fail(MR_ERR_UNSUPPORTED, "strategy %d is infeasible for item %u", (int)strat[q], ii[q]);
      continue;
    }
    const uint32_t G = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)job->n_cu * 2, (n + 1023) / 1024));
    if (strat[q] == MR_STRAT_LDS_ARRAY || strat[q] == MR_STRAT_GLOBAL_ARRAY) {
      dense_r = std::max(dense_r, it.key_range);
      dense_b = std::max(dense_b, it.key_range * 12 + 8);
      scratch_b = std::max(scratch_b, dense_carve(strat[q], n, it.key_range, op, G).bytes);
    } else if (strat[q] == MR_STRAT_HASH) {
      table_s = std::max(table_s, int_table_slots(job, it.kind, it.input_bytes, n, it.key_range));
      scratch_b = std::max(scratch_b, hash_carve(it.key_range ? std::min(n, it.key_range) : n).bytes);
    } else {
      scratch_b = std::max(scratch_b, sort_carve(n).bytes);
    }
  }
  if (dense_b) {
    bool fresh = false;
    st = int_ensure(job, kRegDense, &job->int_dense, &job->int_dense_bytes, dense_b, 0, &fresh);
    if (st != MR_OK) return st;
    if (fresh) job->int_dense_R = dense_r;
  }
  if (table_s) {
    bool fresh = false;
    st = dev_region(job, kRegTable, &job->int_table, &job->int_table_bytes, table_s * kIntSlotBytes, table_s * kIntSlotBytes,
                    &fresh);
    if (st != MR_OK) return st;
    if (fresh) {
      job->int_table_cap = table_s;
      MR_HIP(hipMemsetAsync(job->int_table, 0xFF, table_s * 4, s));
      MR_HIP(hipMemsetAsync(static_cast<uint8_t*>(job->int_table) + table_s * 4, 0, table_s * 16, s));
    }
  }
  if (scratch_b) {
    st = int_ensure(job, kRegScratch, &job->int_scratch, &job->int_scratch_bytes, scratch_b, -1);
    if (st != MR_OK) return st;
  }
  if (!job->ev_int0) MR_HIP(hipEventCreate(&job->ev_int0));
  if (!job->ev_int1) MR_HIP(hipEventCreate(&job->ev_int1));
  MR_HIP(hipEventRecord(job->ev_int0, s));
  for (uint32_t q = 0; q < ni; ++q) {
    if (per[ii[q]] != MR_OK) continue;
    const mr_batch_item& it = items[ii[q]];
    const U32Ctx ctx{strat[q], chosen[q] != 0, sm + q};
    st = run_u32(job, it.kind, it.op, it.d_input, it.input_bytes, it.key_range, &outs[ii[q]], &ctx);
    if (st == MR_ERR_HIP) return st;
    per[ii[q]] = st;
  }
  MR_HIP(hipEventRecord(job->ev_int1, s));
  return MR_OK;
}

mr_status batch_ints_finish(mr_job* job, const std::vector<uint32_t>& ii, mr_output* outs, std::vector<mr_status>& per) {
  const uint32_t ni = (uint32_t)ii.size();
  std::vector<IntSmall> hs(ni);
  MR_HIP(hipMemcpyAsync(hs.data(), job->int_small, sizeof(IntSmall) * ni, hipMemcpyDeviceToHost, job->stream));
  MR_HIP(hipStreamSynchronize(job->stream));
  float ms = 0.f;
  MR_HIP(hipEventElapsedTime(&ms, job->ev_int0, job->ev_int1));
  for (uint32_t q = 0; q < ni; ++q) {
    mr_output* o = &outs[ii[q]];
    o->stats.gpu_ms = ms;
    if (per[ii[q]] == MR_OK) per[ii[q]] = u32_finish(job, o, hs[q]);
  }
  return MR_OK;
}

mr_status mlp_scratch(mr_job* job, uint32_t B) {
  const uint64_t need = (uint64_t)B * (4 + 64 + 64) + 64;
  return int_ensure(job, kRegMlp, &job->mlp_dev, &job->mlp_dev_bytes, 4 * need, -1);
}

}  // namespace

extern "C" mr_status mr_mlp_forward(mr_job* job, const float* params, const float* X, uint32_t B, float* H1, float* H2,
                                    float* Y) {
  if (!job || !params || (B && (!X || !Y))) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  ScopedDevice sd(job->device);
  MR_HIP(mlp_forward_enqueue(params, X, B, H1, H2, Y, job->stream));
  return MR_OK;
}

extern "C" mr_status mr_mlp_loss_backward(mr_job* job, const float* params, const float* X, const float* H1,
                                          const float* H2, const float* Y, const float* T, const float* M, uint32_t B,
                                          float* loss, float* grad) {
  if (!job || !params || !loss || !grad || (B && (!X || !H1 || !H2 || !Y || !T || !M)))
    return fail(MR_ERR_INVALID_ARG, "NULL argument");
  ScopedDevice sd(job->device);
  arena_begin(job, kFamMlp);
  mr_status st = mlp_scratch(job, B);
  if (st != MR_OK) return st;
  float* d = static_cast<float*>(job->mlp_dev);
  float* dY = d;
  float* dZ1 = d + 4ull * B;
  float* dZ2 = dZ1 + 64ull * B;
  MR_HIP(mlp_backward_enqueue(params, X, H1, H2, Y, T, M, B, dY, dZ1, dZ2, loss, grad, job->stream));
  return MR_OK;
}

extern "C" mr_status mr_mlp_adam(mr_job* job, float* params, const float* grad, float* m, float* v, uint32_t step, float lr,
                                 float beta1, float beta2, float eps) {
  if (!job || !params || !grad || !m || !v) return fail(MR_ERR_INVALID_ARG, "NULL argument");
  if (step == 0) return fail(MR_ERR_INVALID_ARG, "Adam steps count from 1");
  ScopedDevice sd(job->device);
  MR_HIP(adam_enqueue(params, grad, m, v, step, lr, beta1, beta2, eps, job->stream));
  return MR_OK;
}

// ----------------------------------------------------------------------------
// selector training: the whole loop on the device with the network kernels
// ----------------------------------------------------------------------------

namespace {

// SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
// generators", 2014): initialisation and shuffling of the training loop.
struct SplitMix64 {
  uint64_t x;
  uint64_t next() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }  // [0, 1)
};

mr_status write_selector_json(const char* path, const std::vector<float>& P, const float* mean, const float* scale,
                              const float* lo, const float* hi, double mu, double sd) {
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(MR_ERR_INVALID_ARG, "cannot write %s", path);
  auto arr = [&](const char* name, const float* a, size_t n, bool last) {
    std::fprintf(f, "\"%s\": [", name);
    for (size_t i = 0; i < n; ++i) std::fprintf(f, "%s%.9g", i ? ", " : "", (double)a[i]);
    std::fprintf(f, "]%s", last ? "" : ", ");
  };
  std::fprintf(f, "{");
  arr("params", P.data(), P.size(), false);
  arr("feat_mean", mean, MR_N_FEATURES, false);
  arr("feat_scale", scale, MR_N_FEATURES, false);
  arr("feat_lo", lo, MR_N_FEATURES, false);
  arr("feat_hi", hi, MR_N_FEATURES, false);
  std::fprintf(f, "\"target_mu\": %.17g, \"target_sd\": %.17g, "
                  "\"strategies\": [\"lds_array\", \"global_array\", \"hash\", \"sort\"]}", mu, sd);
  const bool ok = std::fclose(f) == 0;
  return ok ? MR_OK : fail(MR_ERR_INVALID_ARG, "writing %s failed", path);
}

}  // namespace

extern "C" mr_status mr_selector_train(mr_job* job, const float* feats, const float* times, const uint8_t* feasible,
                                       uint32_t n, const mr_train_config* tc, float* loss_out, const char* out_json) {
  if (!job || !feats || !times || !feasible || !tc || n == 0) return fail(MR_ERR_INVALID_ARG, "NULL argument or no jobs");
  const uint32_t epochs = tc->epochs ? tc->epochs : 500, B = tc->batch ? tc->batch : 64;
  const float lr = tc->lr > 0.f ? tc->lr : 1e-3f, b1 = tc->beta1 > 0.f ? tc->beta1 : 0.9f;
  const float b2 = tc->beta2 > 0.f ? tc->beta2 : 0.999f, eps = tc->eps > 0.f ? tc->eps : 1e-8f;
  if (B > 4096 || b1 >= 1.f || b2 >= 1.f) return fail(MR_ERR_INVALID_ARG, "batch above 4096 or a beta not below 1");
  const uint32_t F = MR_N_FEATURES, S = MR_N_STRATS;
  // feature normalisation: mean and standard deviation (a constant feature keeps scale 1)
  std::vector<double> mean(F, 0.0), var(F, 0.0);
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t f = 0; f < F; ++f) mean[f] += feats[(size_t)i * F + f];
  for (uint32_t f = 0; f < F; ++f) mean[f] /= n;
  for (uint32_t i = 0; i < n; ++i)
    for (uint32_t f = 0; f < F; ++f) {
      const double dlt = feats[(size_t)i * F + f] - mean[f];
      var[f] += dlt * dlt;
    }
  std::vector<float> fmean(F), fscale(F), flo(F), fhi(F);
  for (uint32_t f = 0; f < F; ++f) {
    fmean[f] = (float)mean[f];
    const double sdv = std::sqrt(var[f] / n);
    fscale[f] = sdv < 1e-6 ? 1.f : (float)sdv;
    double mn = feats[f], mx = feats[f];
    for (uint32_t i = 1; i < n; ++i) {
      mn = std::min<double>(mn, feats[(size_t)i * F + f]);
      mx = std::max<double>(mx, feats[(size_t)i * F + f]);
    }
    // the range seen in training, widened by a tenth: outside it the rule decides
    flo[f] = (float)(mn - 0.1 * (mx - mn) - 1e-3);
    fhi[f] = (float)(mx + 0.1 * (mx - mn) + 1e-3);
  }
  // targets: log device times over the feasible containers, standardised with one mean and scale
  double mu = 0.0, m2 = 0.0;
  uint64_t nf = 0;
  for (uint64_t i = 0; i < (uint64_t)n * S; ++i)
    if (feasible[i]) {
      if (!(times[i] > 0.f)) return fail(MR_ERR_INVALID_ARG, "a feasible time is not positive (job %llu)", (unsigned long long)(i / S));
      mu += std::log((double)times[i]);
      ++nf;
    }
  if (!nf) return fail(MR_ERR_INVALID_ARG, "no feasible container in any job");
  mu /= nf;
  for (uint64_t i = 0; i < (uint64_t)n * S; ++i)
    if (feasible[i]) m2 += (std::log((double)times[i]) - mu) * (std::log((double)times[i]) - mu);
  double sd = std::sqrt(m2 / nf);
  if (!(sd > 0.0)) sd = 1.0;
  // one row per job: normalised features, targets, mask
  constexpr uint32_t kRow = MR_N_FEATURES + 2 * MR_N_STRATS;
  std::vector<float> rows((size_t)n * kRow);
  for (uint32_t i = 0; i < n; ++i) {
    float* r = &rows[(size_t)i * kRow];
    for (uint32_t f = 0; f < F; ++f) r[f] = (float)((feats[(size_t)i * F + f] - fmean[f]) / fscale[f]);
    for (uint32_t k = 0; k < S; ++k) {
      const bool ok = feasible[(size_t)i * S + k] != 0;
      r[F + k] = ok ? (float)((std::log((double)times[(size_t)i * S + k]) - mu) / sd) : 0.f;
      r[F + S + k] = ok ? 1.f : 0.f;
    }
  }
  // He-uniform initialisation: weights U(-sqrt(6 / fan_in), +sqrt(6 / fan_in)), biases 0
  SplitMix64 rng{tc->seed};
  std::vector<float> P(MR_MLP_PARAMS, 0.f);
  {
    size_t o = 0;
    const uint32_t dims[4] = {MR_N_FEATURES, 64, 64, MR_N_STRATS};
    for (int l = 0; l < 3; ++l) {
      const double lim = std::sqrt(6.0 / dims[l]);
      for (uint32_t i = 0; i < dims[l] * dims[l + 1]; ++i) P[o++] = (float)((2.0 * rng.uniform() - 1.0) * lim);
      o += dims[l + 1];
    }
  }
  ScopedDevice sd_(job->device);
  arena_begin(job, kFamTrain);
  // device memory: parameters, gradient, moments, the epoch's shuffled rows,
  // activations and backward scratch of one batch, per-batch losses
  const uint32_t nb = (n + B - 1) / B;
  Carve c;
  const uint64_t o_p = c.take(4ull * MR_MLP_PARAMS), o_g = c.take(4ull * MR_MLP_PARAMS);
  const uint64_t o_m = c.take(4ull * MR_MLP_PARAMS), o_v = c.take(4ull * MR_MLP_PARAMS);
  const uint64_t o_x = c.take(4ull * n * F), o_t = c.take(4ull * n * S), o_k = c.take(4ull * n * S);
  const uint64_t o_h1 = c.take(4ull * B * 64), o_h2 = c.take(4ull * B * 64), o_y = c.take(4ull * B * S);
  const uint64_t o_dy = c.take(4ull * B * S), o_dz1 = c.take(4ull * B * 64), o_dz2 = c.take(4ull * B * 64);
  const uint64_t o_loss = c.take(4ull * nb);
  void* mem = nullptr;
  uint64_t have = 0;
  bool fresh = false;
  mr_status st = dev_region(job, kRegTrain, &mem, &have, c.off, c.off, &fresh);
  if (st != MR_OK) return st;
  uint8_t* d = static_cast<uint8_t*>(mem);
  auto F32 = [&](uint64_t o) { return reinterpret_cast<float*>(d + o); };
  const hipStream_t s = job->stream;
  mr_status result = MR_OK;
  std::vector<float> X((size_t)n * F), T((size_t)n * S), M((size_t)n * S), losses(nb);
  std::vector<uint32_t> perm(n);
  for (uint32_t i = 0; i < n; ++i) perm[i] = i;
  do {
    hipError_t e = hipMemcpyAsync(F32(o_p), P.data(), 4ull * MR_MLP_PARAMS, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemsetAsync(F32(o_m), 0, 4ull * MR_MLP_PARAMS, s);
    if (e == hipSuccess) e = hipMemsetAsync(F32(o_v), 0, 4ull * MR_MLP_PARAMS, s);
    uint32_t step = 0;
    for (uint32_t ep = 0; ep < epochs && e == hipSuccess; ++ep) {
      // Fisher-Yates shuffle, then the rows in that order as split arrays
      for (uint32_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[(uint32_t)(rng.next() % (i + 1))]);
      for (uint32_t i = 0; i < n; ++i) {
        const float* r = &rows[(size_t)perm[i] * kRow];
        std::memcpy(&X[(size_t)i * F], r, 4 * F);
        std::memcpy(&T[(size_t)i * S], r + F, 4 * S);
        std::memcpy(&M[(size_t)i * S], r + F + S, 4 * S);
      }
      e = hipMemcpyAsync(F32(o_x), X.data(), 4ull * n * F, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(F32(o_t), T.data(), 4ull * n * S, hipMemcpyHostToDevice, s);
      if (e == hipSuccess) e = hipMemcpyAsync(F32(o_k), M.data(), 4ull * n * S, hipMemcpyHostToDevice, s);
      for (uint32_t b = 0; b < nb && e == hipSuccess; ++b) {
        const uint32_t i0 = b * B, bs = std::min(B, n - i0);
        const float* xb = F32(o_x) + (size_t)i0 * F;
        const float* tb = F32(o_t) + (size_t)i0 * S;
        const float* mb = F32(o_k) + (size_t)i0 * S;
        e = mlp_forward_enqueue(F32(o_p), xb, bs, F32(o_h1), F32(o_h2), F32(o_y), s);
        if (e == hipSuccess)
          e = mlp_backward_enqueue(F32(o_p), xb, F32(o_h1), F32(o_h2), F32(o_y), tb, mb, bs, F32(o_dy), F32(o_dz1),
                                   F32(o_dz2), F32(o_loss) + b, F32(o_g), s);
        if (e == hipSuccess) e = adam_enqueue(F32(o_p), F32(o_g), F32(o_m), F32(o_v), ++step, lr, b1, b2, eps, s);
      }
      // the epoch's mean loss (batches weighted by their size); the host
      // arrays are rewritten only after this synchronisation
      if (e == hipSuccess) e = hipMemcpyAsync(losses.data(), F32(o_loss), 4ull * nb, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e == hipSuccess && loss_out) {
        double tot = 0.0;
        for (uint32_t b = 0; b < nb; ++b) tot += (double)losses[b] * std::min(B, n - b * B);
        loss_out[ep] = (float)(tot / n);
      }
    }
    if (e == hipSuccess) e = hipMemcpyAsync(P.data(), F32(o_p), 4ull * MR_MLP_PARAMS, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) result = fail(MR_ERR_HIP, "selector training: %s", hipGetErrorString(e));
  } while (false);
  if (job->cws == nullptr) (void)hipFree(mem);  // library memory of this call only
  if (result != MR_OK) return result;
  st = mr_selector_set(job, P.data(), fmean.data(), fscale.data(), flo.data(), fhi.data());
  if (st != MR_OK) return st;
  if (out_json) return write_selector_json(out_json, P, fmean.data(), fscale.data(), flo.data(), fhi.data(), mu, sd);
  return MR_OK;
}

// ----------------------------------------------------------------------------
// word hashing one character per lane per step (SIMDH-Padding / SIMDH-Stream)
// ----------------------------------------------------------------------------

extern "C" mr_status mr_hash_words(mr_job* job, const void* d_input, uint64_t input_bytes, uint32_t mode, uint32_t units,
                                   uint32_t block, uint64_t* d_hashes, uint32_t* d_sched, uint64_t cap_words,
                                   uint64_t* n_words, float* hash_ms) {
  if (!job || !n_words || (input_bytes && !d_input) || (cap_words && !d_hashes))
    return fail(MR_ERR_INVALID_ARG, "NULL argument");
  if (mode > 1 || units == 0 || units > 64) return fail(MR_ERR_INVALID_ARG, "mode must be 0 or 1 and units 1..64");
  if (input_bytes >= (1ull << 32)) return fail(MR_ERR_UNSUPPORTED, "inputs must be below 4 GiB");
  const uint64_t blk = block ? block : 4096;
  ScopedDevice sd(job->device);
  arena_begin(job, kFamHash);
  const hipStream_t s = job->stream;
  const uint8_t* in = static_cast<const uint8_t*>(d_input);
  const uint64_t n_chunks = (input_bytes + 15) / 16;
  Carve c;
  const uint64_t o_cnt = c.take(4 * std::max<uint64_t>(n_chunks, 1)), o_sums = c.take(4 * scan_sums_count(n_chunks));
  const uint64_t o_tot = c.take(8);
  mr_status st = int_ensure(job, kRegScratch, &job->int_scratch, &job->int_scratch_bytes, c.off, -1);
  if (st != MR_OK) return st;
  uint8_t* sc = static_cast<uint8_t*>(job->int_scratch);
  uint32_t* counts = reinterpret_cast<uint32_t*>(sc + o_cnt);
  unsigned long long total = 0;
  MR_HIP(hw_enqueue_list(in, input_bytes, counts, n_chunks, reinterpret_cast<uint32_t*>(sc + o_sums),
                         reinterpret_cast<unsigned long long*>(sc + o_tot), s));
  MR_HIP(hipMemcpyAsync(&total, sc + o_tot, 8, hipMemcpyDeviceToHost, s));
  MR_HIP(hipStreamSynchronize(s));
  *n_words = total;
  if (total > cap_words) return fail(MR_ERR_CAPACITY, "the input has %llu words", (unsigned long long)total);
  void* lst = nullptr;
  uint64_t lst_have = 0;
  bool fresh = false;
  st = dev_region(job, kRegHashList, &lst, &lst_have, 8 * std::max<uint64_t>(total, 1), 8 * std::max<uint64_t>(total, 1),
                  &fresh);
  if (st != MR_OK) return st;
  uint32_t* off = static_cast<uint32_t*>(lst);
  uint32_t* len = off + total;
  mr_status result = MR_OK;
  do {
    hipError_t e = hw_enqueue_words(in, input_bytes, counts, n_chunks, off, len, s);
    if (e == hipSuccess) e = hipEventRecord(job->ev0, s);
    if (e == hipSuccess)
      e = hw_enqueue_hash(in, off, len, total, mode == 1, units, blk, reinterpret_cast<unsigned long long*>(d_hashes),
                          d_sched, s);
    if (e == hipSuccess) e = hipEventRecord(job->ev1, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, job->ev0, job->ev1);
    if (e != hipSuccess) result = fail(MR_ERR_HIP, "mr_hash_words: %s", hipGetErrorString(e));
    if (hash_ms) *hash_ms = ms;
  } while (false);
  if (!job->cws) (void)hipFree(lst);  // library memory of this call only
  return result;
}
