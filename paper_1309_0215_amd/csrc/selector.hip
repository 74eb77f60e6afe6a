// Learned reduce-strategy selector on gfx950: job features from a sample of
// the input, and the kernels of a 12-64-64-4 ReLU network (forward, masked
// mean-squared-error backward, Adam). The paper's framework decides which
// technique to apply from properties of the job (Sections III-B, III-E); here
// the decision among the four reduce containers is learned from measured
// times, with the paper-style rule as the fallback and the yardstick.
#include "common.h"
#include "launch.h"

namespace mr {

// ----------------------------------------------------------------------------
// features
// ----------------------------------------------------------------------------
constexpr int kFeatThreads = 1024;
constexpr uint32_t kHllLog = 11;                    // 2048 registers
constexpr uint32_t kHllM = 1u << kHllLog;
constexpr uint32_t kWindows = 32;
constexpr uint32_t kWindowBytes = 4096;
constexpr uint32_t kSegBlocks = kWindowBytes / 16 + 1;  // aligned 16-byte blocks covering one window

MR_DEV void hll_add(uint32_t* reg, uint64_t h) {
  const uint32_t idx = (uint32_t)(h >> (64 - kHllLog));
  const uint64_t rest = (h << kHllLog) | (1ull << (kHllLog - 1));  // guard bit bounds the rank
  const uint32_t rank = (uint32_t)__clzll((long long)rest) + 1;
  atomicMax(&reg[idx], rank);
}

MR_DEV float hll_estimate(const uint32_t* reg, float* red) {
  // sum of 2^-M and zero registers, by the whole block
  float s = 0.f;
  float z = 0.f;
  for (uint32_t i = threadIdx.x; i < kHllM; i += blockDim.x) {
    s += exp2f(-(float)reg[i]);
    z += reg[i] == 0 ? 1.f : 0.f;
  }
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o);
    z += __shfl_xor(z, o);
  }
  __syncthreads();
  if (lane_id() == 0) {
    red[2 * (threadIdx.x / kWave)] = s;
    red[2 * (threadIdx.x / kWave) + 1] = z;
  }
  __syncthreads();
  float S = 0.f, Z = 0.f;
  for (uint32_t w = 0; w < blockDim.x / kWave; ++w) {
    S += red[2 * w];
    Z += red[2 * w + 1];
  }
  __syncthreads();
  const float m = (float)kHllM;
  const float alpha = 0.7213f / (1.f + 1.079f / m);
  float E = alpha * m * m / S;
  if (E <= 2.5f * m && Z > 0.f) E = m * logf(m / Z);  // small-range correction (linear counting)
  return E;
}

// hist[bin] += 1 for every active lane, one atomic per distinct bin of the
// wave (the bins of neighbouring slots are mostly equal; same-address LDS
// atomics from many lanes would run one after another).
MR_DEV void wave_hist_add(uint32_t* hist, uint32_t bin, bool act) {
  while (true) {
    const uint64_t m = __ballot(act);
    if (!m) return;
    const uint32_t lb = (uint32_t)__shfl((int)bin, (int)(__ffsll((unsigned long long)m) - 1));
    const uint64_t eq = __ballot(act && bin == lb);
    if (act && bin == lb) {
      if (__popcll(eq & ((1ull << lane_id()) - 1)) == 0) atomicAdd(&hist[lb], (uint32_t)__popcll(eq));
      act = false;
    }
  }
}

// Count c more of key in an exact count table of `slots` slots (a power of
// two). At most half of the slots are claimed (used counts the claims): a key
// without a slot by then is not counted, and the probe runs stay short.
MR_DEV void feat_insert(uint32_t* tk, uint32_t* tc, uint32_t slots, uint32_t* used, uint32_t key, uint32_t c) {
  uint32_t s = (uint32_t)hash_u32(key) & (slots - 1);
  for (int p = 0; p < 32; ++p) {
    uint32_t cur = tk[s];
    if (cur == 0xFFFFFFFFu) {
      if (*used >= slots / 2) return;
      cur = atomicCAS(&tk[s], 0xFFFFFFFFu, key);
      if (cur == 0xFFFFFFFFu) {
        atomicAdd(used, 1u);
        atomicAdd(&tc[s], c);
        return;
      }
    }
    if (cur == key) {
      atomicAdd(&tc[s], c);
      return;
    }
    s = (s + 1) & (slots - 1);
  }
}

// The 64 largest of the n counts tc[0, n) (LDS), in descending order, into
// top[64] (LDS), padded as described below. Called by the whole workgroup;
// n is a multiple of blockDim.x. (counts stay below 2^17: the sample holds
// at most 64 Ki elements)
MR_DEV void top64_of(const uint32_t* tc, uint32_t n, uint32_t* top) {
  // The 64 largest counts, exactly: radix-select the 64th largest value v64
  // with two histogram passes over the count bits (counts stay below 2^17:
  // the sample holds at most 64 Ki elements), then collect the counts above
  // v64, order them by rank, and pad with v64 (ties) or zeros (fewer than 64
  // keys). The bucket walks are wave prefix sums, not a serial loop.
  {
    __shared__ uint32_t hist[512];
    __shared__ uint32_t s_b1, s_above, s_v64, s_ngt;
    __shared__ uint32_t gt[64];
    const uint32_t lane = lane_id();
    for (uint32_t i = threadIdx.x; i < 512; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) {
      s_ngt = 0;
      s_b1 = 0xFFFFFFFFu;  // none: fewer than 64 nonzero counts
      s_above = 0;
      s_v64 = 0;
    }
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t c = tc[i];
      wave_hist_add(hist, min(c >> 9, 255u), c != 0);
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
      // lane l holds buckets 255 - 4l down to 252 - 4l
      uint32_t h4[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        h4[q] = hist[255 - 4 * lane - q];
        sum += h4[q];
      }
      uint32_t incl = sum;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
        if (lane >= (uint32_t)o) incl += y;
      }
      uint32_t acc = incl - sum;
      if (acc < 64 && incl >= 64) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (acc + h4[q] >= 64) {
            s_b1 = 255 - 4 * lane - (uint32_t)q;
            s_above = acc;
            break;
          }
          acc += h4[q];
        }
      }
    }
    __syncthreads();
    const uint32_t b1 = s_b1;
    if (b1 != 0xFFFFFFFFu) {
      for (uint32_t i = threadIdx.x; i < 512; i += blockDim.x) hist[i] = 0;
      __syncthreads();
      for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
        const uint32_t c = tc[i];
        wave_hist_add(hist, c & 511u, c && min(c >> 9, 255u) == b1);
      }
      __syncthreads();
      if (threadIdx.x < kWave) {
        // lane l holds values 511 - 8l down to 504 - 8l of bucket b1
        uint32_t h8[8], sum = 0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          h8[q] = hist[511 - 8 * lane - q];
          sum += h8[q];
        }
        uint32_t incl = sum;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
          const uint32_t y = (uint32_t)__shfl_up((int)incl, o);
          if (lane >= (uint32_t)o) incl += y;
        }
        uint32_t acc = s_above + incl - sum;
        const bool last = lane == kWave - 1;
        if ((acc < 64 && acc + sum >= 64) || (last && acc + sum < 64)) {
          uint32_t lo = 0;
#pragma unroll
          for (int q = 0; q < 8; ++q) {
            const uint32_t v = 511 - 8 * lane - (uint32_t)q;
            if (acc + h8[q] >= 64 || v == 0) {
              lo = v;
              break;
            }
            acc += h8[q];
          }
          s_v64 = (b1 << 9) | lo;
        }
      }
    }
    __syncthreads();
    const uint32_t v64 = s_v64;
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
      const uint32_t c = tc[i];
      // one place reservation per wave
      const uint64_t m = __ballot(c > v64);
      if (m) {
        const uint32_t lane = lane_id();
        uint32_t base = 0;
        if (lane == (uint32_t)(__ffsll((unsigned long long)m) - 1)) base = atomicAdd(&s_ngt, (uint32_t)__popcll(m));
        base = (uint32_t)__shfl((int)base, (int)(__ffsll((unsigned long long)m) - 1));
        if (c > v64) {
          const uint32_t q = base + (uint32_t)__popcll(m & ((1ull << lane) - 1));
          if (q < 64) gt[q] = c;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x < 64) {
      // descending order by rank (ties keep their collection order)
      const uint32_t n = min(s_ngt, 64u), t = threadIdx.x;
      if (t < n) {
        const uint32_t x = gt[t];
        uint32_t rank = 0;
        for (uint32_t u = 0; u < n; ++u) rank += (gt[u] > x || (gt[u] == x && u < t)) ? 1u : 0u;
        top[rank] = x;
      } else {
        top[t] = v64;
      }
    }
    __syncthreads();
  }
}

constexpr int kSampThreads = 256;
constexpr uint32_t kLocalSlots = 2048;  // distinct keys of one window (at most 2048 elements)

// Per-window results written by the sampling workgroups (every field is
// rewritten on each call, so nothing needs clearing).
struct FeatWindow {
  uint8_t hll_all[kHllM];
  uint8_t hll_half[kHllM];
  uint32_t key[kLocalSlots];
  uint32_t cnt[kLocalSlots];
  uint32_t n_keys;
  uint32_t pad;
  unsigned long long n, len, len2;
};

// Geometry of the sample: kWindows evenly spaced windows of wel elements, or
// the whole input in consecutive pieces of wel elements when it is small.
struct Sample {
  uint64_t esz, n_elem, wel;
  bool whole;
  uint32_t nseg;
};

MR_DEV Sample sample_of(uint64_t bytes, int kind) {
  Sample S;
  S.esz = kind == 0 ? 1 : (kind == 1 ? 4 : 8);
  S.n_elem = bytes / S.esz;
  S.wel = kWindowBytes / S.esz;
  S.whole = S.n_elem <= (uint64_t)kWindows * S.wel;
  S.nseg = S.whole ? (uint32_t)((S.n_elem + S.wel - 1) / S.wel) : kWindows;
  return S;
}

// One workgroup per segment: its elements into LDS registers and counts,
// written out as the window's registers, (key, count) list and sums.
__global__ __launch_bounds__(kSampThreads) void k_feat_sample(const uint8_t* __restrict__ in, uint64_t bytes, int kind,
                                                               FeatWindow* __restrict__ win) {
  __shared__ uint32_t hll_all[kHllM];
  __shared__ uint32_t hll_half[kHllM];
  __shared__ uint32_t tk[kLocalSlots];
  __shared__ uint32_t tc[kLocalSlots];
  __shared__ uint4 stage[kSegBlocks];
  __shared__ unsigned long long s_n, s_len, s_len2;
  __shared__ uint32_t s_keys;
  const Sample S = sample_of(bytes, kind);
  const uint32_t w = blockIdx.x;
  if (w >= S.nseg) return;
  for (uint32_t i = threadIdx.x; i < kHllM; i += blockDim.x) hll_all[i] = hll_half[i] = 0;
  for (uint32_t i = threadIdx.x; i < kLocalSlots; i += blockDim.x) {
    tk[i] = 0xFFFFFFFFu;
    tc[i] = 0;
  }
  if (threadIdx.x == 0) {
    s_n = s_len = s_len2 = 0;
    s_keys = 0;
  }
  const uint64_t esz = S.esz;
  const uint64_t e0 = S.whole ? (uint64_t)w * S.wel : (S.n_elem - S.wel) * w / (kWindows - 1);
  const uint64_t e1 = S.whole ? (e0 + S.wel < S.n_elem ? e0 + S.wel : S.n_elem) : e0 + S.wel;
  const bool half_win = w < (kWindows + 1) / 2;
  const uint64_t lo = ((uint64_t)in + e0 * esz) & ~15ull;
  // the 16-byte aligned blocks covering the segment, all loads in flight at once
  for (uint32_t q = threadIdx.x; q < kSegBlocks; q += blockDim.x) {
    const uint64_t blk = lo + 16ull * q;
    uint4 v = make_uint4(0x20202020u, 0x20202020u, 0x20202020u, 0x20202020u);
    // a block that holds a byte of the input lies inside its allocation
    if (blk < (uint64_t)in + bytes && blk + 16 > (uint64_t)in) v = *reinterpret_cast<const uint4*>(blk);
    stage[q] = v;
  }
  __syncthreads();
  const uint8_t* seg = reinterpret_cast<const uint8_t*>(stage);
  // byte p of the input: from the staged span when it holds it
  auto byte_at = [&](uint64_t p) -> uint32_t {
    const uint64_t a = (uint64_t)in + p;
    return (a >= lo && a < lo + kSegBlocks * 16ull) ? seg[a - lo] : in[p];
  };
  unsigned long long my_n = 0, my_len = 0, my_len2 = 0;
  for (uint64_t e = e0 + threadIdx.x; e < e1; e += blockDim.x) {
    bool act = false;
    uint32_t key = 0;
    uint64_t hh = 0;
    if (kind == 0) {
      // a word starting at byte e (it may run past the segment)
      if (!is_sep_byte(byte_at(e)) && (e == 0 || is_sep_byte(byte_at(e - 1)))) {
        uint32_t hf = 2166136261u;
        uint64_t q = e;
        while (q < bytes && q - e < 256) {
          const uint32_t c = byte_at(q);
          if (is_sep_byte(c)) break;
          hf = (hf ^ c) * 16777619u;
          ++q;
        }
        const uint64_t len = q - e;
        hh = hash_u32(hf ^ (uint32_t)(len * 0x9E3779B9u));
        key = (uint32_t)hh;
        act = true;
        ++my_n;
        my_len += len;
        my_len2 += len * len;
      }
    } else {
      const uint64_t a = (uint64_t)in + e * esz;
      const uint32_t k = *reinterpret_cast<const uint32_t*>(seg + (a - lo));
      hh = hash_u32(k);
      key = k;
      act = true;
      ++my_n;
    }
    if (act) {
      hll_add(hll_all, hh);
      if (S.whole ? (e & 1) != 0 : half_win) hll_add(hll_half, hh);
      uint32_t sl = (uint32_t)hash_u32(key) & (kLocalSlots - 1);
      for (uint32_t p = 0; p < kLocalSlots; ++p) {
        uint32_t cur = tk[sl];
        if (cur == 0xFFFFFFFFu) cur = atomicCAS(&tk[sl], 0xFFFFFFFFu, key);
        if (cur == 0xFFFFFFFFu || cur == key) {
          atomicAdd(&tc[sl], 1u);
          break;
        }
        sl = (sl + 1) & (kLocalSlots - 1);
      }
    }
  }
  if (my_n) atomicAdd(&s_n, my_n);
  if (my_len) atomicAdd(&s_len, my_len);
  if (my_len2) atomicAdd(&s_len2, my_len2);
  __syncthreads();
  FeatWindow& W = win[w];
  for (uint32_t i = threadIdx.x; i < kHllM; i += blockDim.x) {
    W.hll_all[i] = (uint8_t)hll_all[i];
    W.hll_half[i] = (uint8_t)hll_half[i];
  }
  for (uint32_t i = threadIdx.x; i < kLocalSlots; i += blockDim.x) {
    if (tc[i]) {
      const uint32_t at = atomicAdd(&s_keys, 1u);
      W.key[at] = tk[i];
      W.cnt[at] = tc[i];
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    W.n_keys = s_keys;
    W.n = s_n;
    W.len = s_len;
    W.len2 = s_len2;
  }
}

constexpr uint32_t kMergeParts = 16;     // key partitions merged by separate workgroups
constexpr uint32_t kMergeSlots = 4096;   // count table of one partition

// Exact counts of the sampled keys, one workgroup per hash partition of the
// keys (every occurrence of a key lands in the same partition): the windows'
// (key, count) lists into an LDS table, then the partition's 64 largest
// counts into cand[partition][64].
__global__ __launch_bounds__(kFeatThreads) void k_feat_merge(uint64_t bytes, int kind, const FeatWindow* __restrict__ win,
                                                              uint32_t* __restrict__ cand) {
  __shared__ uint32_t tk[kMergeSlots];
  __shared__ uint32_t tc[kMergeSlots];
  __shared__ uint32_t s_first[kWindows + 1];  // first entry of each window in the concatenated lists
  __shared__ uint32_t s_used;                 // claimed slots of the count table
  __shared__ uint32_t top[64];
  const Sample S = sample_of(bytes, kind);
  for (uint32_t i = threadIdx.x; i < kMergeSlots; i += blockDim.x) {
    tk[i] = 0xFFFFFFFFu;
    tc[i] = 0;
  }
  if (threadIdx.x == 0) {
    s_used = 0;
    uint32_t acc = 0;
    for (uint32_t w = 0; w < S.nseg; ++w) {
      s_first[w] = acc;
      acc += win[w].n_keys;
    }
    s_first[S.nseg] = acc;
  }
  __syncthreads();
  const uint32_t total = s_first[S.nseg];
  auto entry = [&](uint32_t i, uint32_t& k, uint32_t& c) {
    uint32_t lo = 0, hi = S.nseg;  // last window w with s_first[w] <= i
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (s_first[mid] <= i) lo = mid; else hi = mid;
    }
    k = win[lo].key[i - s_first[lo]];
    c = win[lo].cnt[i - s_first[lo]];
  };
  // 8 entries per thread loaded together (their loads in flight at once), then inserted
  for (uint32_t i0 = 0; i0 < total; i0 += 8 * blockDim.x) {
    uint32_t k[8], c[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint32_t i = i0 + u * blockDim.x + threadIdx.x;
      k[u] = 0;
      c[u] = 0;
      if (i < total) entry(i, k[u], c[u]);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (c[u] && (uint32_t)(hash_u32(k[u]) >> 60) == blockIdx.x) feat_insert(tk, tc, kMergeSlots, &s_used, k[u], c[u]);
  }
  __syncthreads();
  top64_of(tc, kMergeSlots, top);
  if (threadIdx.x < 64) cand[blockIdx.x * 64 + threadIdx.x] = top[threadIdx.x];
}

// Merges the windows' registers and sums and the partitions' largest counts,
// then estimates, top-64 counts and the 12 features. One workgroup.
__global__ __launch_bounds__(kFeatThreads) void k_feat_final(const uint8_t* __restrict__ in, uint64_t bytes, int kind, int op,
                                                              uint64_t key_range, uint32_t lds_budget,
                                                              const FeatWindow* __restrict__ win,
                                                              const uint32_t* __restrict__ cand, float* __restrict__ feats) {
  __shared__ uint32_t hll_all[kHllM];
  __shared__ uint32_t hll_half[kHllM];
  __shared__ uint32_t tc[kMergeParts * 64];  // the partitions' 64 largest counts
  __shared__ float red[2 * kFeatThreads / kWave];
  __shared__ unsigned long long s_n, s_len, s_len2;
  __shared__ uint32_t top[64];
  const Sample S = sample_of(bytes, kind);
  const uint64_t esz = S.esz, n_elem = S.n_elem;
  const bool whole = S.whole;
  for (uint32_t i = threadIdx.x; i < kMergeParts * 64; i += blockDim.x) tc[i] = cand[i];
  // register maxima: thread t takes word t of the two register arrays (4
  // registers a word) across the windows, loads of 8 windows in flight
  static_assert(2 * kHllM / 4 <= kFeatThreads, "one register word per thread");
  if (threadIdx.x < 2 * kHllM / 4) {
    const uint32_t t = threadIdx.x, half = t >= kHllM / 4, q = t % (kHllM / 4);
    uint32_t m[4] = {0, 0, 0, 0};
    for (uint32_t w0 = 0; w0 < S.nseg; w0 += 8) {
      uint32_t v[8];
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u) {
        const uint32_t w = w0 + u;
        v[u] = w < S.nseg ? reinterpret_cast<const uint32_t*>(half ? win[w].hll_half : win[w].hll_all)[q] : 0u;
      }
#pragma unroll
      for (uint32_t u = 0; u < 8; ++u)
#pragma unroll
        for (int b = 0; b < 4; ++b) m[b] = max(m[b], (v[u] >> (8 * b)) & 0xFFu);
    }
    uint32_t* dst = half ? hll_half : hll_all;
#pragma unroll
    for (int b = 0; b < 4; ++b) dst[4 * q + b] = m[b];
  }
  if (threadIdx.x == 0) {
    unsigned long long n = 0, l = 0, l2 = 0;
    for (uint32_t w = 0; w < S.nseg; ++w) {
      n += win[w].n;
      l += win[w].len;
      l2 += win[w].len2;
    }
    s_n = n;
    s_len = l;
    s_len2 = l2;
  }
  __syncthreads();
  const float D_all = hll_estimate(hll_all, red);
  const float D_half = hll_estimate(hll_half, red);
  top64_of(tc, kMergeParts * 64, top);
  if (threadIdx.x >= kWave) return;
  // Zipf exponent: least-squares slope of log count against log rank over the top counts
  float sx = 0, sy = 0, sxx = 0, sxy = 0, m = 0, top64 = 0;
  {
    const uint32_t r = lane_id();
    const float cnt = (float)top[r];
    top64 = cnt;
    if (cnt > 0.f) {
      const float x = logf((float)(r + 1)), y = logf(cnt);
      sx = x; sy = y; sxx = x * x; sxy = x * y; m = 1.f;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      sx += __shfl_xor(sx, o);
      sy += __shfl_xor(sy, o);
      sxx += __shfl_xor(sxx, o);
      sxy += __shfl_xor(sxy, o);
      m += __shfl_xor(m, o);
      top64 += __shfl_xor(top64, o);
    }
  }
  if (threadIdx.x != 0) return;
  const float n_s = (float)(s_n ? s_n : 1ull);
  // elements in the whole input (words: scaled from the sample's word density)
  const float sample_bytes = whole ? (float)bytes : (float)kWindows * (float)kWindowBytes;
  const float T = kind == 0 ? n_s * (float)bytes / fmaxf(sample_bytes, 1.f) : (float)n_elem;
  // growth exponent of distinct keys with sample size (Heaps' law), from half vs all
  float beta = (D_half > 0.f && D_all > D_half) ? log2f(D_all / D_half) : 0.f;
  beta = fminf(fmaxf(beta, 0.f), 1.f);
  float D_est = fmaxf(D_all, 1.f) * powf(fmaxf(T / n_s, 1.f), beta);
  D_est = fminf(D_est, fmaxf(T, 1.f));
  if (key_range) D_est = fminf(D_est, (float)key_range);
  const float den = m * sxx - sx * sx;
  const float zipf = (m >= 2.f && den > 0.f) ? -(m * sxy - sx * sy) / den : 0.f;
  const float mean_len = kind == 0 ? (float)s_len / n_s : (float)esz;
  const float var_len = kind == 0 ? fmaxf((float)s_len2 / n_s - mean_len * mean_len, 0.f) : 0.f;
  feats[0] = log2f(fmaxf((float)bytes, 1.f));
  feats[1] = kind == 0 ? 1.f : 0.f;
  feats[2] = kind == 0 ? 0.f : 1.f;
  feats[3] = op == 1 ? 1.f : 0.f;
  feats[4] = log2f(fmaxf(D_est, 1.f));
  feats[5] = zipf;
  feats[6] = (float)top[0] / n_s;
  feats[7] = top64 / n_s;
  feats[8] = mean_len;
  feats[9] = sqrtf(var_len);
  feats[10] = key_range ? log2f((float)key_range) : 0.f;
  feats[11] = log2f(fmaxf(D_est * 32.f, 1.f) / (float)lds_budget);  // table bytes at load 1/2, 16-byte slots
}

uint64_t feature_state_bytes() { return sizeof(FeatWindow) * kWindows + 4ull * kMergeParts * 64; }

hipError_t features_enqueue(const uint8_t* in, uint64_t bytes, int kind, int op, uint64_t key_range, uint32_t lds_budget,
                            float* feats, void* state, hipStream_t s) {
  FeatWindow* win = static_cast<FeatWindow*>(state);
  const uint64_t esz = kind == 0 ? 1 : (kind == 1 ? 4 : 8);
  const uint64_t n_elem = bytes / esz, wel = kWindowBytes / esz;
  const uint32_t nseg = n_elem <= (uint64_t)kWindows * wel ? (uint32_t)((n_elem + wel - 1) / wel) : kWindows;
  uint32_t* cand = reinterpret_cast<uint32_t*>(win + kWindows);
  if (nseg) hipLaunchKernelGGL(k_feat_sample, dim3(nseg), dim3(kSampThreads), 0, s, in, bytes, kind, win);
  hipLaunchKernelGGL(k_feat_merge, dim3(kMergeParts), dim3(kFeatThreads), 0, s, bytes, kind, win, cand);
  hipLaunchKernelGGL(k_feat_final, dim3(1), dim3(kFeatThreads), 0, s, in, bytes, kind, op, key_range, lds_budget, win, cand,
                     feats);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------
// MLP 12 -> 64 -> 64 -> 4 (float32), parameter layout W1[64][12] b1 W2[64][64] b2 W3[4][64] b3
// ----------------------------------------------------------------------------
constexpr int kIn = 12, kH = 64, kOut = 4;
constexpr int oW1 = 0, ob1 = oW1 + kH * kIn, oW2 = ob1 + kH, ob2 = oW2 + kH * kH, oW3 = ob2 + kH, ob3 = oW3 + kOut * kH;
constexpr int kParams = ob3 + kOut;
static_assert(kParams == 5252, "parameter count");

// One workgroup of 64 threads per sample.
__global__ __launch_bounds__(64) void k_mlp_fwd(const float* __restrict__ P, const float* __restrict__ X, uint32_t B,
                                                float* __restrict__ H1, float* __restrict__ H2, float* __restrict__ Y) {
  __shared__ float x[kIn], h1[kH], h2[kH];
  for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int j = threadIdx.x;
    if (j < kIn) x[j] = X[(uint64_t)b * kIn + j];
    __syncthreads();
    float z = P[ob1 + j];
    for (int i = 0; i < kIn; ++i) z = fmaf(P[oW1 + j * kIn + i], x[i], z);
    h1[j] = fmaxf(z, 0.f);
    __syncthreads();
    z = P[ob2 + j];
    for (int i = 0; i < kH; ++i) z = fmaf(P[oW2 + j * kH + i], h1[i], z);
    h2[j] = fmaxf(z, 0.f);
    __syncthreads();
    if (H1) H1[(uint64_t)b * kH + j] = h1[j];
    if (H2) H2[(uint64_t)b * kH + j] = h2[j];
    if (j < kOut) {
      float y = P[ob3 + j];
      for (int i = 0; i < kH; ++i) y = fmaf(P[oW3 + j * kH + i], h2[i], y);
      Y[(uint64_t)b * kOut + j] = y;
    }
    __syncthreads();
  }
}

// loss = sum M (Y - T)^2 / max(sum M, 1); dY = 2 M (Y - T) / max(sum M, 1). One workgroup.
__global__ __launch_bounds__(256) void k_mlp_dy(const float* __restrict__ Y, const float* __restrict__ T,
                                                const float* __restrict__ M, uint32_t B, float* __restrict__ dY,
                                                float* __restrict__ loss) {
  __shared__ float r1[256 / kWave], r2[256 / kWave];
  float sm = 0.f, sl = 0.f;
  for (uint32_t i = threadIdx.x; i < B * kOut; i += blockDim.x) {
    const float d = Y[i] - T[i];
    sm += M[i];
    sl += M[i] * d * d;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sm += __shfl_xor(sm, o);
    sl += __shfl_xor(sl, o);
  }
  if (lane_id() == 0) {
    r1[threadIdx.x / kWave] = sm;
    r2[threadIdx.x / kWave] = sl;
  }
  __syncthreads();
  float SM = 0.f, SL = 0.f;
  for (int w = 0; w < 256 / kWave; ++w) {
    SM += r1[w];
    SL += r2[w];
  }
  const float den = fmaxf(SM, 1.f);
  if (threadIdx.x == 0) *loss = SL / den;
  for (uint32_t i = threadIdx.x; i < B * kOut; i += blockDim.x) dY[i] = 2.f * M[i] * (Y[i] - T[i]) / den;
}

// dZ2 = (dY W3) * [H2 > 0], dZ1 = (dZ2 W2) * [H1 > 0]; one workgroup of 64 per sample.
__global__ __launch_bounds__(64) void k_mlp_dz(const float* __restrict__ P, const float* __restrict__ H1,
                                               const float* __restrict__ H2, const float* __restrict__ dY, uint32_t B,
                                               float* __restrict__ dZ1, float* __restrict__ dZ2) {
  __shared__ float dz2[kH], dy[kOut];
  for (uint32_t b = blockIdx.x; b < B; b += gridDim.x) {
    const int j = threadIdx.x;
    if (j < kOut) dy[j] = dY[(uint64_t)b * kOut + j];
    __syncthreads();
    float g = 0.f;
    for (int o = 0; o < kOut; ++o) g = fmaf(dy[o], P[oW3 + o * kH + j], g);
    const float d2 = H2[(uint64_t)b * kH + j] > 0.f ? g : 0.f;
    dz2[j] = d2;
    dZ2[(uint64_t)b * kH + j] = d2;
    __syncthreads();
    g = 0.f;
    for (int i = 0; i < kH; ++i) g = fmaf(dz2[i], P[oW2 + i * kH + j], g);
    dZ1[(uint64_t)b * kH + j] = H1[(uint64_t)b * kH + j] > 0.f ? g : 0.f;
    __syncthreads();
  }
}

// One thread per parameter: the sum over the batch of its chain-rule term.
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ X, const float* __restrict__ H1,
                                                  const float* __restrict__ H2, const float* __restrict__ dY,
                                                  const float* __restrict__ dZ1, const float* __restrict__ dZ2, uint32_t B,
                                                  float* __restrict__ G) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float s = 0.f;
  if (p < ob1) {  // W1[j][i] = sum_b dZ1[b][j] X[b][i]
    const int j = p / kIn, i = p % kIn;
    for (uint32_t b = 0; b < B; ++b) s = fmaf(dZ1[(uint64_t)b * kH + j], X[(uint64_t)b * kIn + i], s);
  } else if (p < oW2) {
    const int j = p - ob1;
    for (uint32_t b = 0; b < B; ++b) s += dZ1[(uint64_t)b * kH + j];
  } else if (p < ob2) {
    const int j = (p - oW2) / kH, i = (p - oW2) % kH;
    for (uint32_t b = 0; b < B; ++b) s = fmaf(dZ2[(uint64_t)b * kH + j], H1[(uint64_t)b * kH + i], s);
  } else if (p < oW3) {
    const int j = p - ob2;
    for (uint32_t b = 0; b < B; ++b) s += dZ2[(uint64_t)b * kH + j];
  } else if (p < ob3) {
    const int o = (p - oW3) / kH, i = (p - oW3) % kH;
    for (uint32_t b = 0; b < B; ++b) s = fmaf(dY[(uint64_t)b * kOut + o], H2[(uint64_t)b * kH + i], s);
  } else {
    const int o = p - ob3;
    for (uint32_t b = 0; b < B; ++b) s += dY[(uint64_t)b * kOut + o];
  }
  G[p] = s;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ m,
                                              float* __restrict__ v, uint32_t step, float lr, float b1, float b2, float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  const float g = G[p];
  const float mm = b1 * m[p] + (1.f - b1) * g;
  const float vv = b2 * v[p] + (1.f - b2) * g * g;
  m[p] = mm;
  v[p] = vv;
  const float mh = mm / (1.f - powf(b1, (float)step));
  const float vh = vv / (1.f - powf(b2, (float)step));
  P[p] -= lr * mh / (sqrtf(vh) + eps);
}

// Choose a container for one job: normalise its features, run the network,
// take the lowest output among the feasible containers (bit i of feas).
// Features outside [lo, hi] (the training range) give -1: the rule decides.
__global__ __launch_bounds__(64) void k_select(const float* __restrict__ feats, const float* __restrict__ norm,
                                               const float* __restrict__ P, uint32_t feas, int32_t* __restrict__ choice) {
  __shared__ float x[kIn], h1[kH], h2[kH], y[kOut];
  __shared__ int inside;
  const int j = threadIdx.x;
  if (j == 0) inside = 1;
  __syncthreads();
  if (j < kIn) {
    const float f = feats[j];
    if (!(f >= norm[32 + j] && f <= norm[48 + j])) inside = 0;
    x[j] = (f - norm[j]) / norm[16 + j];
  }
  __syncthreads();
  float z = P[ob1 + j];
  for (int i = 0; i < kIn; ++i) z = fmaf(P[oW1 + j * kIn + i], x[i], z);
  h1[j] = fmaxf(z, 0.f);
  __syncthreads();
  z = P[ob2 + j];
  for (int i = 0; i < kH; ++i) z = fmaf(P[oW2 + j * kH + i], h1[i], z);
  h2[j] = fmaxf(z, 0.f);
  __syncthreads();
  if (j < kOut) {
    float v = P[ob3 + j];
    for (int i = 0; i < kH; ++i) v = fmaf(P[oW3 + j * kH + i], h2[i], v);
    y[j] = v;
  }
  __syncthreads();
  if (j == 0) {
    int best = -1;
    for (int o = 0; o < kOut; ++o)
      if (((feas >> o) & 1u) && (best < 0 || y[o] < y[best])) best = o;
    *choice = inside ? best : -1;
  }
}

hipError_t select_enqueue(const float* feats, const float* norm, const float* P, uint32_t feas, int32_t* choice,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_select, dim3(1), dim3(64), 0, s, feats, norm, P, feas, choice);
  return hipGetLastError();
}

hipError_t mlp_forward_enqueue(const float* P, const float* X, uint32_t B, float* H1, float* H2, float* Y, hipStream_t s) {
  const uint32_t g = B < 4096 ? (B ? B : 1) : 4096;
  hipLaunchKernelGGL(k_mlp_fwd, dim3(g), dim3(64), 0, s, P, X, B, H1, H2, Y);
  return hipGetLastError();
}

hipError_t mlp_backward_enqueue(const float* P, const float* X, const float* H1, const float* H2, const float* Y,
                                const float* T, const float* M, uint32_t B, float* dY, float* dZ1, float* dZ2, float* loss,
                                float* G, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_dy, dim3(1), dim3(256), 0, s, Y, T, M, B, dY, loss);
  const uint32_t g = B < 4096 ? (B ? B : 1) : 4096;
  hipLaunchKernelGGL(k_mlp_dz, dim3(g), dim3(64), 0, s, P, H1, H2, dY, B, dZ1, dZ2);
  hipLaunchKernelGGL(k_mlp_grad, dim3((kParams + 255) / 256), dim3(256), 0, s, X, H1, H2, dY, dZ1, dZ2, B, G);
  return hipGetLastError();
}

hipError_t adam_enqueue(float* P, const float* G, float* m, float* v, uint32_t step, float lr, float b1, float b2, float eps,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_adam, dim3((kParams + 255) / 256), dim3(256), 0, s, P, G, m, v, step, lr, b1, b2, eps);
  return hipGetLastError();
}

}  // namespace mr
