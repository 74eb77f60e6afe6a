// Oracle: a plain, sequential CPU MapReduce used ONLY as test infrastructure.
//
// Nothing in the product path may include, link or call this file. It shares
// no code with the GPU library: tests, the smoke check and the CPU-baseline leg
// of the benchmark call it through ctypes.
//
// What it computes follows the paper's programming model (Section II-A): the
// map function is applied to every element of the input array and emits
// intermediate (key, value) pairs; the reduce function is then applied to all
// pairs that share a key; the result pairs are output in key order (ordering is
// optional in the paper; it is always done here).
//
// The reduce containers are the two the paper names (Section III-A): an
// ordered associative container (std::map) for arbitrary keys, and a plain
// array for integer keys in a fixed range (the RGB histogram). No blocking,
// fusion or reordering is applied: one element at a time, in input order.
//
// Readings of points the paper leaves open (the same readings the GPU path
// implements):
//   * A word is a maximal run of non-separator bytes. Separators are the six
//     ASCII whitespace bytes 0x09..0x0D and 0x20. Every other byte (including
//     NUL and bytes >= 0x80) is a word byte. No case folding.
//   * Optional record offsets u64[n+1] cut the input into records
//     [off[i], off[i+1]); a record boundary ends a word. Bytes outside
//     [off[0], off[n]) are ignored. With no offsets the input is one record.
//   * Word keys are ordered bytewise as unsigned bytes, a proper prefix first.
//   * COUNT values are reported as 64-bit here; callers compare against the
//     32-bit GPU output and flag counts above 2^32-1.
#include <cstdint>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace {

bool is_sep(uint8_t b) { return b == 0x20 || (b >= 0x09 && b <= 0x0D); }

struct WordsResult {
  std::vector<uint8_t> key_bytes;
  std::vector<uint64_t> key_offsets;  // n+1
  std::vector<uint64_t> values;       // n
};

struct U32Result {
  std::vector<uint32_t> keys;
  std::vector<uint64_t> values;
};

}  // namespace

extern "C" {

// ---------------------------------------------------------------------------
// Word count (Section II-A model; hash-table container of Section III-A).
// map: for each word in each record emit (word, 1); reduce: sum per word.
// Returns an opaque handle, or NULL when the record offsets are malformed
// (not non-decreasing, or past the end of the input).
// ---------------------------------------------------------------------------
void* oracle_words_run(const uint8_t* buf, uint64_t n, const uint64_t* rec_off, uint64_t n_rec) {
  std::map<std::vector<uint8_t>, uint64_t> m;
  std::vector<std::pair<uint64_t, uint64_t>> records;
  if (rec_off == nullptr) {
    records.push_back({0, n});
  } else {
    for (uint64_t r = 0; r < n_rec; ++r) {
      if (rec_off[r] > rec_off[r + 1] || rec_off[r + 1] > n) return nullptr;
      records.push_back({rec_off[r], rec_off[r + 1]});
    }
  }
  for (auto& rec : records) {
    uint64_t i = rec.first, e = rec.second;
    while (i < e) {
      while (i < e && is_sep(buf[i])) ++i;          // skip separators
      uint64_t j = i;
      while (j < e && !is_sep(buf[j])) ++j;         // one word [i, j)
      if (j > i) {
        std::vector<uint8_t> key(buf + i, buf + j);  // map emits (word, 1)
        m[key] += 1;                                 // reduce: sum
      }
      i = j;
    }
  }
  auto* r = new WordsResult();
  r->key_offsets.push_back(0);
  for (auto& kv : m) {  // std::map iterates in key order
    r->key_bytes.insert(r->key_bytes.end(), kv.first.begin(), kv.first.end());
    r->key_offsets.push_back(r->key_bytes.size());
    r->values.push_back(kv.second);
  }
  return r;
}

uint64_t oracle_words_n(void* h) { return static_cast<WordsResult*>(h)->values.size(); }
uint64_t oracle_words_bytes(void* h) { return static_cast<WordsResult*>(h)->key_bytes.size(); }

void oracle_words_copy(void* h, uint8_t* key_bytes, uint64_t* key_offsets, uint64_t* values) {
  auto* r = static_cast<WordsResult*>(h);
  if (!r->key_bytes.empty()) std::memcpy(key_bytes, r->key_bytes.data(), r->key_bytes.size());
  std::memcpy(key_offsets, r->key_offsets.data(), r->key_offsets.size() * sizeof(uint64_t));
  if (!r->values.empty()) std::memcpy(values, r->values.data(), r->values.size() * sizeof(uint64_t));
}

void oracle_words_free(void* h) { delete static_cast<WordsResult*>(h); }

// ---------------------------------------------------------------------------
// Integer keys (Section II-A model; containers of Section III-A).
// map: element i emits (keys[i], vals[i]) (vals == NULL means value 1);
// reduce op: 0 = COUNT, 1 = SUM, 2 = MIN, 3 = MAX.
// ---------------------------------------------------------------------------
void* oracle_u32_run(const uint32_t* keys, const uint32_t* vals, uint64_t n, int op) {
  std::map<uint32_t, uint64_t> m;
  for (uint64_t i = 0; i < n; ++i) {
    uint64_t v = vals ? vals[i] : 1;
    auto it = m.find(keys[i]);
    if (it == m.end()) {
      m.emplace(keys[i], op == 0 ? 1 : v);
      continue;
    }
    switch (op) {
      case 0: it->second += 1; break;
      case 1: it->second += v; break;
      case 2: if (v < it->second) it->second = v; break;
      case 3: if (v > it->second) it->second = v; break;
    }
  }
  auto* r = new U32Result();
  for (auto& kv : m) {
    r->keys.push_back(kv.first);
    r->values.push_back(kv.second);
  }
  return r;
}

uint64_t oracle_u32_n(void* h) { return static_cast<U32Result*>(h)->keys.size(); }

void oracle_u32_copy(void* h, uint32_t* keys, uint64_t* values) {
  auto* r = static_cast<U32Result*>(h);
  if (!r->keys.empty()) {
    std::memcpy(keys, r->keys.data(), r->keys.size() * sizeof(uint32_t));
    std::memcpy(values, r->values.data(), r->values.size() * sizeof(uint64_t));
  }
}

void oracle_u32_free(void* h) { delete static_cast<U32Result*>(h); }

// ---------------------------------------------------------------------------
// RGB histogram (Table of benchmark applications: Histogram, array container).
// Pixel p has bytes (R, G, B) at 3p, 3p+1, 3p+2; map emits ((c, byte), 1) for
// each channel c; reduce sums into a 3 x 256 array. A trailing partial pixel
// is not a pixel; callers reject lengths that are not a multiple of 3.
// ---------------------------------------------------------------------------
void oracle_rgb_run(const uint8_t* buf, uint64_t n, uint64_t* bins /* [3*256] */) {
  for (int i = 0; i < 3 * 256; ++i) bins[i] = 0;
  for (uint64_t p = 0; p + 3 <= n; p += 3)
    for (int c = 0; c < 3; ++c) bins[c * 256 + buf[p + c]] += 1;
}

// ---------------------------------------------------------------------------
// Bloom filter build (Table of benchmark applications: Bloom Filter, large
// array container; Section III-E). map: each k-mer of the DNA input, taken
// only when all of its k bytes are A, C, G or T, emits h bit positions;
// reduce: OR into one array of m bits. Readings (the paper names the
// application but not its hashing):
//   v     = k-mer packed two bits per base, A 0, C 1, G 2, T 3, first base
//           in the most significant position
//   x     = fmix64(v), the 64-bit finaliser of MurmurHash3
//   g_i   = (low32(x) + i * (high32(x) | 1)) mod 2^32, i = 0 .. h-1
//           (double hashing, Kirsch and Mitzenmacher)
//   pos_i = floor(g_i * m / 2^32)
// Every k-mer is recomputed from its k bytes; nothing is rolled or reused.
// ---------------------------------------------------------------------------
uint64_t oracle_fmix64(uint64_t x) {
  // MurmurHash3's fmix64: xor-shift by 33, multiply, xor-shift, multiply, xor-shift
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

static int dna_code(uint8_t b) {
  switch (b) {
    case 'A': return 0;
    case 'C': return 1;
    case 'G': return 2;
    case 'T': return 3;
    default: return -1;
  }
}

// words: ceil(m / 32) uint32, cleared here; bit b lives in bit b % 32 of word b / 32.
// Returns the number of k-mers that emitted positions.
uint64_t oracle_bloom_run(const uint8_t* buf, uint64_t n, uint32_t k, uint32_t h, uint64_t m, uint32_t* words) {
  const uint64_t n_words = (m + 31) / 32;
  for (uint64_t w = 0; w < n_words; ++w) words[w] = 0;
  uint64_t emitted = 0;
  for (uint64_t s = 0; s + k <= n; ++s) {
    uint64_t v = 0;
    bool valid = true;
    for (uint32_t q = 0; q < k; ++q) {
      const int c = dna_code(buf[s + q]);
      if (c < 0) {
        valid = false;
        break;
      }
      v = v * 4 + (uint64_t)c;
    }
    if (!valid) continue;
    ++emitted;
    const uint64_t x = oracle_fmix64(v);
    const uint32_t a = (uint32_t)(x & 0xffffffffu);
    const uint32_t b = (uint32_t)(x >> 32) | 1u;
    for (uint32_t i = 0; i < h; ++i) {
      const uint32_t g = a + i * b;  // mod 2^32 by unsigned wrap-around
      const uint64_t pos = ((uint64_t)g * m) >> 32;
      words[pos / 32] |= 1u << (pos % 32);
    }
  }
  return emitted;
}

// ---------------------------------------------------------------------------
// Reverse Index (Table of benchmark applications: Reverse Index, hash table
// container). Records are files, numbered from 0. map: every link emits
// (URL, file); reduce: per URL, the number of links and the ascending list of
// distinct files that hold one. Reading of "link" (the paper does not define
// it): the nine bytes <a href=" followed by 1 to 4095 bytes other than a
// double quote and then a double quote, all inside one record; the URL is the
// bytes between the quotes. Matching is exact (case and spacing included).
// Output in unsigned bytewise URL order, a proper prefix first.
// ---------------------------------------------------------------------------
struct LinksResult {
  std::vector<uint8_t> key_bytes;
  std::vector<uint64_t> key_offsets;   // n+1
  std::vector<uint64_t> counts;        // links per URL
  std::vector<uint64_t> list_offsets;  // n+1
  std::vector<uint32_t> ids;           // files, ascending within each URL
};

void* oracle_links_run(const uint8_t* buf, uint64_t n, const uint64_t* rec_off, uint64_t n_rec) {
  static const uint8_t kMarker[9] = {'<', 'a', ' ', 'h', 'r', 'e', 'f', '=', '"'};
  const uint64_t kMaxUrl = 4095;
  uint64_t one[2] = {0, n};
  if (!rec_off) {
    rec_off = one;
    n_rec = 1;
  }
  for (uint64_t r = 0; r < n_rec; ++r)
    if (rec_off[r] > rec_off[r + 1] || rec_off[r + 1] > n) return nullptr;
  struct Entry {
    uint64_t count = 0;
    std::vector<uint32_t> files;  // appended in file order, so ascending
  };
  std::map<std::string, Entry> index;
  for (uint64_t r = 0; r < n_rec; ++r) {
    const uint64_t lo = rec_off[r], hi = rec_off[r + 1];
    for (uint64_t p = lo; p + 9 <= hi; ++p) {
      if (std::memcmp(buf + p, kMarker, 9) != 0) continue;
      const uint64_t u = p + 9;
      uint64_t q = u;
      while (q < hi && buf[q] != '"' && q - u <= kMaxUrl) ++q;
      if (q >= hi || buf[q] != '"') continue;  // no closing quote in the record (or URL too long)
      const uint64_t len = q - u;
      if (len < 1 || len > kMaxUrl) continue;
      Entry& e = index[std::string(reinterpret_cast<const char*>(buf + u), len)];
      e.count += 1;
      if (e.files.empty() || e.files.back() != (uint32_t)r) e.files.push_back((uint32_t)r);
    }
  }
  auto* res = new LinksResult();
  res->key_offsets.push_back(0);
  res->list_offsets.push_back(0);
  for (auto& kv : index) {  // std::string compares as unsigned bytes (char_traits<char>::compare uses memcmp)
    res->key_bytes.insert(res->key_bytes.end(), kv.first.begin(), kv.first.end());
    res->key_offsets.push_back(res->key_bytes.size());
    res->counts.push_back(kv.second.count);
    res->ids.insert(res->ids.end(), kv.second.files.begin(), kv.second.files.end());
    res->list_offsets.push_back(res->ids.size());
  }
  return res;
}

uint64_t oracle_links_n(void* h) { return static_cast<LinksResult*>(h)->counts.size(); }
uint64_t oracle_links_bytes(void* h) { return static_cast<LinksResult*>(h)->key_bytes.size(); }
uint64_t oracle_links_ids(void* h) { return static_cast<LinksResult*>(h)->ids.size(); }

void oracle_links_copy(void* h, uint8_t* key_bytes, uint64_t* key_offsets, uint64_t* counts, uint64_t* list_offsets,
                       uint32_t* ids) {
  auto* r = static_cast<LinksResult*>(h);
  if (!r->key_bytes.empty()) std::memcpy(key_bytes, r->key_bytes.data(), r->key_bytes.size());
  std::memcpy(key_offsets, r->key_offsets.data(), r->key_offsets.size() * sizeof(uint64_t));
  if (!r->counts.empty()) std::memcpy(counts, r->counts.data(), r->counts.size() * sizeof(uint64_t));
  std::memcpy(list_offsets, r->list_offsets.data(), r->list_offsets.size() * sizeof(uint64_t));
  if (!r->ids.empty()) std::memcpy(ids, r->ids.data(), r->ids.size() * sizeof(uint32_t));
}

void oracle_links_free(void* h) { delete static_cast<LinksResult*>(h); }

}  // extern "C"
