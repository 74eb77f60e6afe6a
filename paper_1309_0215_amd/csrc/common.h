// Shared device helpers and job descriptors of the MapReduce hot path (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "jobs.h"

#define MR_DEV __device__ __forceinline__
// Global address space: a pointer loaded from a descriptor is generic, and
// generic (flat) accesses count against the LDS wait counter too, so every
// LDS wait would also wait for outstanding global loads. Casting to the
// global space makes them global_* instructions.
#define MR_GLOBAL __attribute__((address_space(1)))

namespace mr {

template <typename T>
MR_DEV MR_GLOBAL T* gp(T* p) {
  return (MR_GLOBAL T*)p;
}

typedef uint32_t gu32x4 __attribute__((ext_vector_type(4)));

// 16-byte global load / store at a 16-byte aligned address.
MR_DEV uint4 gload16(const void* p) {
  const gu32x4 v = *gp(reinterpret_cast<const gu32x4*>(p));
  return make_uint4(v[0], v[1], v[2], v[3]);
}

MR_DEV void gstore16(void* p, uint4 x) {
  gu32x4 v;
  v[0] = x.x;
  v[1] = x.y;
  v[2] = x.z;
  v[3] = x.w;
  *gp(reinterpret_cast<gu32x4*>(p)) = v;
}

constexpr int kWave = 64;
constexpr uint32_t kXcds = 8;  // accelerator complex dies; workgroups are dispatched to them in turn

// ---------------------------------------------------------------------------
// hashing (the hash only places keys; equality is always decided on full keys)
// ---------------------------------------------------------------------------
MR_DEV uint64_t fmix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

MR_DEV uint64_t rotl64(uint64_t x, int r) { return (x << r) | (x >> (64 - r)); }

// Hash of one 16-byte block (little-endian words w0, w1) chained onto h.
MR_DEV uint64_t hash_block(uint64_t h, uint64_t w0, uint64_t w1) {
  return fmix64(h ^ (w0 * 0x9E3779B97F4A7C15ULL) ^ rotl64(w1 * 0xC2B2AE3D27D4EB4FULL, 29));
}

MR_DEV uint64_t hash_seed(uint32_t len) { return 0x27D4EB2F165667C5ULL ^ ((uint64_t)len * 0x165667B19E3779F9ULL); }

MR_DEV uint64_t hash_u32(uint32_t k) { return fmix64((uint64_t)k * 0x9E3779B97F4A7C15ULL + 0x632BE59BD9B4E019ULL); }

// ---------------------------------------------------------------------------
// separators: the six ASCII whitespace bytes 0x09..0x0D and 0x20
// ---------------------------------------------------------------------------
// Lane l receives lane l + 1's value (lane 63 keeps `fill`), and lane l
// receives lane l - 1's value (lane 0 keeps `fill`): DPP whole-wave shifts.
MR_DEV uint32_t from_next_lane(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x130, 0xF, 0xF, false);  // wave_shl:1
}
MR_DEV uint32_t from_prev_lane(uint32_t v, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)v, 0x138, 0xF, 0xF, false);  // wave_shr:1
}

// Inclusive prefix sum over the 64 lanes with DPP: shifts within rows of 16
// lanes, then the last lane of row 0 (row 2) is broadcast into row 1 (row 3),
// and the last lane of row 1 into rows 2 and 3. No LDS traffic.
MR_DEV uint32_t wave_incl_scan(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

MR_DEV bool is_sep_byte(uint32_t b) { return b == 0x20u || (b - 0x09u) < 5u; }

// Separator flags of a little-endian word: bit 7 of byte i is set when byte i
// is a separator (branch-free SWAR; bytes >= 0x80 are word bytes, and the
// 0x7F mask keeps the byte sums below from carrying into the next byte).
MR_DEV uint32_t sep_flags4(uint32_t w) {
  const uint32_t t = w & 0x7F7F7F7Fu;
  const uint32_t not20 = (t ^ 0x20202020u) + 0x7F7F7F7Fu;  // bit 7: t != 0x20
  const uint32_t ge9 = t + 0x77777777u;                    // bit 7: t >= 0x09
  const uint32_t ge14 = t + 0x72727272u;                   // bit 7: t >= 0x0E
  const uint32_t word = not20 & ~(ge9 & ~ge14);            // bit 7: neither 0x20 nor 0x09..0x0D
  return ~(word | w) & 0x80808080u;
}

// Flags of two words (bytes 0..7) gathered into bits 0..7. The flag bits sit
// at 0, 8, 16, 24 (first word) and 4, 12, 20, 28 (second); multiplying by
// 1 + 2^7 + 2^14 + 2^21 puts byte i's flag at bit 21 + i, and no two partial
// products share a bit, so nothing carries.
MR_DEV uint32_t gather8(uint32_t f0, uint32_t f1) {
  const uint32_t x = (f0 >> 7) | (f1 >> 3);
  return (x * 0x00204081u) >> 21 & 0xFFu;
}

// 4-bit mask (bit i = byte i of w is a separator).
MR_DEV uint32_t sep_mask4(uint32_t w) { return gather8(sep_flags4(w), 0u) & 0xFu; }

// 16-bit mask of a 16-byte chunk (bit i = byte i is a separator).
MR_DEV uint32_t sep_mask16(uint32_t a, uint32_t b, uint32_t c, uint32_t d) {
  return gather8(sep_flags4(a), sep_flags4(b)) | (gather8(sep_flags4(c), sep_flags4(d)) << 8);
}

// bytes [0, n) of a little-endian word kept, the rest zeroed (n in 0..4)
MR_DEV uint32_t keep_bytes(uint32_t w, int n) {
  return n >= 4 ? w : (n <= 0 ? 0u : (w & ((1u << (8 * n)) - 1u)));
}

MR_DEV uint32_t bswap32(uint32_t x) { return __builtin_bswap32(x); }

// ---------------------------------------------------------------------------
// wave helpers
// ---------------------------------------------------------------------------
MR_DEV uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

MR_DEV uint64_t ballot(bool p) { return __ballot(p); }

MR_DEV uint32_t popc64(uint64_t m) { return (uint32_t)__popcll(m); }

// Number of set bits of m below this lane.
MR_DEV uint32_t mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// One slot per calling lane from a counter, with one atomic per wave: safe
// under divergence (only the calling lanes take part).
MR_DEV unsigned long long wave_claim(unsigned long long* counter) {
  const uint64_t active = __ballot(true);
  const int leader = __ffsll((long long)active) - 1;
  unsigned long long base = 0;
  if ((int)lane_id() == leader) base = atomicAdd(counter, (unsigned long long)popc64(active));
  base = __shfl(base, leader);
  return base + mbcnt(active);
}

}  // namespace mr
