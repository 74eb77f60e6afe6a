// One k-means (Lloyd) step on gfx950: map = nearest centroid, reduce = per-
// cluster sum and count (array container over the k clusters).
//
// Assignment (d = 32, k = 64): the scores s_j = |c_j|^2 - 2 <x, c_j> come from
// a contraction on the matrix cores. Points and centroids are split exactly
// into three bfloat16 pieces each (x = xh + xm + xl); the six largest of the
// nine piece products (all but xm.cl, xl.cm, xl.cl, which together stay below
// 2^-20 |x| |c|) are accumulated in float32 by v_mfma_f32_32x32x16_bf16:
// A = 32 centroids x 16 dims, B = 16 dims x 32 points, two steps cover
// d = 32, two centroid blocks cover k = 64. Each lane ends with one point's
// scores for 32 centroids; lanes l and l ^ 32 hold the other 32. The argmin
// takes the lowest index on equal scores. When the float32 gap between the
// best and the second best score is within a rounding bound eps(x) (which
// covers the dropped products), the decision is made again in float64 from
// the direct form sum_t (x_t - c_t)^2.
//
// Update: the per-cluster sums are a second contraction on the matrix cores
// (one-hot assignment x points). Each float32 coordinate is split exactly into
// three bfloat16 pieces (x = hi + mid + lo), so the one-hot products are
// exact and the contraction runs on the bfloat16 unit
// (v_mfma_f32_32x32x16_bf16) with float32 accumulation, as the float32
// contraction did. The float32 sums stay in the accumulators for at most 16
// groups of 32 points per wave and are then added into float64 LDS sums; the
// per-workgroup float64 partials are added in a fixed order at the end.
#include "common.h"
#include "launch.h"

namespace mr {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

MR_DEV __bf16 bf16_bits(uint32_t hi16) { return __builtin_bit_cast(__bf16, (unsigned short)hi16); }

// x = hi + mid + lo exactly (finite x above the float32 subnormal range):
// hi keeps the top 8 significant bits, mid the next 8 of the remainder, and
// the last remainder has at most 8 significant bits left.
MR_DEV void split_bf16x3(float x, __bf16& hi, __bf16& mid, __bf16& lo) {
  const uint32_t u0 = __float_as_uint(x);
  const float r1 = x - __uint_as_float(u0 & 0xFFFF0000u);
  const uint32_t u1 = __float_as_uint(r1);
  const float r2 = r1 - __uint_as_float(u1 & 0xFFFF0000u);
  hi = bf16_bits(u0 >> 16);
  mid = bf16_bits(u1 >> 16);
  lo = bf16_bits(__float_as_uint(r2) >> 16);
}

constexpr int kKmThreads = 256;  // 4 waves

// Nonzero float32 magnitudes below 2^-100 (bit patterns 1 .. kTinyBits - 1):
// their bfloat16 pieces can fall below the normal range, where the split
// into pieces is no longer exact, so the matrix-core path is not used.
constexpr uint32_t kTinyBits = 0x0D800000u;  // 2^-100

// Squared norms of the centroids (rounded to float32) and max |c| (float64);
// *tiny is set when a centroid has a nonzero coordinate below 2^-100.
__global__ __launch_bounds__(256) void k_km_prep(const float* __restrict__ C, uint32_t k, uint32_t d, float* __restrict__ cn,
                                                 double* __restrict__ cmax, unsigned long long* __restrict__ tiny) {
  __shared__ double m[256];
  double best = 0.0;
  bool small = false;
  for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) {
    double s = 0.0;
    for (uint32_t t = 0; t < d; ++t) {
      const float f = C[(uint64_t)j * d + t];
      const uint32_t b = __float_as_uint(f) & 0x7FFFFFFFu;
      small |= b != 0u && b < kTinyBits;
      const double v = f;
      s += v * v;
    }
    cn[j] = (float)s;
    best = s > best ? s : best;
  }
  if (small) atomicOr(tiny, 1ull);
  m[threadIdx.x] = best;
  __syncthreads();
  if (threadIdx.x == 0) {
    double b = 0.0;
    for (int i = 0; i < 256; ++i) b = m[i] > b ? m[i] : b;
    *cmax = sqrt(b);
  }
}

// float64 direct-form squared distance (the definition of the step).
MR_DEV double dist64(const float* __restrict__ x, const float* __restrict__ c, uint32_t d) {
  double s = 0.0;
#pragma unroll 1
  for (uint32_t t = 0; t < d; ++t) {
    const double q = (double)x[t] - (double)c[t];
    s += q * q;
  }
  return s;
}

// Assignment + local sums for d = 32, k = 64.
constexpr int kKmFlushIters = 16;  // wave iterations between float32 -> float64 flushes of the sums

MR_DEV void load_group(const float* __restrict__ X, uint64_t N, uint64_t g, uint64_t groups, uint32_t col, uint32_t h,
                       float (&xs)[16]) {
  const uint64_t p = g * 32 + col;
  if (g < groups && p < N) {
    // dims 8h..8h+7 (xs[0..7]) and 16+8h..16+8h+7 (xs[8..15])
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4* src = reinterpret_cast<const f32x4*>(X + p * 32 + 16 * (q / 2) + 8 * h + 4 * (q % 2));
      const f32x4 v = __builtin_nontemporal_load(src);
      xs[4 * q + 0] = v.x;
      xs[4 * q + 1] = v.y;
      xs[4 * q + 2] = v.z;
      xs[4 * q + 3] = v.w;
    }
  } else {
#pragma unroll
    for (int s = 0; s < 16; ++s) xs[s] = 0.f;
  }
}

// Each wave takes groups of 32 points. Lane (col, h) holds dims 16h..16h+15
// of point col (B operand of the score contraction) and centroid rows col and
// 32 + col come from LDS (A operand). After the argmin, the per-cluster sums
// are a second contraction S[c][d] += sum_p [a_p = c] x[p][d]: the one-hot
// assignment is the A operand (clusters x points), the points transposed
// through LDS are the B operand (points x dims), and the float32 sums stay in
// the accumulators until they are flushed into float64 LDS sums.
__global__ __launch_bounds__(kKmThreads) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_km_mfma(const float* __restrict__ X, uint64_t N, const float* __restrict__ C,
                                                        const float* __restrict__ cn_g, const double* __restrict__ cmax_g,
                                                        int32_t* __restrict__ assign, double* __restrict__ part_sum,
                                                        uint32_t* __restrict__ part_cnt, unsigned long long* __restrict__ n_recheck,
                                                        unsigned long long* __restrict__ tiny) {
  constexpr int D = 32, K = 64, W = kKmThreads / kWave;
  __shared__ double s64[K * D];
  __shared__ uint32_t scnt[K];
  __shared__ float sC[K * D];
  __shared__ float sCn[K];
  // centroid pieces (hi, mid, lo) as A operands: sCp[piece][row][...] holds
  // the row's four 8-dim chunks, chunk c at position c ^ ((row / 4) % 4), so
  // that the 16 lanes of one 16-byte read (rows r..r+15) meet 16 different
  // bank groups
  __shared__ __bf16 sCp[3][K][D];
  // per wave: x transposed, xt[w][row(d)][p] = x[p][d] with row(d) =
  // 16 (d / 16) + 2 (d % 8) + (d / 8) % 2 (the two lanes of a pair write rows
  // of different parity, hence different banks), and the assignments,
  // ab[w][p] = a_p (-1 for no point)
  __shared__ float xt[W][32][32];
  __shared__ int32_t ab[W][32];
  for (int i = threadIdx.x; i < K * D; i += blockDim.x) {
    s64[i] = 0.0;
    sC[i] = C[i];
    const int r = i / D, e = ((((i % D) / 8) ^ ((r / 4) % 4)) * 8) + i % 8;
    split_bf16x3(C[i], sCp[0][r][e], sCp[1][r][e], sCp[2][r][e]);
  }
  if (threadIdx.x < K) {
    scnt[threadIdx.x] = 0;
    sCn[threadIdx.x] = cn_g[threadIdx.x];
  }
  __syncthreads();

  const uint32_t lane = lane_id();
  const uint32_t wv = threadIdx.x / kWave;
  const uint32_t h = lane >> 5;     // which half of the dims (0: 0..15, 1: 16..31)
  const uint32_t col = lane & 31u;  // point within the 32-point group / centroid row within a block
  const float cmax = (float)*cmax_g;
  const float u = 5.9604645e-08f;                     // 2^-24
  // float32 accumulation of the piece products: 12 instructions of 16 products
  // each per score, counted as 48 sequential additions (with margin)
  const float gam = 48.f * u / (1.f - 48.f * u);
  const float drop = 9.5367432e-07f;                  // 2^-20: the three dropped piece products
  const float e_c = 8.f * u * cmax * cmax;            // centroid-norm rounding, both scores, x2 margin
  const float e_x = 8.f * (gam + u + drop) * cmax;    // times |x|: dot products and the subtraction

  const uint32_t waves_total = gridDim.x * W;
  const uint32_t wave_g = blockIdx.x * W + wv;
  const uint64_t groups = (N + 31) / 32;
  const uint64_t iters = (groups + waves_total - 1) / waves_total;  // uniform across the grid
  unsigned long long rechecks = 0;
  uint32_t tmin = 0xFFFFFFFFu;  // min over this lane's coordinates of (|bits| - 1): zero stays above every tiny value
  f32x16 sum0 = {}, sum1 = {};  // cluster rows 0..31 and 32..63 x dims (float32, since the last flush)

  float xs[16], xn[16];
  load_group(X, N, wave_g, groups, col, h, xs);
  for (uint64_t it = 0; it < iters; ++it) {
    const uint64_t g = it * waves_total + wave_g;
    const uint64_t p = g * 32 + col;
    const bool valid = g < groups && p < N;
    // the next group's loads are in flight while this group is computed
    load_group(X, N, g + waves_total, groups, col, h, xn);
    f32x16 acc0 = {}, acc1 = {};
#pragma unroll
    for (int kc = 0; kc < 2; ++kc) {
      // B: dims 16 kc + 8h + j of point col (xs[8 kc + j]) as three pieces
      bf16x8 xh, xm, xl;
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        __bf16 vh, vm, vl;
        split_bf16x3(xs[8 * kc + j], vh, vm, vl);
        xh[j] = vh;
        xm[j] = vm;
        xl[j] = vl;
      }
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        // A: centroid row blk * 32 + col, the same 8 dims
        const uint32_t row = blk * 32 + col, pc = ((2 * kc + h) ^ ((row / 4) % 4)) * 8;
        const bf16x8 ch = *reinterpret_cast<const bf16x8*>(&sCp[0][row][pc]);
        const bf16x8 cm = *reinterpret_cast<const bf16x8*>(&sCp[1][row][pc]);
        const bf16x8 cl = *reinterpret_cast<const bf16x8*>(&sCp[2][row][pc]);
        f32x16 acc = blk ? acc1 : acc0;
        // smaller products first
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cm, xm, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cl, xh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, xl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(cm, xh, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, xm, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ch, xh, acc, 0, 0, 0);
        if (blk) acc1 = acc; else acc0 = acc;
      }
    }
#pragma unroll
    for (int t = 0; t < 16; ++t) {
      const uint32_t b = (__float_as_uint(xs[t]) & 0x7FFFFFFFu) - 1u;
      tmin = b < tmin ? b : tmin;
    }
    // |x| for the bound
    float nx = 0.f;
#pragma unroll
    for (int s = 0; s < 16; ++s) nx = fmaf(xs[s], xs[s], nx);
    nx += __shfl_xor(nx, 32);
    nx = sqrtf(nx);
    // scores of this lane's 32 rows, then best and second best; rows are
    // visited in increasing index order, so a strict < keeps the lowest index
    float sc[32];
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r)
        sc[b * 16 + r] = sCn[b * 32 + 8 * (r / 4) + 4 * (int)h + (r % 4)] - 2.f * (b ? acc1[r] : acc0[r]);
    float b1 = INFINITY, b2 = INFINITY;
    int i1 = 0;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int idx = b * 32 + 8 * (r / 4) + 4 * (int)h + (r % 4);
        const float v = sc[b * 16 + r];
        const bool better = v < b1;
        b2 = better ? b1 : (v < b2 ? v : b2);
        i1 = better ? idx : i1;
        b1 = better ? v : b1;
      }
    }
    // combine with the partner lane (other 32 rows of the same point)
    const float o1 = __shfl_xor(b1, 32), o2 = __shfl_xor(b2, 32);
    const int oi = __shfl_xor(i1, 32);
    const bool other = o1 < b1 || (o1 == b1 && oi < i1);
    const float best = other ? o1 : b1;
    const float second = other ? (b1 < o2 ? b1 : o2) : (b2 < o1 ? b2 : o1);
    int bi = other ? oi : i1;
    // Near tie: every float32 score is within eps/2 of its exact value, so the
    // exact argmin is among the rows scoring <= best + eps. Those candidates
    // (usually two) are decided again in float64 from the direct form; both
    // lanes of the pair take part, each for its own rows.
    const float eps = e_c + e_x * nx;
    const bool need = valid && !(second - best > eps);
    if (__any(need)) {
      uint32_t cand = 0;
      if (need) {
        const float thr = best + eps;
#pragma unroll
        for (int t = 0; t < 32; ++t) cand |= (sc[t] <= thr ? 1u : 0u) << t;
      }
      // the partner's half of the point: this lane then holds all 32 dims
      float xo[16];
#pragma unroll
      for (int s = 0; s < 16; ++s) xo[s] = __shfl_xor(xs[s], 32);
      double bd = INFINITY;
      int bj = 0x7fffffff;
#pragma unroll 1
      while (cand) {  // rows in increasing index order: strict < keeps the lowest index
        const int bit = __builtin_ctz(cand);
        cand &= cand - 1u;
        const int rr = bit & 15;
        const int idx = (bit >> 4) * 32 + 8 * (rr / 4) + 4 * (int)h + (rr % 4);
        // own dims first, then the partner's: lane half g holds dims 8g..8g+7
        // and 16+8g..16+8g+7, in xs order
        double dj = 0.0;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const uint32_t g = q < 4 ? h : 1u - h;
          const f32x4 c = *reinterpret_cast<const f32x4*>(sC + idx * D + 16 * ((q % 4) / 2) + 8 * g + 4 * (q % 2));
          const float* xv = q < 4 ? xs + 4 * q : xo + 4 * (q - 4);
          float x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
          // keeps the float64 conversions of x inside this rare loop (hoisted
          // they would hold 64 more registers for the whole kernel)
          asm volatile("" : "+v"(x0), "+v"(x1), "+v"(x2), "+v"(x3));
          double e;
          e = (double)x0 - (double)c.x; dj = fma(e, e, dj);
          e = (double)x1 - (double)c.y; dj = fma(e, e, dj);
          e = (double)x2 - (double)c.z; dj = fma(e, e, dj);
          e = (double)x3 - (double)c.w; dj = fma(e, e, dj);
        }
        if (dj < bd) {
          bd = dj;
          bj = idx;
        }
      }
      const double obd = __shfl_xor(bd, 32);
      const int obj = __shfl_xor(bj, 32);
      if (obd < bd || (obd == bd && obj < bj)) {
        bd = obd;
        bj = obj;
      }
      if (need) {
        bi = bj;
        if (h == 0) ++rechecks;
      }
    }
    bi = __shfl(bi, (int)col);  // lane col (h = 0) decided for both halves
    if (valid && h == 0) {
      assign[p] = bi;
      atomicAdd(&scnt[bi], 1u);
    }
    // update: x transposed through LDS, one-hot assignments as the A operand
#pragma unroll
    for (int t = 0; t < 16; ++t) xt[wv][16 * (t / 8) + 2 * (t % 8) + h][col] = xs[t];  // xs[t] is dim 16 (t / 8) + 8h + t % 8
    if (h == 0) ab[wv][col] = valid ? bi : -1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    {
      // 16 points per instruction: lane (col, h) supplies A[col][8h + j] =
      // [a_p = blk * 32 + col] and B[8h + j][col] = x[p][col] (as three
      // pieces) for the points p = 16 kc + 8h + j, j = 0..7
      const float* xrow = &xt[wv][16 * (col / 16) + 2 * (col % 8) + (col / 8) % 2][0];
#pragma unroll
      for (int kc = 0; kc < 2; ++kc) {
        const f32x4 xa = *reinterpret_cast<const f32x4*>(xrow + 16 * kc + 8 * h);
        const f32x4 xb = *reinterpret_cast<const f32x4*>(xrow + 16 * kc + 8 * h + 4);
        const int4 aa = *reinterpret_cast<const int4*>(&ab[wv][16 * kc + 8 * h]);
        const int4 ac = *reinterpret_cast<const int4*>(&ab[wv][16 * kc + 8 * h + 4]);
        const float xv[8] = {xa.x, xa.y, xa.z, xa.w, xb.x, xb.y, xb.z, xb.w};
        const int av[8] = {aa.x, aa.y, aa.z, aa.w, ac.x, ac.y, ac.z, ac.w};
        bf16x8 ph, pm, pl, o0, o1;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          __bf16 vh, vm, vl;
          split_bf16x3(xv[j], vh, vm, vl);
          ph[j] = vh;
          pm[j] = vm;
          pl[j] = vl;
          o0[j] = bf16_bits(av[j] == (int)col ? 0x3F80u : 0u);
          o1[j] = bf16_bits(av[j] == (int)(32 + col) ? 0x3F80u : 0u);
        }
        sum0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o0, ph, sum0, 0, 0, 0);
        sum1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o1, ph, sum1, 0, 0, 0);
        sum0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o0, pm, sum0, 0, 0, 0);
        sum1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o1, pm, sum1, 0, 0, 0);
        sum0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o0, pl, sum0, 0, 0, 0);
        sum1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(o1, pl, sum1, 0, 0, 0);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if ((it + 1) % kKmFlushIters == 0 || it + 1 == iters) {
      // D layout: register r of lane (col, h) is cluster 8 (r / 4) + 4 h + r % 4 (+ 32 for sum1), dim col
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int c = 8 * (r / 4) + 4 * (int)h + (r % 4);
        atomicAdd(&s64[c * D + col], (double)sum0[r]);
        atomicAdd(&s64[(32 + c) * D + col], (double)sum1[r]);
      }
      sum0 = f32x16{};
      sum1 = f32x16{};
    }
#pragma unroll
    for (int s = 0; s < 16; ++s) xs[s] = xn[s];
  }
  __syncthreads();
  if (rechecks) atomicAdd(n_recheck, rechecks);
  if (tmin < kTinyBits - 1u) atomicOr(tiny, 1ull);
  for (int i = threadIdx.x; i < K * D; i += blockDim.x) part_sum[(uint64_t)blockIdx.x * K * D + i] = s64[i];
  if (threadIdx.x < K) part_cnt[(uint64_t)blockIdx.x * K + threadIdx.x] = scnt[threadIdx.x];
}

// Any d, k: float64 direct-form assignment (exact decisions) and float64 sums.
__global__ __launch_bounds__(256) void k_km_generic(const float* __restrict__ X, uint64_t N, const float* __restrict__ C,
                                                    uint32_t k, uint32_t d, int32_t* __restrict__ assign,
                                                    double* __restrict__ part_sum, uint32_t* __restrict__ part_cnt) {
  // part_sum/part_cnt hold a single partial here, accumulated with atomics
  for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < N; p += (uint64_t)gridDim.x * blockDim.x) {
    const float* xp = X + p * d;
    double bd = INFINITY;
    uint32_t bj = 0;
    for (uint32_t j = 0; j < k; ++j) {
      const double dj = dist64(xp, C + (uint64_t)j * d, d);
      if (dj < bd) {
        bd = dj;
        bj = j;
      }
    }
    assign[p] = (int32_t)bj;
    atomicAdd(&part_cnt[bj], 1u);
    for (uint32_t t = 0; t < d; ++t) atomicAdd(&part_sum[(uint64_t)bj * d + t], (double)xp[t]);
  }
}

__global__ void k_km_zero(double* __restrict__ a, uint64_t na, uint32_t* __restrict__ b, uint64_t nb) {
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < na; i += (uint64_t)gridDim.x * blockDim.x) a[i] = 0.0;
  for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < nb; i += (uint64_t)gridDim.x * blockDim.x) b[i] = 0u;
}

// Sum the G partials in a fixed order (deterministic), write float32 sums,
// counts and new centroids (old centroid for an empty cluster). Workgroup =
// 64 consecutive (cluster, dim) entries x 16 waves; wave w adds partials
// g = w, w + 16, ... (loads unrolled, in flight together), then the 16 wave
// sums are added in wave order. The same split for every launch keeps the
// result bit-identical from run to run.
constexpr int kFinalWaves = 16;

__global__ __launch_bounds__(kFinalWaves * kWave) void k_km_final(const double* __restrict__ part_sum,
                                                                  const uint32_t* __restrict__ part_cnt, uint32_t G,
                                                                  uint32_t k, uint32_t d, const float* __restrict__ C,
                                                                  float* __restrict__ sums, uint32_t* __restrict__ counts,
                                                                  float* __restrict__ cent) {
  __shared__ double ws[kFinalWaves][kWave];
  __shared__ unsigned long long wn[kFinalWaves][kWave];
  const uint64_t kd = (uint64_t)k * d;
  const uint32_t w = threadIdx.x / kWave, lane = lane_id();
  const uint64_t i = (uint64_t)blockIdx.x * kWave + lane;
  double s = 0.0;
  unsigned long long n = 0;
  if (i < kd) {
    const uint32_t j = (uint32_t)(i / d);
    uint32_t g = w;
    for (; g + 3 * kFinalWaves < G; g += 4 * kFinalWaves) {
      const double a0 = part_sum[(uint64_t)g * kd + i], a1 = part_sum[(uint64_t)(g + kFinalWaves) * kd + i];
      const double a2 = part_sum[(uint64_t)(g + 2 * kFinalWaves) * kd + i];
      const double a3 = part_sum[(uint64_t)(g + 3 * kFinalWaves) * kd + i];
      const uint32_t c0 = part_cnt[(uint64_t)g * k + j], c1 = part_cnt[(uint64_t)(g + kFinalWaves) * k + j];
      const uint32_t c2 = part_cnt[(uint64_t)(g + 2 * kFinalWaves) * k + j];
      const uint32_t c3 = part_cnt[(uint64_t)(g + 3 * kFinalWaves) * k + j];
      s += a0;
      s += a1;
      s += a2;
      s += a3;
      n += (unsigned long long)c0 + c1 + c2 + c3;
    }
    for (; g < G; g += kFinalWaves) {
      s += part_sum[(uint64_t)g * kd + i];
      n += part_cnt[(uint64_t)g * k + j];
    }
  }
  ws[w][lane] = s;
  wn[w][lane] = n;
  __syncthreads();
  if (w == 0 && i < kd) {
    double t = 0.0;
    unsigned long long c = 0;
    for (int q = 0; q < kFinalWaves; ++q) {
      t += ws[q][lane];
      c += wn[q][lane];
    }
    const uint32_t j = (uint32_t)(i / d);
    if (sums) sums[i] = (float)t;
    if (cent) cent[i] = c ? (float)(t / (double)c) : C[i];
    if (counts && i % d == 0) counts[j] = (uint32_t)c;
  }
}

hipError_t km_enqueue(const KmLaunch& L, hipStream_t s, hipEvent_t map0, hipEvent_t map1) {
  hipLaunchKernelGGL(k_km_prep, dim3(1), dim3(256), 0, s, L.C, L.k, L.d, L.cn, L.cmax, L.tiny);
  if (map0) (void)hipEventRecord(map0, s);
  if (L.mfma) {
    hipLaunchKernelGGL(k_km_mfma, dim3(L.G), dim3(kKmThreads), 0, s, L.X, L.N, L.C, L.cn, L.cmax, L.assign, L.part_sum,
                       L.part_cnt, L.n_recheck, L.tiny);
  } else {
    hipLaunchKernelGGL(k_km_zero, dim3(256), dim3(256), 0, s, L.part_sum, (uint64_t)L.k * L.d, L.part_cnt, (uint64_t)L.k);
    const uint64_t b = (L.N + 255) / 256;
    hipLaunchKernelGGL(k_km_generic, dim3((uint32_t)(b ? (b < 4096 ? b : 4096) : 1)), dim3(256), 0, s, L.X, L.N, L.C, L.k,
                       L.d, L.assign, L.part_sum, L.part_cnt);
  }
  if (map1) (void)hipEventRecord(map1, s);
  const uint64_t kd = (uint64_t)L.k * L.d;
  hipLaunchKernelGGL(k_km_final, dim3((uint32_t)((kd + kWave - 1) / kWave)), dim3(kFinalWaves * kWave), 0, s, L.part_sum, L.part_cnt,
                     L.mfma ? L.G : 1u, L.k, L.d, L.C, L.sums, L.counts, L.cent);
  return hipGetLastError();
}

}  // namespace mr
