// Pippenger multi-scalar multiplication over BN254 G1, plus the KZG setup
// (SRS from a trapdoor) and the fold's challenge products.
//
// KZG commits to f as [f(tau)]_1 = sum_i f_i [tau^i]_1 (Polynomial Commitment
// preliminaries), i.e. Q = sum_i s_i P_i.  Bucket method with signed c-bit
// digits: if s > (r-1)/2 the pair (s, P) is replaced by (r - s, -P) so every
// scalar has at most 253 bits; window w contributes digits d in
// [-2^(c-1), 2^(c-1)] and point P lands in bucket |d| with sign(d).
//
//   Q = sum_w 2^(cw) sum_k k B_(w,k),   B_(w,k) = sum of +-P with |digit| = k.
//
// Two layouts of the same computation:
//  * generic (any bases): W*K buckets, then a Horner combine of the window
//    sums with c doublings per window;
//  * table (a prepared SRS): the table holds 2^(cw) P_i for every window, so
//    window w's digit of s_i selects table point (w, i) and the window sums
//    are simply added -- no doubling chain.  Windows keep their own buckets
//    (one large MSM: short runs, parallel reduction) or share K buckets (a
//    batch of many MSMs, one bucket set each).
//
// Pipeline (all on the caller's stream):
//  1 decompose  scalars -> W signed digits each
//  2 histogram  per (window, chunk) workgroup, counts in LDS, flushed to HBM
//  3 scan       bucket offsets
//  4 scatter    counting sort of (point index, sign) by bucket
//  5 accumulate each thread sums exactly L consecutive sorted entries with
//               mixed additions (load balanced whatever the bucket sizes);
//               runs that cross thread boundaries are finished by a segmented
//               tree in LDS, runs that cross workgroups by further levels
//               over 2 records per workgroup
//  6 reduce     sum_k k B_k by running sums over chunks of LB buckets and
//               bit-sliced sums of the chunk totals (wide trees, one short
//               doubling chain per bucket set)
//  7 combine    Horner over windows (generic) or a plain sum (table), affine
#include <algorithm>

#include "curve.h"
#include "curve_quad.h"
#include "device.h"
#include "msm_store.h"
#include "msm.h"
#include "prof.h"
#include "setup.h"

namespace zk {

namespace {

// (r - 1) / 2 in 32-bit words
__constant__ uint32_t FR_HALF[8] = {0xf8000000u, 0xa1f0fac9u, 0x3cdcb848u, 0x9419f424u,
                                    0x40c0ac2eu, 0xdc2822dbu, 0x7098d014u, 0x18322739u};
// G1 generator (1, 2)
__constant__ uint32_t G1_GEN[16] = {1, 0, 0, 0, 0, 0, 0, 0, 2, 0, 0, 0, 0, 0, 0, 0};

__device__ __forceinline__ void ldw(const uint32_t* p, uint32_t* w, int n4) {
  for (int q = 0; q < n4; q++) {
    const uint4 v = reinterpret_cast<const uint4*>(p)[q];
    w[4 * q] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
}

__device__ __forceinline__ void stw(uint32_t* p, const uint32_t* w, int n4) {
  for (int q = 0; q < n4; q++)
    reinterpret_cast<uint4*>(p)[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// Montgomery affine point from 16 packed words; false for (0, 0) = infinity.
__device__ __forceinline__ bool ld_aff(const uint32_t* p, aff& a) {
  uint32_t w[16];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const uint4 v = reinterpret_cast<const uint4*>(p)[q];
    w[4 * q] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < 16; i++) o |= w[i];
  a.x = unpack(w);
  a.y = unpack(w + 8);
  return o != 0;
}

// XYZZ -> Montgomery canonical affine words (infinity -> zeros).
__device__ void st_aff_mont(uint32_t* p, const xyzz& a) {
  uint32_t w[16];
  if (is_inf(a)) {
    for (int i = 0; i < 16; i++) w[i] = 0;
  } else {
    const f29 I = mont_inv<Fq>(mont_mul<Fq>(a.ZZ, a.ZZZ));
    pack(reduce_full<Fq>(mont_mul<Fq>(a.X, mont_mul<Fq>(I, a.ZZZ))), w);
    pack(reduce_full<Fq>(mont_mul<Fq>(a.Y, mont_mul<Fq>(I, a.ZZ))), w + 8);
  }
  stw(p, w, 4);
}

// ---------------------------------------------------------------- decompose
// Signed c-bit digits of a canonical scalar, with the negation trick: if
// s > (r-1)/2 the pair (s, P) becomes (r - s, -P), so s has at most 253 bits
// and W windows hold its digits d_w in [-2^(c-1), 2^(c-1)] with no carry out.
// f(w, |d_w|, sign) is called for every nonzero digit.
template <class Fn>
__device__ __forceinline__ void for_each_digit(const uint32_t* __restrict__ scalar, uint32_t c, uint32_t W, Fn f) {
  uint32_t s[8];
  ldw(scalar, s, 2);
  // s > (r-1)/2 ?  (borrow of HALF - s)
  unsigned br = 0;
#pragma unroll
  for (int q = 0; q < 8; q++) (void)__builtin_subc(FR_HALF[q], s[q], br, &br);
  const uint32_t neg = br;
  if (neg) {
    unsigned b2 = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) s[q] = __builtin_subc(FrP::M32[q], s[q], b2, &b2);
  }
  const uint32_t full = 1u << c, half = 1u << (c - 1);
  uint32_t carry = 0;
  for (uint32_t w = 0; w < W; w++) {
    const uint32_t o = c * w, j = o >> 5, sh = o & 31;
    uint64_t two = s[j];
    if (j + 1 < 8) two |= (uint64_t)s[j + 1] << 32;
    const uint32_t d = (uint32_t)((two >> sh) & (full - 1)) + carry;
    uint32_t mag, sg;
    if (d > half) {
      mag = full - d;
      sg = 1;
      carry = 1;
    } else {
      mag = d;
      sg = 0;
      carry = 0;
    }
    if (mag) f(w, mag, sg ^ neg);
  }
}

// ---------------------------------------------------------------- items
// Host segment offsets travel as kernel arguments (no host buffer outlives
// the call; capture-safe).  One thread per segment writes its offset and its
// histogram items (chunks of at most p.chunk scalars of one segment).
constexpr uint32_t SEG_ARGS = 128;
struct SegArgs {
  uint32_t first;                 // first segment of this launch
  uint32_t count;                 // segments in this launch
  uint32_t off[SEG_ARGS + 1];     // scalar offsets of segments first..first+count
  uint32_t item0[SEG_ARGS];       // first item index of each segment
};

__global__ void make_items_kernel(SegArgs a, uint32_t chunk, uint32_t* __restrict__ seg_off,
                                  uint4* __restrict__ items) {
  const uint32_t t = threadIdx.x;
  if (t >= a.count) return;
  const uint32_t b = a.first + t;
  const uint32_t g0 = a.off[t], g1 = a.off[t + 1];
  seg_off[b] = g0;
  if (t + 1 == a.count) seg_off[b + 1] = g1;
  uint32_t it = a.item0[t];
  for (uint32_t g = g0; g < g1; g += chunk) items[it++] = make_uint4(b, g, min(g + chunk, g1), 0);
}

// ---------------------------------------------------------------- two-level counting sort
// Entries (point index | sign << 31) are sorted by bin = bucket set base +
// |digit| - 1.  A one-level counting sort over the K = 2^15 buckets of an
// MSM costs about one global atomic per entry (a block of a few thousand
// scalars touches most buckets once) and scatters 4-byte writes over the
// whole output.  Two levels avoid both:
//  coarse  blocks of scalars partition their digits by bin >> S (at most a
//          few thousand coarse bins per block, each receiving runs of
//          entries): counts, scan, scatter of (entry, bin) pairs;
//  fine    blocks of consecutive coarse-sorted pairs see only a few hundred
//          distinct bins, so their histograms and claimed output ranges cost
//          one global atomic per (block, bin) with many entries each.
__device__ __forceinline__ uint32_t bin_base(const MsmPlan& p, uint32_t seg, uint32_t w) {
  return (seg * p.Wb + (p.Wb > 1 ? w : 0u)) * p.K;
}

// Coarse bins of one item's segment: [cbase, cbase + Wb * K >> S).
__device__ __forceinline__ uint32_t coarse_span(const MsmPlan& p) { return (p.Wb * p.K) >> p.S; }

// Block's item: from the item list (several segments) or, for one segment,
// chunk blockIdx.x of [0, n).
__device__ __forceinline__ uint4 block_item(const MsmPlan& p, const uint4* __restrict__ items) {
  if (items) return items[blockIdx.x];
  const uint32_t g0 = blockIdx.x * p.chunk;
  return make_uint4(0u, g0, min(g0 + p.chunk, p.n), 0u);
}

__global__ void __launch_bounds__(MSM_NT)
coarse_count_kernel(const uint32_t* __restrict__ scalars, MsmPlan p, const uint4* __restrict__ items,
                    uint32_t* __restrict__ ccounts, uint32_t* __restrict__ block_counts) {
  extern __shared__ uint32_t h[];
  const uint4 it = block_item(p, items);
  const uint32_t span = coarse_span(p), cbase = bin_base(p, it.x, 0) >> p.S;
  for (uint32_t b = threadIdx.x; b < span; b += MSM_NT) h[b] = 0;
  __syncthreads();
  for (uint32_t i = it.y + threadIdx.x; i < it.z; i += MSM_NT)
    for_each_digit(scalars + (size_t)i * 8, p.c, p.W, [&](uint32_t w, uint32_t mag, uint32_t) {
      atomicAdd(&h[((bin_base(p, it.x, w) + mag - 1) >> p.S) - cbase], 1u);
    });
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < span; b += MSM_NT) {
    if (h[b]) atomicAdd(&ccounts[cbase + b], h[b]);
    // one segment: the block's counts, for the staged scatter
    if (block_counts) block_counts[(size_t)blockIdx.x * span + b] = h[b];
  }
}

__global__ void __launch_bounds__(MSM_NT)
coarse_scatter_kernel(const uint32_t* __restrict__ scalars, MsmPlan p, const uint4* __restrict__ items,
                      const uint32_t* __restrict__ seg_off, uint32_t* __restrict__ ccursor,
                      uint2* __restrict__ pairs, const uint32_t* __restrict__ ctotal, uint32_t dense_min) {
  extern __shared__ uint32_t h[];
  if (*ctotal >= dense_min) return;  // the staged kernel takes dense digits
  const uint4 it = block_item(p, items);
  const uint32_t span = coarse_span(p), cbase = bin_base(p, it.x, 0) >> p.S;
  for (uint32_t b = threadIdx.x; b < span; b += MSM_NT) h[b] = 0;
  __syncthreads();
  for (uint32_t i = it.y + threadIdx.x; i < it.z; i += MSM_NT)
    for_each_digit(scalars + (size_t)i * 8, p.c, p.W, [&](uint32_t w, uint32_t mag, uint32_t) {
      atomicAdd(&h[((bin_base(p, it.x, w) + mag - 1) >> p.S) - cbase], 1u);
    });
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < span; b += MSM_NT)
    if (h[b]) h[b] = atomicAdd(&ccursor[cbase + b], h[b]);
  __syncthreads();
  // point index: the base itself (generic) or table row w of the segment's point
  const uint32_t s0 = items ? seg_off[it.x] : 0u;
  for (uint32_t i = it.y + threadIdx.x; i < it.z; i += MSM_NT)
    for_each_digit(scalars + (size_t)i * 8, p.c, p.W, [&](uint32_t w, uint32_t mag, uint32_t sg) {
      const uint32_t bin = bin_base(p, it.x, w) + mag - 1;
      const uint32_t pos = atomicAdd(&h[(bin >> p.S) - cbase], 1u);
      const uint32_t pt = p.table ? w * p.tab_stride + (i - s0) : i;
      pairs[pos] = make_uint2(pt | (sg << 31), bin);
    });
}

// Staged coarse scatter, for one segment with few coarse bins.  The direct
// scatter above has every lane write its own 8-byte pair into one of the
// block's bins, so a wave's writes land on up to 64 lines.  Here the block
// takes its digits' counts per coarse bin (kept by the counting kernel), claims each bin's global range, ranks
// every digit into an LDS copy of its pairs ordered by bin, and writes the
// copy out in order: consecutive lanes write consecutive positions of one
// bin's run.  LDS: counts / rank cursors, stage offsets and claimed global
// starts (span words each), the scan's thread sums, then the staged pairs.
constexpr uint32_t STAGED_NT = 1024;
constexpr size_t STAGED_MAX_LDS = 160 * 1024;

__host__ __device__ inline size_t staged_lds_words(uint32_t span) {
  return ((size_t)3 * span + STAGED_NT + 1) & ~(size_t)1;  // pairs 8-byte aligned
}

__global__ void __launch_bounds__(STAGED_NT)
coarse_scatter_staged_kernel(const uint32_t* __restrict__ scalars, MsmPlan p, const uint32_t* __restrict__ block_counts,
                             uint32_t* __restrict__ ccursor, uint2* __restrict__ pairs,
                             const uint32_t* __restrict__ ctotal, uint32_t dense_min) {
  extern __shared__ uint32_t sm[];
  if (*ctotal < dense_min) return;  // sparse digits: the direct kernel
  const uint32_t span = coarse_span(p);  // one segment: coarse bins [0, span)
  uint32_t* cnt = sm;
  uint32_t* loff = sm + span;
  uint32_t* gpos = sm + 2 * span;
  uint32_t* tsum = sm + 3 * span;
  uint2* stage = reinterpret_cast<uint2*>(sm + staged_lds_words(span));
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (span + STAGED_NT - 1) / STAGED_NT;
  const uint32_t b0 = min(tid * per, span), b1 = min(b0 + per, span);
  // one workgroup per compute unit (the LDS holds one) walks the items, so a
  // launch that finds sparse digits ends at once
  for (uint32_t item = blockIdx.x; item < p.nitems; item += gridDim.x) {
    const uint32_t g0 = item * p.chunk, g1 = min(g0 + p.chunk, p.n);
    // the counting kernel's counts of this block
    for (uint32_t b = tid; b < span; b += STAGED_NT) cnt[b] = block_counts[(size_t)item * span + b];
    __syncthreads();
    // exclusive scan of the counts: thread t sums bins [b0, b1), the thread
    // sums are scanned in LDS (Hillis-Steele)
    uint32_t run = 0;
    for (uint32_t b = b0; b < b1; b++) run += cnt[b];
    tsum[tid] = run;
    __syncthreads();
    for (uint32_t d = 1; d < STAGED_NT; d <<= 1) {
      const uint32_t v = tid >= d ? tsum[tid - d] : 0u;
      __syncthreads();
      tsum[tid] += v;
      __syncthreads();
    }
    uint32_t at = tsum[tid] - run;
    for (uint32_t b = b0; b < b1; b++) {
      const uint32_t c = cnt[b];
      loff[b] = at;
      gpos[b] = c ? atomicAdd(&ccursor[b], c) : 0u;
      cnt[b] = at;
      at += c;
    }
    const uint32_t total = tsum[STAGED_NT - 1];
    __syncthreads();
    for (uint32_t i = g0 + tid; i < g1; i += STAGED_NT)
      for_each_digit(scalars + (size_t)i * 8, p.c, p.W, [&](uint32_t w, uint32_t mag, uint32_t sg) {
        const uint32_t bin = bin_base(p, 0, w) + mag - 1;
        const uint32_t j = atomicAdd(&cnt[bin >> p.S], 1u);
        stage[j] = make_uint2((p.table ? w * p.tab_stride + i : i) | (sg << 31), bin);
      });
    __syncthreads();
    for (uint32_t j = tid; j < total; j += STAGED_NT) {
      const uint2 q = stage[j];
      const uint32_t b = q.y >> p.S;
      pairs[gpos[b] + (j - loff[b])] = q;
    }
    __syncthreads();
  }
}

// Fine level: block k takes pairs [k * FINE_CHUNK, ...) of the coarse-sorted
// list.  Its bins lie in [lo, hi) (whole coarse bins from the first to the
// last pair's); a range that fits in LDS is histogrammed there, a wider one
// (sparse pairs) goes straight to global atomics.
constexpr uint32_t FINE_CHUNK = 4096;
constexpr uint32_t FINE_LDS_BINS = 4096;

__device__ __forceinline__ bool fine_range(const uint2* pairs, uint32_t e0, uint32_t e1, uint32_t S, uint32_t& lo,
                                           uint32_t& hi) {
  lo = (pairs[e0].y >> S) << S;
  hi = ((pairs[e1 - 1].y >> S) + 1) << S;
  return hi - lo <= FINE_LDS_BINS;
}

__global__ void __launch_bounds__(MSM_NT)
fine_count_kernel(const uint2* __restrict__ pairs, const uint32_t* __restrict__ ctotal, MsmPlan p,
                  uint32_t* __restrict__ counts) {
  extern __shared__ uint32_t h[];
  const uint32_t E = *ctotal;
  const uint32_t e0 = blockIdx.x * FINE_CHUNK;
  if (e0 >= E) return;
  const uint32_t e1 = min(e0 + FINE_CHUNK, E);
  uint32_t lo, hi;
  if (!fine_range(pairs, e0, e1, p.S, lo, hi)) {
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += MSM_NT) atomicAdd(&counts[pairs[e].y], 1u);
    return;
  }
  for (uint32_t b = threadIdx.x; b < hi - lo; b += MSM_NT) h[b] = 0;
  __syncthreads();
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += MSM_NT) atomicAdd(&h[pairs[e].y - lo], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < hi - lo; b += MSM_NT)
    if (h[b]) atomicAdd(&counts[lo + b], h[b]);
}

__global__ void __launch_bounds__(MSM_NT)
fine_scatter_kernel(const uint2* __restrict__ pairs, const uint32_t* __restrict__ ctotal, MsmPlan p,
                    uint32_t* __restrict__ cursor, uint32_t* __restrict__ entries, uint32_t dense_min) {
  extern __shared__ uint32_t h[];
  const uint32_t E = *ctotal;
  if (E >= dense_min) return;  // the staged kernel takes dense digits
  const uint32_t e0 = blockIdx.x * FINE_CHUNK;
  if (e0 >= E) return;
  const uint32_t e1 = min(e0 + FINE_CHUNK, E);
  uint32_t lo, hi;
  if (!fine_range(pairs, e0, e1, p.S, lo, hi)) {
    for (uint32_t e = e0 + threadIdx.x; e < e1; e += MSM_NT) {
      const uint2 q = pairs[e];
      entries[atomicAdd(&cursor[q.y], 1u)] = q.x;
    }
    return;
  }
  for (uint32_t b = threadIdx.x; b < hi - lo; b += MSM_NT) h[b] = 0;
  __syncthreads();
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += MSM_NT) atomicAdd(&h[pairs[e].y - lo], 1u);
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < hi - lo; b += MSM_NT)
    if (h[b]) h[b] = atomicAdd(&cursor[lo + b], h[b]);
  __syncthreads();
  for (uint32_t e = e0 + threadIdx.x; e < e1; e += MSM_NT) {
    const uint2 q = pairs[e];
    entries[atomicAdd(&h[q.y - lo], 1u)] = q.x;
  }
}

// Fine scatter, staged (for dense digits; the direct kernel above serves
// sparse ones): the block's pairs are read once into LDS, counted
// and ranked there by bin, and the entries written out in bin order, so
// consecutive lanes write consecutive positions of one bucket's run.  A block
// whose bins span more than FINE_STAGED_BINS (sparse pairs) claims each
// entry's position by a global atomic instead.  LDS: the pairs, the ranked
// entries and their bin indices, per-bin counts / rank cursors and
// position offsets, the scan's thread sums.
constexpr uint32_t FINE_STAGED_BINS = 1024;
constexpr size_t FINE_LITE_LDS = (size_t)FINE_CHUNK * 4 + FINE_CHUNK * 2 + 2 * FINE_STAGED_BINS * 4 + MSM_NT * 4;
constexpr size_t FINE_STAGED_LDS =
    (size_t)FINE_CHUNK * 8 + FINE_CHUNK * 4 + FINE_CHUNK * 2 + 2 * FINE_STAGED_BINS * 4 + MSM_NT * 4;

__global__ void __launch_bounds__(MSM_NT)
fine_scatter_staged_kernel(const uint2* __restrict__ pairs, const uint32_t* __restrict__ ctotal, MsmPlan p,
                           uint32_t* __restrict__ cursor, uint32_t* __restrict__ entries, uint32_t dense_min) {
  extern __shared__ uint32_t sm[];
  const uint32_t E = *ctotal;
  if (E < dense_min) return;  // sparse digits: the direct kernel
  uint2* in = reinterpret_cast<uint2*>(sm);
  uint32_t* out = sm + 2 * FINE_CHUNK;
  uint16_t* obin = reinterpret_cast<uint16_t*>(out + FINE_CHUNK);
  uint32_t* cnt = out + FINE_CHUNK + FINE_CHUNK / 2;
  uint32_t* delta = cnt + FINE_STAGED_BINS;
  uint32_t* tsum = delta + FINE_STAGED_BINS;
  const uint32_t tid = threadIdx.x;
  // a grid of as many workgroups as the LDS holds at once walks the chunks
  for (uint64_t c0 = (uint64_t)blockIdx.x * FINE_CHUNK; c0 < E; c0 += (uint64_t)gridDim.x * FINE_CHUNK) {
    const uint32_t e0 = (uint32_t)c0;
    const uint32_t ne = min(FINE_CHUNK, E - e0);
    for (uint32_t k = tid; k < ne; k += MSM_NT) in[k] = pairs[e0 + k];
    __syncthreads();
    // bins of the chunk: whole coarse bins from the first pair's to the last's
    const uint32_t lo = (in[0].y >> p.S) << p.S;
    const uint32_t hi = ((in[ne - 1].y >> p.S) + 1) << p.S;
    const uint32_t range = hi - lo;
    if (range > FINE_STAGED_BINS) {
      for (uint32_t k = tid; k < ne; k += MSM_NT) entries[atomicAdd(&cursor[in[k].y], 1u)] = in[k].x;
      __syncthreads();
      continue;
    }
    for (uint32_t b = tid; b < range; b += MSM_NT) cnt[b] = 0;
    __syncthreads();
    for (uint32_t k = tid; k < ne; k += MSM_NT) atomicAdd(&cnt[in[k].y - lo], 1u);
    __syncthreads();
    // exclusive scan of the counts (thread sums of contiguous bins, Hillis-Steele)
    const uint32_t per = (range + MSM_NT - 1) / MSM_NT;
    const uint32_t b0 = min(tid * per, range), b1 = min(b0 + per, range);
    uint32_t run = 0;
    for (uint32_t b = b0; b < b1; b++) run += cnt[b];
    tsum[tid] = run;
    __syncthreads();
    for (uint32_t d = 1; d < MSM_NT; d <<= 1) {
      const uint32_t v = tid >= d ? tsum[tid - d] : 0u;
      __syncthreads();
      tsum[tid] += v;
      __syncthreads();
    }
    uint32_t at = tsum[tid] - run;
    for (uint32_t b = b0; b < b1; b++) {
      const uint32_t c = cnt[b];
      // entry j of bin b goes to its claimed start + (j - at) (mod 2^32)
      delta[b] = (c ? atomicAdd(&cursor[lo + b], c) : 0u) - at;
      cnt[b] = at;
      at += c;
    }
    __syncthreads();
    for (uint32_t k = tid; k < ne; k += MSM_NT) {
      const uint2 q = in[k];
      const uint32_t b = q.y - lo;
      const uint32_t j = atomicAdd(&cnt[b], 1u);
      out[j] = q.x;
      obin[j] = (uint16_t)b;
    }
    __syncthreads();
    for (uint32_t j = tid; j < ne; j += MSM_NT) entries[delta[obin[j]] + j] = out[j];
    __syncthreads();
  }
}

// The same with the pairs read from HBM twice instead of copied to LDS: a
// third of the LDS, so four workgroups share a compute unit (coarse bins of
// fewer than 2^7 buckets, where the staged copy's occupancy costs more than
// the second read).
__global__ void __launch_bounds__(MSM_NT)
fine_scatter_lite_kernel(const uint2* __restrict__ pairs, const uint32_t* __restrict__ ctotal, MsmPlan p,
                           uint32_t* __restrict__ cursor, uint32_t* __restrict__ entries, uint32_t dense_min) {
  extern __shared__ uint32_t sm[];
  const uint32_t E = *ctotal;
  if (E < dense_min) return;  // sparse digits: the direct kernel
  uint32_t* out = sm;
  uint16_t* obin = reinterpret_cast<uint16_t*>(out + FINE_CHUNK);
  uint32_t* cnt = out + FINE_CHUNK + FINE_CHUNK / 2;
  uint32_t* delta = cnt + FINE_STAGED_BINS;
  uint32_t* tsum = delta + FINE_STAGED_BINS;
  const uint32_t tid = threadIdx.x;
  // a grid of as many workgroups as the LDS holds at once walks the chunks
  for (uint64_t c0 = (uint64_t)blockIdx.x * FINE_CHUNK; c0 < E; c0 += (uint64_t)gridDim.x * FINE_CHUNK) {
    const uint32_t e0 = (uint32_t)c0;
    const uint32_t ne = min(FINE_CHUNK, E - e0);
    const uint2* in = pairs + e0;
    // bins of the chunk: whole coarse bins from the first pair's to the last's
    const uint32_t lo = (in[0].y >> p.S) << p.S;
    const uint32_t hi = ((in[ne - 1].y >> p.S) + 1) << p.S;
    const uint32_t range = hi - lo;
    if (range > FINE_STAGED_BINS) {
      for (uint32_t k = tid; k < ne; k += MSM_NT) entries[atomicAdd(&cursor[in[k].y], 1u)] = in[k].x;
      __syncthreads();
      continue;
    }
    for (uint32_t b = tid; b < range; b += MSM_NT) cnt[b] = 0;
    __syncthreads();
    for (uint32_t k = tid; k < ne; k += MSM_NT) atomicAdd(&cnt[in[k].y - lo], 1u);
    __syncthreads();
    // exclusive scan of the counts (thread sums of contiguous bins, Hillis-Steele)
    const uint32_t per = (range + MSM_NT - 1) / MSM_NT;
    const uint32_t b0 = min(tid * per, range), b1 = min(b0 + per, range);
    uint32_t run = 0;
    for (uint32_t b = b0; b < b1; b++) run += cnt[b];
    tsum[tid] = run;
    __syncthreads();
    for (uint32_t d = 1; d < MSM_NT; d <<= 1) {
      const uint32_t v = tid >= d ? tsum[tid - d] : 0u;
      __syncthreads();
      tsum[tid] += v;
      __syncthreads();
    }
    uint32_t at = tsum[tid] - run;
    for (uint32_t b = b0; b < b1; b++) {
      const uint32_t c = cnt[b];
      // entry j of bin b goes to its claimed start + (j - at) (mod 2^32)
      delta[b] = (c ? atomicAdd(&cursor[lo + b], c) : 0u) - at;
      cnt[b] = at;
      at += c;
    }
    __syncthreads();
    for (uint32_t k = tid; k < ne; k += MSM_NT) {
      const uint2 q = in[k];
      const uint32_t b = q.y - lo;
      const uint32_t j = atomicAdd(&cnt[b], 1u);
      out[j] = q.x;
      obin[j] = (uint16_t)b;
    }
    __syncthreads();
    for (uint32_t j = tid; j < ne; j += MSM_NT) entries[delta[obin[j]] + j] = out[j];
    __syncthreads();
  }
}

// ---------------------------------------------------------------- segmented combine
// LDS record block: keys[SLOTS], flags[SLOTS], points[SLOTS][36].
struct RecLds {
  uint32_t* keys;
  uint32_t* flags;
  uint32_t* pts;
};

__device__ __forceinline__ RecLds rec_lds(uint32_t* sm) {
  RecLds r;
  r.keys = sm;
  r.flags = sm + MSM_SLOTS;
  r.pts = sm + 2 * MSM_SLOTS;
  return r;
}

__device__ __forceinline__ uint32_t lower_bound_lds(const uint32_t* k, uint32_t key) {
  uint32_t lo = 0, hi = MSM_SLOTS;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (k[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ __forceinline__ uint32_t upper_bound_lds(const uint32_t* k, uint32_t key) {
  uint32_t lo = 0, hi = MSM_SLOTS;
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (k[mid] <= key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

__device__ void put_slot(RecLds& r, uint32_t i, uint32_t key, uint32_t flag, const xyzz& a) {
  r.keys[i] = key;
  r.flags[i] = flag;
  st_xyzz(r.pts + i * XYZZ_WORDS, a);
}

__device__ __forceinline__ void put_rec(uint32_t* rec, uint32_t key, uint32_t flag, const uint32_t* pts_or_null) {
  reinterpret_cast<uint4*>(rec)[0] = make_uint4(key, flag, 0, 0);
  uint4* dst = reinterpret_cast<uint4*>(rec + 4);
  const uint4* src = reinterpret_cast<const uint4*>(pts_or_null);
  for (int w = 0; w < 9; w++) dst[w] = pts_or_null ? src[w] : make_uint4(0, 0, 0, 0);
}

// Sum every run of equal keys held in the LDS slots; runs closed on both sides
// are written to their bucket, the first and last run of the block go out as
// records for the next level (data only if still open there).  The runs are
// summed by a segmented tree: at level d the slot at offset 0 mod 2d of its
// run adds the slot d further on.  The pairs that have work at a level are
// listed first and handed to consecutive threads, so a wave only runs
// additions when its lanes have them (runs are often long, and most pairs
// of a naive slot-per-thread sweep would be idle).
__device__ void combine_and_emit(RecLds& r, bool left_open, bool right_open, uint32_t* __restrict__ buckets,
                                 uint32_t* out_rec) {
  __shared__ uint32_t act[MSM_SLOTS / 2];  // pairs are disjoint: at most SLOTS/2 per level
  __shared__ uint32_t nact, maxrun;
  const uint32_t tid = threadIdx.x;
  if (tid == 0) maxrun = 1;
  __syncthreads();
  uint32_t head[MSM_SLOTS / MSM_NT];
#pragma unroll
  for (uint32_t q = 0; q < MSM_SLOTS / MSM_NT; q++) {
    const uint32_t i = tid + q * MSM_NT;
    head[q] = lower_bound_lds(r.keys, r.keys[i]);
    if (head[q] == i) atomicMax(&maxrun, upper_bound_lds(r.keys, r.keys[i]) - i);
  }
  __syncthreads();
  const uint32_t runmax = maxrun;
  for (uint32_t d = 1; d < runmax; d <<= 1) {
    if (tid == 0) nact = 0;
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < MSM_SLOTS / MSM_NT; q++) {
      const uint32_t i = tid + q * MSM_NT;
      if (((i - head[q]) & (2 * d - 1)) == 0 && i + d < MSM_SLOTS && r.keys[i + d] == r.keys[i] &&
          r.flags[i + d])
        act[atomicAdd(&nact, 1u)] = i;
    }
    __syncthreads();
    const uint32_t n = nact;
    for (uint32_t k = tid; k < n; k += MSM_NT) {
      const uint32_t i = act[k];
      const xyzz s = add(ld_xyzz(r.pts + i * XYZZ_WORDS), ld_xyzz(r.pts + (i + d) * XYZZ_WORDS));
      st_xyzz(r.pts + i * XYZZ_WORDS, s);
      r.flags[i] = 1;
    }
    __syncthreads();
  }
#pragma unroll
  for (uint32_t q = 0; q < MSM_SLOTS / MSM_NT; q++) {
    const uint32_t i = tid + q * MSM_NT;
    if (head[q] != i) continue;
    const uint32_t key = r.keys[i];
    const uint32_t e = upper_bound_lds(r.keys, key);
    const bool lo = (i == 0) && left_open;
    const bool ro = (e == MSM_SLOTS) && right_open;
    const bool has = r.flags[i] != 0;
    if (!lo && !ro && has && key != KEY_SENTINEL) {
      uint4* dst = reinterpret_cast<uint4*>(buckets + (size_t)key * XYZZ_WORDS);
      const uint4* src = reinterpret_cast<const uint4*>(r.pts + i * XYZZ_WORDS);
      for (int w = 0; w < 9; w++) dst[w] = src[w];
    }
    if (!out_rec) continue;
    const size_t rb = 2 * (size_t)blockIdx.x;
    if (i == 0) {
      const bool send = (lo || ro) && has;
      put_rec(out_rec + rb * REC_WORDS, key, send ? 1u : 0u, send ? r.pts + i * XYZZ_WORDS : nullptr);
    }
    if (e == MSM_SLOTS) {
      const bool send = ro && has && i != 0;
      put_rec(out_rec + (rb + 1) * REC_WORDS, key, send ? 1u : 0u, send ? r.pts + i * XYZZ_WORDS : nullptr);
    }
  }
}

// Level of the record reduction: 2*MSM_NT records per workgroup.
__global__ void __launch_bounds__(MSM_NT)
record_reduce_kernel(const uint32_t* __restrict__ in_rec, uint32_t nrec, uint32_t* __restrict__ buckets,
                     uint32_t* out_rec) {
  extern __shared__ uint32_t sm[];
  RecLds r = rec_lds(sm);
  const uint32_t rb = blockIdx.x * MSM_SLOTS;
  for (uint32_t q = 0; q < MSM_SLOTS / MSM_NT; q++) {
    const uint32_t i = threadIdx.x + q * MSM_NT;
    const uint32_t g = rb + i;
    if (g < nrec) {
      const uint32_t* src = in_rec + (size_t)g * REC_WORDS;
      const uint4 kf = reinterpret_cast<const uint4*>(src)[0];
      r.keys[i] = kf.x;
      r.flags[i] = kf.y;
      const uint4* s4 = reinterpret_cast<const uint4*>(src + 4);
      uint4* dst = reinterpret_cast<uint4*>(r.pts + i * XYZZ_WORDS);
      for (int w = 0; w < 9; w++) dst[w] = s4[w];
    } else {
      put_slot(r, i, KEY_SENTINEL, 0, xyzz_inf());
    }
  }
  __syncthreads();
  const uint32_t re = min(rb + MSM_SLOTS, nrec);
  const bool nonempty = rb < nrec;
  const bool left_open = nonempty && rb > 0 && in_rec[(size_t)(rb - 1) * REC_WORDS] == in_rec[(size_t)rb * REC_WORDS];
  const bool right_open =
      nonempty && re < nrec && in_rec[(size_t)re * REC_WORDS] == in_rec[(size_t)(re - 1) * REC_WORDS];
  combine_and_emit(r, left_open, right_open, buckets, out_rec);
}

// ---------------------------------------------------------------- bucket reduction
// A bucket set's weighted sum V = sum_b (b + 1) B_b, b < K, is split over
// J = K / LB chunks of LB buckets: with b = j LB + m,
//   V = sum_j T_j + LB sum_j j S_j,  S_j = sum_m B_(j,m),  T_j = sum_m (m + 1) B_(j,m).
// One thread per chunk forms S_j and T_j by running sums (2 LB dependent
// additions).  sum_j j S_j is taken bit by bit: U_i = sum of the S_j whose
// index j has bit i set, so sum_j j S_j = sum_i 2^i U_i.  The U_i and
// sum_j T_j are wide plain sums (parallel trees); only one doubling chain of
// log2(K) steps per bucket set remains, instead of a small scalar multiple
// per chunk.
__global__ void __launch_bounds__(64)
chunk_sums_kernel(const uint32_t* __restrict__ buckets, const uint32_t* __restrict__ counts, MsmPlan p,
                  uint32_t* __restrict__ vbuf) {
  const uint32_t id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= p.groups * p.J) return;
  const uint32_t g = id / p.J, j = id % p.J;
  const uint32_t base = g * p.K + j * p.LB;
  xyzz acc = xyzz_inf(), sum = xyzz_inf();
  for (int m = (int)p.LB - 1; m >= 0; --m) {
    if (counts[base + m]) acc = add(acc, ld_xyzz(buckets + (size_t)(base + m) * XYZZ_WORDS));
    sum = add(sum, acc);
  }
  st_xyzz(vbuf + (size_t)id * 2 * XYZZ_WORDS, acc);
  st_xyzz(vbuf + ((size_t)id * 2 + 1) * XYZZ_WORDS, sum);
}

// The same with each chunk on a quad (four lanes per point operation): for
// few chunks, where the sums' latency matters more than their total work.
__global__ void __launch_bounds__(64)
chunk_sums_quad_kernel(const uint32_t* __restrict__ buckets, const uint32_t* __restrict__ counts, MsmPlan p,
                       uint32_t* __restrict__ vbuf) {
  const uint32_t id = (blockIdx.x * blockDim.x + threadIdx.x) >> 2, c = threadIdx.x & 3u;
  if (id >= p.groups * p.J) return;  // whole quads
  const uint32_t g = id / p.J, j = id % p.J;
  const uint32_t base = g * p.K + j * p.LB;
  f29 acc = f29_zero(), sum = f29_zero();
  for (int m = (int)p.LB - 1; m >= 0; --m) {
    if (counts[base + m]) acc = quad_add(acc, ldq(buckets + (size_t)(base + m) * XYZZ_WORDS, c));
    sum = quad_add(sum, acc);
  }
  stq(vbuf + (size_t)id * 2 * XYZZ_WORDS, c, acc);
  stq(vbuf + ((size_t)id * 2 + 1) * XYZZ_WORDS, c, sum);
}

// Partial sums of one bit slice: block (part, i, g) adds its share of the
// terms of slice i of bucket set g -- the S_j with bit i of j set (i < nbits)
// or every T_j (i = nbits) -- sequentially per thread, then by a tree in LDS.
constexpr uint32_t BITS_NT = 64;
__global__ void __launch_bounds__(BITS_NT)
bit_sums_kernel(const uint32_t* __restrict__ vbuf, MsmPlan p, uint32_t* __restrict__ partial) {
  __shared__ uint32_t sm[BITS_NT * XYZZ_WORDS];
  const uint32_t part = blockIdx.x, i = blockIdx.y, g = blockIdx.z, tid = threadIdx.x;
  const bool tslice = i == p.nbits;
  const uint32_t count = tslice ? p.J : p.J / 2;
  const uint32_t per = (count + p.parts - 1) / p.parts;
  const uint32_t t0 = part * per, t1 = min(t0 + per, count);
  const uint32_t low = (1u << i) - 1u;
  xyzz acc = xyzz_inf();
  for (uint32_t t = t0 + tid; t < t1; t += BITS_NT) {
    const uint32_t j = tslice ? t : (((t >> i) << (i + 1)) | (1u << i) | (t & low));
    acc = add(acc, ld_xyzz(vbuf + ((size_t)(g * p.J + j) * 2 + (tslice ? 1 : 0)) * XYZZ_WORDS));
  }
  st_xyzz(sm + tid * XYZZ_WORDS, acc);
  __syncthreads();
  for (uint32_t h = BITS_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const xyzz a = add(ld_xyzz(sm + tid * XYZZ_WORDS), ld_xyzz(sm + (tid + h) * XYZZ_WORDS));
      st_xyzz(sm + tid * XYZZ_WORDS, a);
    }
    __syncthreads();
  }
  if (tid == 0)
    st_xyzz(partial + ((size_t)(g * (p.nbits + 1) + i) * p.parts + part) * XYZZ_WORDS, ld_xyzz(sm));
}

// The same on quads (four lanes per point operation; block (part, i, g) has
// BITS_QUADS quads): for few bucket sets, where the sums' latency matters
// more than their total work.
constexpr uint32_t BITS_QUADS = 64;
__global__ void __launch_bounds__(BITS_QUADS * 4)
bit_sums_quad_kernel(const uint32_t* __restrict__ vbuf, MsmPlan p, uint32_t* __restrict__ partial) {
  __shared__ uint32_t sm[BITS_QUADS * XYZZ_WORDS];
  const uint32_t part = blockIdx.x, i = blockIdx.y, g = blockIdx.z;
  const uint32_t quad = threadIdx.x >> 2, c = threadIdx.x & 3u;
  const bool tslice = i == p.nbits;
  const uint32_t count = tslice ? p.J : p.J / 2;
  const uint32_t per = (count + p.parts - 1) / p.parts;
  const uint32_t t0 = part * per, t1 = min(t0 + per, count);
  const uint32_t low = (1u << i) - 1u;
  f29 acc = f29_zero();
  for (uint32_t t = t0 + quad; t < t1; t += BITS_QUADS) {  // quad-uniform bounds
    const uint32_t j = tslice ? t : (((t >> i) << (i + 1)) | (1u << i) | (t & low));
    acc = quad_add(acc, ldq(vbuf + ((size_t)(g * p.J + j) * 2 + (tslice ? 1 : 0)) * XYZZ_WORDS, c));
  }
  stq(sm + quad * XYZZ_WORDS, c, acc);
  __syncthreads();
  for (uint32_t h = BITS_QUADS / 2; h > 0; h >>= 1) {
    if (quad < h) {
      acc = quad_add(acc, ldq(sm + (quad + h) * XYZZ_WORDS, c));
      stq(sm + quad * XYZZ_WORDS, c, acc);
    }
    __syncthreads();
  }
  if (quad == 0) stq(partial + ((size_t)(g * (p.nbits + 1) + i) * p.parts + part) * XYZZ_WORDS, c, acc);
}

// One tree level over slice partials: block (k, i, g) adds partials
// 64k .. 64k+63 of slice i of set g (fewer partials per slice for the next
// level or the finishing kernel).
__global__ void __launch_bounds__(BITS_NT)
partial_tree_kernel(const uint32_t* __restrict__ in, uint32_t nin, uint32_t nslices, uint32_t* __restrict__ out) {
  __shared__ uint32_t sm[BITS_NT * XYZZ_WORDS];
  const uint32_t k = blockIdx.x, i = blockIdx.y, g = blockIdx.z, tid = threadIdx.x;
  const uint32_t nout = (nin + BITS_NT - 1) / BITS_NT;
  const uint32_t src = k * BITS_NT + tid;
  const xyzz a = src < nin ? ld_xyzz(in + ((size_t)(g * nslices + i) * nin + src) * XYZZ_WORDS) : xyzz_inf();
  st_xyzz(sm + tid * XYZZ_WORDS, a);
  __syncthreads();
  for (uint32_t h = BITS_NT / 2; h > 0; h >>= 1) {
    if (tid < h) {
      const xyzz t = add(ld_xyzz(sm + tid * XYZZ_WORDS), ld_xyzz(sm + (tid + h) * XYZZ_WORDS));
      st_xyzz(sm + tid * XYZZ_WORDS, t);
    }
    __syncthreads();
  }
  if (tid == 0) st_xyzz(out + ((size_t)(g * nslices + i) * nout + k) * XYZZ_WORDS, ld_xyzz(sm));
}

// Bucket set g: U_i from the slice partials, V = U_T + sum_i 2^(log2 LB + i) U_i,
// and the result written as canonical affine (table layout: the set is one
// output) or as XYZZ (the generic layout's window sums, combined by Horner
// next).  Every point operation runs on a quad (see curve_quad.h): this
// kernel is one dependent chain per set.  qps quads share a slice's
// partials, then the slice sums are doubled into place (one quad per slice)
// and added by a tree.
constexpr uint32_t FIN_SLICES = 32;  // nbits + 1 <= 32
constexpr uint32_t FIN_NT = 256;     // 64 quads
constexpr uint32_t FIN_QUADS = FIN_NT / 4;
// Quads per slice: FIN_QUADS over the slice count rounded up to a power of two.
inline uint32_t fin_qps(uint32_t nslices) {
  uint32_t p2 = 1;
  while (p2 < nslices) p2 <<= 1;
  return FIN_QUADS / p2;
}
__global__ void __launch_bounds__(FIN_NT)
bit_finish_kernel(const uint32_t* __restrict__ partial, uint32_t nparts, uint32_t qps, MsmPlan p,
                  uint32_t* __restrict__ out_affine, uint32_t* __restrict__ out_xyzz) {
  __shared__ uint32_t sm[FIN_QUADS * XYZZ_WORDS];
  const uint32_t g = blockIdx.x, tid = threadIdx.x, quad = tid >> 2, c = tid & 3u;
  const uint32_t i = quad / qps, k0 = quad % qps;
  const uint32_t ns = p.nbits + 1, nsp = FIN_QUADS / qps;
  f29 acc = f29_zero();
  if (i < ns)
    for (uint32_t k = k0; k < nparts; k += qps)
      acc = quad_add(acc, ldq(partial + ((size_t)(g * ns + i) * nparts + k) * XYZZ_WORDS, c));
  stq(sm + quad * XYZZ_WORDS, c, acc);
  __syncthreads();
  for (uint32_t h = qps / 2; h > 0; h >>= 1) {
    if (k0 < h) {
      acc = quad_add(acc, ldq(sm + (quad + h) * XYZZ_WORDS, c));
      stq(sm + quad * XYZZ_WORDS, c, acc);
    }
    __syncthreads();
  }
  // slice i's sum is in slot i*qps; quad i takes it, scales it and moves it
  // to slot i.  The doubling chains are the kernel's longest, and they run
  // as issue-bound single waves: packed into the first wave (or two) they
  // share no SIMD, where spread over the block's waves two of them would
  // share each SIMD and take twice as long.
  f29 v = quad < ns ? ldq(sm + quad * qps * XYZZ_WORDS, c) : f29_zero();
  __syncthreads();
  if (quad < nsp) {
    if (quad < p.nbits) {
      const uint32_t e = p.lgLB + quad;
      for (uint32_t k = 0; k < e; k++) v = quad_dbl(v);
    }
    stq(sm + quad * XYZZ_WORDS, c, v);
  }
  __syncthreads();
  for (uint32_t h = nsp / 2; h > 0; h >>= 1) {
    if (quad < h) {
      v = quad_add(v, ldq(sm + (quad + h) * XYZZ_WORDS, c));
      stq(sm + quad * XYZZ_WORDS, c, v);
    }
    __syncthreads();
  }
  if (quad != 0) return;
  if (out_xyzz) {
    stq(out_xyzz + (size_t)g * XYZZ_WORDS, c, v);
    return;
  }
  xyzz r = quad_gather(v);
  if (c != 0) return;
  force_vgpr(r);
  uint32_t o[16];
  to_affine_words(r, o);
  stw(out_affine + (size_t)g * 16, o, 4);
}

// Generic layout: Q = sum_w 2^(c w) S_w by Horner (on one quad), then
// canonical affine.
__global__ void __launch_bounds__(64) combine_kernel(const uint32_t* __restrict__ wsum, uint32_t nwin, uint32_t c,
                               uint32_t* __restrict__ out16) {
  if (blockIdx.x != 0 || threadIdx.x >= 4) return;
  const uint32_t ln = threadIdx.x;
  f29 q = ldq(wsum + (size_t)(nwin - 1) * XYZZ_WORDS, ln);
  for (int w = (int)nwin - 2; w >= 0; --w) {
    for (uint32_t t = 0; t < c; t++) q = quad_dbl(q);
    q = quad_add(q, ldq(wsum + (size_t)w * XYZZ_WORDS, ln));
  }
  xyzz r = quad_gather(q);
  if (ln != 0) return;
  force_vgpr(r);
  uint32_t o[16];
  to_affine_words(r, o);
  stw(out16, o, 4);
}

__global__ void zero16_kernel(uint32_t* out16) {
  if (threadIdx.x < 16) out16[threadIdx.x] = 0;
}

// Zero fill by a kernel (graph-capture friendly, unlike a memset node).
// ---------------------------------------------------------------- conversions / tables
__global__ void to_mont_kernel(const uint32_t* __restrict__ plain, uint32_t* __restrict__ mont, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t w[16];
  ldw(plain + i * 16, w, 4);
  aff a;
  aff_from_plain_words(w, a);  // (0,0) stays (0,0)
  pack(a.x, w);
  pack(a.y, w + 8);
  stw(mont + i * 16, w, 4);
}

__global__ void build_table_kernel(const uint32_t* __restrict__ plain, uint32_t* __restrict__ tab, uint64_t n,
                                   uint32_t c, uint32_t W) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t w[16];
  ldw(plain + i * 16, w, 4);
  aff a;
  const bool fin = aff_from_plain_words(w, a);
  pack(a.x, w);
  pack(a.y, w + 8);
  stw(tab + i * 16, w, 4);
  xyzz acc = fin ? from_aff(a) : xyzz_inf();
  for (uint32_t win = 1; win < W; win++) {
    for (uint32_t t = 0; t < c; t++) acc = dbl(acc);
    st_aff_mont(tab + ((uint64_t)win * n + i) * 16, acc);
  }
}

// gtab[j] = 2^j G, Montgomery affine, j < 256.
__global__ void gen_table_kernel(uint32_t* gtab) {
  const uint32_t j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= 256) return;
  uint32_t w[16];
  for (int q = 0; q < 16; q++) w[q] = G1_GEN[q];
  aff g;
  aff_from_plain_words(w, g);
  xyzz acc = from_aff(g);
  for (uint32_t t = 0; t < j; t++) acc = dbl(acc);
  st_aff_mont(gtab + (size_t)j * 16, acc);
}

// out[i] = [tau^i] G as canonical plain affine words.
__global__ void srs_kernel(Tau8 tw, const uint32_t* __restrict__ gtab, uint32_t* __restrict__ out, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const f29 tau = reduce_full<FrP>(to_mont<FrP>(unpack(tw.w)));
  uint32_t e[8] = {(uint32_t)i, (uint32_t)(i >> 32), 0, 0, 0, 0, 0, 0};
  const f29 ti = (i == 0) ? f29_from(FrP::ONE) : mont_pow<FrP>(tau, e);
  uint32_t s[8];
  pack(from_mont<FrP>(ti), s);
  xyzz acc = xyzz_inf();
  for (int b = 0; b < 254; b++) {
    if ((s[b >> 5] >> (b & 31)) & 1u) {
      aff g;
      ld_aff(gtab + (size_t)b * 16, g);
      acc = madd(acc, g);
    }
  }
  uint32_t o[16];
  to_affine_words(acc, o);
  stw(out + i * 16, o, 4);
}

// [s] G by double-and-add over the table 2^b G, canonical plain affine words.
__device__ __forceinline__ void gen_mul_words(const uint32_t s[8], const uint32_t* __restrict__ gtab, uint32_t o[16]) {
  xyzz acc = xyzz_inf();
  for (int b = 0; b < 254; b++) {
    if ((s[b >> 5] >> (b & 31)) & 1u) {
      aff g;
      ld_aff(gtab + (size_t)b * 16, g);
      acc = madd(acc, g);
    }
  }
  to_affine_words(acc, o);
}

__global__ void lagrange_kernel(Tau8 tw, uint32_t L, f29 c_mont, uint32_t tau_in_h, const f29* __restrict__ lo,
                                const f29* __restrict__ hi, const uint32_t* __restrict__ gtab,
                                uint32_t* __restrict__ out, uint64_t n) {
  const uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const f29 tau = reduce_full<FrP>(to_mont<FrP>(unpack(tw.w)));
  // omega_(2^L)^j = omega_(2^28)^(j 2^(28 - L)), exponent split over the two tables
  const uint32_t E = (uint32_t)j << (28 - L);
  const uint32_t ea = E & 0x3fffu, eb = E >> 14;
  const f29 wj = reduce_full<FrP>(mont_mul<FrP>(lo[ea], hi[eb]));
  f29 lm;
  if (tau_in_h) {
    uint32_t diff = 0;
#pragma unroll
    for (int i = 0; i < 9; i++) diff |= wj.l[i] ^ tau.l[i];
    lm = diff == 0 ? f29_from(FrP::ONE) : f29_zero();
  } else {
    const f29 d = reduce_full<FrP>(sub_k(tau, wj, FrP::K2));
    lm = mont_mul<FrP>(mont_mul<FrP>(c_mont, wj), mont_inv<FrP>(d));
  }
  uint32_t s[8], o[16];
  pack(from_mont<FrP>(lm), s);
  gen_mul_words(s, gtab, o);
  stw(out + j * 16, o, 4);
}

// sigma_i = product of the challenges of the folds where instance i is the
// left operand (adjacent pairs per level, odd last carried, BFS order).
__global__ void fold_sigma_kernel(const uint32_t* __restrict__ gammas, uint32_t m, uint32_t* __restrict__ sigma) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  f29 sg = f29_from(FrP::ONE);
  uint32_t pos = i, ml = m, goff = 0;
  while (ml > 1) {
    if ((pos & 1u) == 0 && pos + 1 < ml) {
      uint32_t gw[8];
      ldw(gammas + (size_t)(goff + pos / 2) * 8, gw, 2);
      sg = mont_mul<FrP>(sg, to_mont<FrP>(unpack(gw)));
    }
    goff += ml / 2;
    ml = (ml + 1) / 2;
    pos >>= 1;
  }
  uint32_t o[8];
  pack(from_mont<FrP>(sg), o);
  stw(sigma + (size_t)i * 8, o, 2);
}

__global__ void gather_kernel(const uint32_t* __restrict__ inst, uint32_t m, uint32_t k, uint32_t comp,
                              uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  uint32_t w[16];
  ldw(inst + ((size_t)i * k + comp) * 16, w, 4);
  stw(out + (size_t)i * 16, w, 4);
}

// ---------------------------------------------------------------- scan
constexpr uint32_t SCAN_ITEMS = 8;
constexpr uint32_t SCAN_BLOCK = MSM_NT * SCAN_ITEMS;

__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* sm, uint32_t* total) {
  const uint32_t tid = threadIdx.x;
  sm[tid] = v;
  __syncthreads();
  for (uint32_t d = 1; d < MSM_NT; d <<= 1) {
    const uint32_t t = tid >= d ? sm[tid - d] : 0;
    __syncthreads();
    sm[tid] += t;
    __syncthreads();
  }
  const uint32_t incl = sm[tid];
  *total = sm[MSM_NT - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(MSM_NT) scan_reduce_kernel(const uint32_t* in, uint32_t n, uint32_t* sums) {
  __shared__ uint32_t sm[MSM_NT];
  const uint32_t base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
  for (uint32_t q = 0; q < SCAN_ITEMS; q++)
    if (base + q < n) s += in[base + q];
  uint32_t tot;
  block_excl_scan(s, sm, &tot);
  if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(MSM_NT)
scan_apply_kernel(const uint32_t* in, uint32_t n, const uint32_t* sums, uint32_t nb, uint32_t* out,
                  uint32_t* copy) {
  __shared__ uint32_t sm[MSM_NT];
  const uint32_t base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS], s = 0;
  for (uint32_t q = 0; q < SCAN_ITEMS; q++) {
    v[q] = base + q < n ? in[base + q] : 0;
    s += v[q];
  }
  uint32_t tot;
  uint32_t run = block_excl_scan(s, sm, &tot) + sums[blockIdx.x];
  for (uint32_t q = 0; q < SCAN_ITEMS; q++) {
    if (base + q < n) {
      out[base + q] = run;
      if (copy) copy[base + q] = run;
    }
    run += v[q];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

// Whole scan in one workgroup for n <= SMALL_SCAN_MAX (each thread a run of
// at most 4 consecutive values).
constexpr uint32_t SMALL_SCAN_NT = 1024;
constexpr uint32_t SMALL_SCAN_MAX = 4 * SMALL_SCAN_NT;
__global__ void __launch_bounds__(SMALL_SCAN_NT)
scan_small_kernel(const uint32_t* in, uint32_t n, uint32_t* out, uint32_t* copy) {
  __shared__ uint32_t sm[SMALL_SCAN_NT];
  const uint32_t tid = threadIdx.x;
  const uint32_t per = (n + SMALL_SCAN_NT - 1) / SMALL_SCAN_NT;
  const uint32_t base = tid * per;
  uint32_t v = 0;
  for (uint32_t q = 0; q < per; q++)
    if (base + q < n) v += in[base + q];
  sm[tid] = v;
  __syncthreads();
  for (uint32_t d = 1; d < SMALL_SCAN_NT; d <<= 1) {
    const uint32_t t = tid >= d ? sm[tid - d] : 0u;
    __syncthreads();
    sm[tid] += t;
    __syncthreads();
  }
  uint32_t run = sm[tid] - v;
  for (uint32_t q = 0; q < per; q++) {
    if (base + q < n) {
      const uint32_t x = in[base + q];
      out[base + q] = run;
      if (copy) copy[base + q] = run;
      run += x;
    }
  }
  if (tid == SMALL_SCAN_NT - 1) out[n] = sm[tid];
}

// scan_apply for nb <= SCAN_BLOCK block sums that are not yet scanned: each
// block adds up the sums before its own (one block reduction) instead of a
// separate launch scanning them.
__global__ void __launch_bounds__(MSM_NT)
scan_apply_raw_kernel(const uint32_t* in, uint32_t n, const uint32_t* sums, uint32_t nb, uint32_t* out,
                      uint32_t* copy) {
  __shared__ uint32_t sm[MSM_NT];
  uint32_t pre = 0;
  for (uint32_t k = threadIdx.x; k < blockIdx.x; k += MSM_NT) pre += sums[k];
  uint32_t tot;
  block_excl_scan(pre, sm, &tot);
  pre = tot;
  const uint32_t base = blockIdx.x * SCAN_BLOCK + threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS], s = 0;
  for (uint32_t q = 0; q < SCAN_ITEMS; q++) {
    v[q] = base + q < n ? in[base + q] : 0;
    s += v[q];
  }
  uint32_t run = block_excl_scan(s, sm, &tot) + pre;
  for (uint32_t q = 0; q < SCAN_ITEMS; q++) {
    if (base + q < n) {
      out[base + q] = run;
      if (copy) copy[base + q] = run;
    }
    run += v[q];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == MSM_NT - 1) out[n] = run;
}

// Zero two arrays in one launch.
__global__ void fill_zero2_kernel(uint32_t* a, uint32_t na, uint32_t* b, uint32_t nb) {
  const uint32_t stride = gridDim.x * blockDim.x;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < na; i += stride) a[i] = 0;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < nb; i += stride) b[i] = 0;
}

inline uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

}  // namespace

// ================================================================ host side

uint32_t msm_default_c(uint32_t n) {
  uint32_t lg = 0;
  while ((1ull << (lg + 1)) <= n) lg++;
  int c = (int)lg - 3;
  if (c < 4) c = 4;
  if (c > 16) c = 16;
  return (uint32_t)c;
}

// Scalars per coarse-sort workgroup.  Measured on one MI355X: 1024 against
// 4096 takes MSMs of 2^14 / 2^16 points from 0.51 / 0.61 ms to 0.40 / 0.50
// ms (four times the workgroups to spread the digit counting over), with
// 2^20 and 2^22 unchanged within run-to-run noise.
constexpr uint32_t ACC_MIN_L = 4;

static void plan_common(MsmPlan& p, const Schedule& sch) {
  p.groups = p.nseg * p.Wb;
  p.nbins = p.groups * p.K;
  // coarse bins of 2^S bins each, sized for about sort_bin_entries (32768 by default) entries per coarse
  // bin when digits are spread evenly: a fine-level block of 4096 entries
  // then meets one or two coarse bins (few distinct bins, long runs), while
  // coarse-level blocks still write runs of useful length (measured best of
  // 8192 / 32768 / 131072 at 2^20; within 3% of the best at 2^22)
  {
    const uint64_t ent = (uint64_t)p.n * p.W;
    uint32_t S = 0;
    while (S < 8 && S + 1 < p.c && (ent << (S + 1)) <= (uint64_t)sch.sort_bin_entries * p.nbins) S++;
    // a coarse-level block histograms Wb*K >> S coarse bins in LDS (<= 64 KB)
    while (((p.Wb * p.K) >> S) > 16384u) S++;
    p.S = S;
  }
  p.ncoarse = p.nbins >> p.S;
  const uint64_t entries = (uint64_t)p.n * p.W;
  // Accumulation grid: whole rounds of acc_blocks_per_cu workgroups per
  // compute unit (a round is resident at once, so no unit waits on a partial
  // last one), as few rounds as keep slices within acc_max_slice entries, and
  // fewer workgroups when the n * W bound gives under ACC_MIN_L entries per
  // thread.  The kernel spreads the sorted total, known only on the device,
  // over the grid.
  const uint64_t per_round = (uint64_t)device_compute_units() * sch.acc_blocks_per_cu * MSM_NT;
  const uint64_t max_l = sch.acc_max_slice;
  const uint64_t rounds = std::max<uint64_t>(1, (entries + per_round * max_l - 1) / (per_round * max_l));
  p.L = ACC_MIN_L;
  p.acc_blocks = (uint32_t)cdiv(std::min<uint64_t>(rounds * per_round, cdiv(entries, ACC_MIN_L)), MSM_NT);
  if (p.acc_blocks == 0) p.acc_blocks = 1;
  // chunk length: short chains for one or a few bucket sets (latency), longer
  // ones when many sets already fill the chip (less bit-slice work)
  uint32_t lb = (uint64_t)p.groups * p.K >= (1u << 20) ? 16 : (p.K > (1u << 15) ? 8 : 4);
  if (sch.reduce_chunk) lb = sch.reduce_chunk;
  if (lb > p.K) lb = p.K;
  p.LB = lb;
  p.lgLB = 31 - __builtin_clz(lb);
  p.J = p.K / p.LB;
  p.nbits = 31 - __builtin_clz(p.J);
  // slice partials: at most 4 terms per thread of a 64-thread block (the
  // T slice has J terms, the others J / 2)
  uint32_t parts = (p.J + 255) / 256;
  if (parts < 1) parts = 1;
  p.parts = parts;
}

MsmPlan msm_plan_generic(uint32_t n, uint32_t c) {
  MsmPlan p{};
  p.n = n;
  p.c = c;
  p.W = (254 + c - 1) / c;
  p.K = 1u << (c - 1);
  p.table = 0;
  p.nseg = 1;
  p.Wb = p.W;
  p.tab_stride = 0;
  const Schedule sch = device_schedule();
  p.chunk = sch.sort_chunk;
  p.nitems = cdiv(n, p.chunk);
  plan_common(p, sch);
  return p;
}

MsmPlan msm_plan_table(const uint64_t* off, uint32_t nmsm, uint32_t c, uint32_t tab_stride) {
  MsmPlan p{};
  p.n = (uint32_t)off[nmsm];
  p.c = c;
  p.W = (254 + c - 1) / c;
  p.K = 1u << (c - 1);
  p.table = 1;
  p.nseg = nmsm;
  p.Wb = 1;
  p.tab_stride = tab_stride;
  const Schedule sch = device_schedule();
  p.chunk = sch.sort_chunk;
  p.nitems = 0;
  for (uint32_t b = 0; b < nmsm; b++) p.nitems += cdiv(off[b + 1] - off[b], p.chunk);
  plan_common(p, sch);
  return p;
}

// Scan: block sums, recursive scan of the sums, then per-block rescans.
size_t scan_tmp_words(uint32_t n) {
  size_t words = 0;
  while (n > SCAN_BLOCK) {
    const uint32_t nb = cdiv(n, SCAN_BLOCK);
    words += 2 * ((size_t)nb + 1) + 64;
    n = nb;
  }
  return words + 64;
}

hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp, hipStream_t s,
                          uint32_t* copy) {
  if (n <= SMALL_SCAN_MAX) {
    hipLaunchKernelGGL(scan_small_kernel, dim3(1), dim3(SMALL_SCAN_NT), 0, s, in, n, out, copy);
    return hipGetLastError();
  }
  const uint32_t nb = cdiv(n, SCAN_BLOCK);
  uint32_t* sums = tmp;                 // nb + 1
  uint32_t* scanned = tmp + nb + 1;     // nb + 1
  uint32_t* rest = scanned + nb + 1 + 32;
  hipLaunchKernelGGL(scan_reduce_kernel, dim3(nb), dim3(MSM_NT), 0, s, in, n, sums);
  hipError_t e;
  if (nb <= SCAN_BLOCK) {
    hipLaunchKernelGGL(scan_apply_raw_kernel, dim3(nb), dim3(MSM_NT), 0, s, in, n, sums, nb, out, copy);
  } else {
    if ((e = scan_exclusive(sums, scanned, nb, rest, s, nullptr))) return e;
    hipLaunchKernelGGL(scan_apply_kernel, dim3(nb), dim3(MSM_NT), 0, s, in, n, scanned, nb, out, copy);
  }
  return hipGetLastError();
}

namespace {
struct Layout {
  size_t off[18];
  size_t total;
};

Layout layout(const MsmPlan& p) {
  Layout L{};
  size_t o = 0;
  auto take = [&](int idx, size_t bytes) {
    L.off[idx] = o;
    o += (bytes + 255) & ~size_t(255);
  };
  const size_t ent = (size_t)p.n * p.W;
  const size_t nrec0 = 2 * (size_t)p.acc_blocks * MSM_NT;
  const size_t nrec1 = 2 * (size_t)p.acc_blocks;
  take(0, ent * 8);                                                     // pairs
  take(1, (size_t)p.nbins * 4);                                         // counts
  take(2, ((size_t)p.nbins + 1) * 4);                                   // offsets
  take(3, (size_t)p.nbins * 4);                                         // cursor
  take(4, scan_tmp_words(p.nbins) * 4);                                 // scan tmp
  take(5, ent * 4);                                                     // entries
  take(6, (size_t)p.nbins * XYZZ_WORDS * 4);                            // buckets
  take(7, nrec0 * REC_WORDS * 4);                                       // records, thread level (and odd levels)
  take(8, nrec1 * REC_WORDS * 4);                                       // records, even levels
  take(9, (size_t)p.groups * p.J * 2 * XYZZ_WORDS * 4);                 // vbuf
  take(10, (size_t)p.groups * XYZZ_WORDS * 4);                          // wsum
  take(11, ((size_t)p.nseg + 2) * 4);                                   // seg_off
  take(12, ((size_t)p.nitems + 1) * 16);                                // items
  take(13, (size_t)p.groups * (p.nbits + 1) * p.parts * XYZZ_WORDS * 4); // partial
  take(14, (size_t)p.ncoarse * 4);                                      // ccounts
  take(15, ((size_t)p.ncoarse + 1) * 4);                                // coff
  take(16, (size_t)p.ncoarse * 4);                                      // ccursor
  L.total = o;
  return L;
}
}  // namespace

size_t msm_workspace_bytes(const MsmPlan& p) { return layout(p).total; }

MsmBuffers msm_carve(const MsmPlan& p, void* base) {
  const Layout L = layout(p);
  char* b = static_cast<char*>(base);
  MsmBuffers m;
  m.pairs = reinterpret_cast<uint2*>(b + L.off[0]);
  m.counts = reinterpret_cast<uint32_t*>(b + L.off[1]);
  m.offsets = reinterpret_cast<uint32_t*>(b + L.off[2]);
  m.cursor = reinterpret_cast<uint32_t*>(b + L.off[3]);
  m.scan_tmp = reinterpret_cast<uint32_t*>(b + L.off[4]);
  m.entries = reinterpret_cast<uint32_t*>(b + L.off[5]);
  m.buckets = reinterpret_cast<uint32_t*>(b + L.off[6]);
  m.rec[0] = reinterpret_cast<uint32_t*>(b + L.off[7]);
  m.rec[1] = reinterpret_cast<uint32_t*>(b + L.off[8]);
  m.vbuf = reinterpret_cast<uint32_t*>(b + L.off[9]);
  m.wsum = reinterpret_cast<uint32_t*>(b + L.off[10]);
  m.seg_off = reinterpret_cast<uint32_t*>(b + L.off[11]);
  m.items = reinterpret_cast<uint4*>(b + L.off[12]);
  m.partial = reinterpret_cast<uint32_t*>(b + L.off[13]);
  m.ccounts = reinterpret_cast<uint32_t*>(b + L.off[14]);
  m.coff = reinterpret_cast<uint32_t*>(b + L.off[15]);
  m.ccursor = reinterpret_cast<uint32_t*>(b + L.off[16]);
  return m;
}

static size_t rec_lds_bytes() { return (size_t)MSM_SLOTS * (2 + XYZZ_WORDS) * 4; }

static hipError_t set_lds_limits() {
  static bool done = false;
  if (done) return hipSuccess;
  hipError_t e;
  const int fine_lds = (int)(FINE_LDS_BINS * 4);
  if ((e = hipFuncSetAttribute((const void*)fine_count_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               fine_lds)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)fine_scatter_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               fine_lds)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)fine_scatter_lite_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)FINE_LITE_LDS)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)fine_scatter_staged_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)FINE_STAGED_LDS)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)coarse_scatter_staged_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)STAGED_MAX_LDS)))
    return e;
  if ((e = hipFuncSetAttribute((const void*)record_reduce_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)rec_lds_bytes())))
    return e;
  done = true;
  return hipSuccess;
}

// Segment offsets and histogram items, from host offsets via kernel arguments.
static hipError_t launch_items(const MsmPlan& p, const uint64_t* off, const MsmBuffers& b, hipStream_t s) {
  uint32_t item = 0;
  for (uint32_t first = 0; first < p.nseg || first == 0; first += SEG_ARGS) {
    SegArgs a{};
    a.first = first;
    a.count = std::min<uint32_t>(SEG_ARGS, p.nseg - first);
    if (!p.table) {  // generic: one segment covering every scalar
      a.first = 0;
      a.count = 1;
      a.off[0] = 0;
      a.off[1] = p.n;
      a.item0[0] = 0;
    } else {
      for (uint32_t t = 0; t < a.count; t++) {
        a.off[t] = (uint32_t)off[first + t];
        a.item0[t] = item;
        item += cdiv(off[first + t + 1] - off[first + t], p.chunk);
      }
      a.off[a.count] = (uint32_t)off[first + a.count];
    }
    hipLaunchKernelGGL(make_items_kernel, dim3(1), dim3(SEG_ARGS), 0, s, a, p.chunk, b.seg_off, b.items);
    if (!p.table) break;
  }
  return hipGetLastError();
}

hipError_t msm_run(const MsmPlan& p, const uint64_t* off, const uint32_t* points, const uint32_t* scalars,
                   const MsmBuffers& b, uint32_t* out, hipStream_t s, hipEvent_t after_accumulate,
                   hipEvent_t before_accumulate) {
  hipError_t e;
  if ((e = set_lds_limits())) return e;
  const uint32_t nout = p.nseg;
  if (p.n == 0) {
    for (uint32_t i = 0; i < nout; i++) hipLaunchKernelGGL(zero16_kernel, dim3(1), dim3(64), 0, s, out + 16 * i);
    if (before_accumulate && (e = hipStreamWaitEvent(s, before_accumulate, 0))) return e;
    if (after_accumulate && (e = hipEventRecord(after_accumulate, s))) return e;
    return hipGetLastError();
  }
  const ProfToken t_sort = prof_begin("msm.sort", s);
  const bool multi = p.table && p.nseg > 1;
  if (multi && (e = launch_items(p, off, b, s))) return e;
  const uint4* items = multi ? b.items : nullptr;
  hipLaunchKernelGGL(fill_zero2_kernel, dim3(std::min(cdiv(p.nbins, 256), 1024u)), dim3(256), 0, s, b.counts,
                     p.nbins, b.ccounts, p.ncoarse);
  const size_t clds = (size_t)((p.Wb * p.K) >> p.S) * 4;
  // the staged scatter serves one segment whose block's pairs and bins fit
  // LDS; the counting kernel keeps its blocks' counts for it in the entries
  // buffer, which the fine level fills only later
  const size_t slds = staged_lds_words((p.Wb * p.K) >> p.S) * 4 + (size_t)p.chunk * p.W * 8;
  const bool staged_coarse = !items && slds <= STAGED_MAX_LDS &&
                             (uint64_t)p.nitems * ((p.Wb * p.K) >> p.S) <= (uint64_t)p.n * p.W;
  if (p.nitems) {
    hipLaunchKernelGGL(coarse_count_kernel, dim3(p.nitems), dim3(MSM_NT), clds, s, scalars, p, items, b.ccounts,
                       staged_coarse ? b.entries : nullptr);
  }
  if ((e = scan_exclusive(b.ccounts, b.coff, p.ncoarse, b.scan_tmp, s, b.ccursor))) return e;
  // Staged scatters pay off when most digits are nonzero (uniform scalars);
  // small quantized scalars leave most windows zero, and their blocks are
  // better served by the direct scatters.  Both kernels of a level are
  // launched; each reads the sorted total and only one of them runs.
  const uint32_t dense_min = (uint32_t)std::min<uint64_t>((uint64_t)p.n * p.W / 2, UINT32_MAX - 1);
  if (p.nitems) {
    hipLaunchKernelGGL(coarse_scatter_kernel, dim3(p.nitems), dim3(MSM_NT), clds, s, scalars, p, items,
                       b.seg_off, b.ccursor, b.pairs, b.coff + p.ncoarse, staged_coarse ? dense_min : UINT32_MAX);
    if (staged_coarse) {
      hipLaunchKernelGGL(coarse_scatter_staged_kernel, dim3(std::min(p.nitems, device_compute_units())),
                         dim3(STAGED_NT), slds, s, scalars, p, b.entries, b.ccursor, b.pairs, b.coff + p.ncoarse,
                         dense_min);
    }
  }
  const uint32_t fine_blocks = (uint32_t)cdiv((uint64_t)p.n * p.W, FINE_CHUNK);
  const size_t flds = (size_t)FINE_LDS_BINS * 4;
  if (fine_blocks) {
    hipLaunchKernelGGL(fine_count_kernel, dim3(fine_blocks), dim3(MSM_NT), flds, s, b.pairs, b.coff + p.ncoarse, p,
                       b.counts);
  }
  if ((e = scan_exclusive(b.counts, b.offsets, p.nbins, b.scan_tmp, s, b.cursor))) return e;
  if (fine_blocks) {
    hipLaunchKernelGGL(fine_scatter_kernel, dim3(fine_blocks), dim3(MSM_NT), flds, s, b.pairs, b.coff + p.ncoarse,
                       p, b.cursor, b.entries, dense_min);
    if (p.S >= 7) {
      hipLaunchKernelGGL(fine_scatter_staged_kernel, dim3(std::min(fine_blocks, 2 * device_compute_units())),
                         dim3(MSM_NT), FINE_STAGED_LDS, s, b.pairs, b.coff + p.ncoarse, p, b.cursor, b.entries,
                         dense_min);
    } else {
      hipLaunchKernelGGL(fine_scatter_lite_kernel, dim3(std::min(fine_blocks, 4 * device_compute_units())),
                         dim3(MSM_NT), FINE_LITE_LDS, s, b.pairs, b.coff + p.ncoarse, p, b.cursor, b.entries,
                         dense_min);
    }
  }
  prof_end(t_sort, s);
  if (before_accumulate && (e = hipStreamWaitEvent(s, before_accumulate, 0))) return e;
  const ProfToken t_acc = prof_begin("msm.accumulate", s);
  if ((e = msm_launch_accumulate(p, b, points, s))) return e;
  prof_end(t_acc, s);
  if (after_accumulate && (e = hipEventRecord(after_accumulate, s))) return e;
  if (p.nbits + 1 > FIN_SLICES) return hipErrorInvalidValue;
  // partial-tree levels until a slice has at most 8 partials per finishing quad
  const uint32_t qps = fin_qps(p.nbits + 1);
  uint32_t levels = 0;
  for (uint32_t np = p.parts; np > 8 * qps; np = (np + BITS_NT - 1) / BITS_NT) levels++;
  const ProfToken t_red = prof_begin("msm.reduce", s);
  uint32_t nrec = 2 * p.acc_blocks * MSM_NT;
  int cur = 0;
  while (true) {
    const uint32_t g2 = cdiv(nrec, MSM_SLOTS);
    const bool last = g2 == 1;
    hipLaunchKernelGGL(record_reduce_kernel, dim3(g2), dim3(MSM_NT), rec_lds_bytes(), s, b.rec[cur], nrec,
                       b.buckets, last ? nullptr : b.rec[cur ^ 1]);
    if (last) break;
    nrec = 2 * g2;
    cur ^= 1;
  }
  // chunk sums on quads while they fill at most about two waves per SIMD
  if ((uint64_t)p.groups * p.J * 4 <= (1u << 17)) {
    hipLaunchKernelGGL(chunk_sums_quad_kernel, dim3(cdiv((uint64_t)p.groups * p.J * 4, 64)), dim3(64), 0, s,
                       b.buckets, b.counts, p, b.vbuf);
  } else {
    hipLaunchKernelGGL(chunk_sums_kernel, dim3(cdiv((uint64_t)p.groups * p.J, 64)), dim3(64), 0, s, b.buckets,
                       b.counts, p, b.vbuf);
  }
  if ((uint64_t)p.groups * p.J * 4 <= (1u << 17)) {
    hipLaunchKernelGGL(bit_sums_quad_kernel, dim3(p.parts, p.nbits + 1, p.groups), dim3(BITS_QUADS * 4), 0, s, b.vbuf,
                       p, b.partial);
  } else {
    hipLaunchKernelGGL(bit_sums_kernel, dim3(p.parts, p.nbits + 1, p.groups), dim3(BITS_NT), 0, s, b.vbuf, p,
                       b.partial);
  }
  // tree levels ping-pong between the partial buffer and the (now free) chunk buffer
  uint32_t* pin = b.partial;
  uint32_t* pout = b.vbuf;
  uint32_t np = p.parts;
  for (uint32_t l = 0; l < levels; l++) {
    const uint32_t nn = (np + BITS_NT - 1) / BITS_NT;
    hipLaunchKernelGGL(partial_tree_kernel, dim3(nn, p.nbits + 1, p.groups), dim3(BITS_NT), 0, s, pin, np,
                       p.nbits + 1, pout);
    np = nn;
    uint32_t* t = pin;
    pin = pout;
    pout = t;
  }
  if (p.table) {
    hipLaunchKernelGGL(bit_finish_kernel, dim3(p.groups), dim3(FIN_NT), 0, s, pin, np, qps, p, out, nullptr);
  } else {
    hipLaunchKernelGGL(bit_finish_kernel, dim3(p.groups), dim3(FIN_NT), 0, s, pin, np, qps, p, nullptr, b.wsum);
    hipLaunchKernelGGL(combine_kernel, dim3(1), dim3(64), 0, s, b.wsum, p.W, p.c, out);
  }
  prof_end(t_red, s);
  return hipGetLastError();
}

hipError_t msm_points_to_mont(const uint32_t* plain, uint32_t* mont, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(to_mont_kernel, dim3(cdiv(n, 256)), dim3(256), 0, s, plain, mont, n);
  return hipGetLastError();
}

hipError_t msm_build_table(const uint32_t* plain_points, uint32_t* tab, uint64_t n, uint32_t c, uint32_t W,
                           hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(build_table_kernel, dim3(cdiv(n, 128)), dim3(128), 0, s, plain_points, tab, n, c, W);
  return hipGetLastError();
}

size_t srs_gtab_words() { return 256 * 16; }

hipError_t srs_from_tau(Tau8 tau, uint32_t* out, uint64_t n, uint32_t* gtab, hipStream_t s) {
  hipLaunchKernelGGL(gen_table_kernel, dim3(4), dim3(64), 0, s, gtab);
  if (n == 0) return hipGetLastError();
  hipLaunchKernelGGL(srs_kernel, dim3(cdiv(n, 128)), dim3(128), 0, s, tau, gtab, out, n);
  return hipGetLastError();
}

hipError_t srs_lagrange_from_tau(Tau8 tau, uint32_t L, f29 c_mont, bool tau_in_h, const f29* tw_lo,
                                 const f29* tw_hi, uint32_t* out, uint32_t* gtab, hipStream_t s) {
  hipLaunchKernelGGL(gen_table_kernel, dim3(4), dim3(64), 0, s, gtab);
  const uint64_t n = 1ull << L;
  hipLaunchKernelGGL(lagrange_kernel, dim3(cdiv(n, 128)), dim3(128), 0, s, tau, L, c_mont, tau_in_h ? 1u : 0u, tw_lo,
                     tw_hi, gtab, out, n);
  return hipGetLastError();
}

hipError_t fold_sigmas(const uint32_t* gammas, uint32_t m, uint32_t* sigma, hipStream_t s) {
  hipLaunchKernelGGL(fold_sigma_kernel, dim3(cdiv(m, 64)), dim3(64), 0, s, gammas, m, sigma);
  return hipGetLastError();
}

hipError_t gather_component(const uint32_t* inst, uint32_t m, uint32_t k, uint32_t comp, uint32_t* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(gather_kernel, dim3(cdiv(m, 64)), dim3(64), 0, s, inst, m, k, comp, out);
  return hipGetLastError();
}

}  // namespace zk
