// Multi-scalar multiplication over BN254 G2, sum_i s_i P_i, for the G2
// commitments [f(tau)]_2 = sum_i f_i [tau^i]_2 that MulScalar, Mul and
// MatMul send beside their G1 ones.
//
// Pippenger with signed 8-bit digits over a pre-shifted table, as for G1:
// tab[w n + i] = 2^(8 w) P_i, so digit w of s_i selects table point (w, i)
// and every window shares one set of 128 buckets (|digit| = 1..128); the
// window sums need no doubling chain.
//   count    per workgroup, a histogram of the digits' buckets (LDS atomics)
//   offsets  one workgroup per bucket scans the workgroups' counts; one more
//            forms the bucket offsets and the accumulation threads per bucket
//   scatter  digits recomputed, entries (table index, sign) written at the
//            workgroup's reserved positions
//   accumulate  each thread adds up to L consecutive entries of one
//            bucket (mixed additions of table points), one partial each
//   buckets  two workgroups per bucket: its partials summed (LDS tree)
//   bitsum   sum_b (b + 1) B_b split by the bits of b + 1: one workgroup per
//            bit j sums the buckets with bit j set and doubles the sum j times
//   final    the eight bit sums added, affine
// Field and point arithmetic: g2.h; the bucket, bit and final sums run their
// additions on quads of lanes (g2_quad.h).
#include "g2.h"
#include "g2_quad.h"
#include "g2msm.h"
#include "prof.h"

namespace zk {

namespace {

constexpr uint32_t G2_NT = 256;
constexpr uint32_t G2_L = 32;               // entries per accumulation thread, at least
constexpr uint32_t G2_XYZZ_WORDS = 72;      // four Fq2 coordinates, 9 limbs per component
constexpr uint32_t G2_BUCKET_NT = 512;      // threads of a bucket workgroup (128 quads)

struct Words8x {
  uint32_t w[8];
};

uint32_t cdiv(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

__device__ __forceinline__ void ldw(const uint32_t* p, uint32_t* w, int n4) {
  for (int i = 0; i < n4; i++) {
    const uint4 v = reinterpret_cast<const uint4*>(p)[i];
    w[4 * i] = v.x;
    w[4 * i + 1] = v.y;
    w[4 * i + 2] = v.z;
    w[4 * i + 3] = v.w;
  }
}

__device__ __forceinline__ void stw(uint32_t* p, const uint32_t* w, int n4) {
  for (int i = 0; i < n4; i++) reinterpret_cast<uint4*>(p)[i] = make_uint4(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3]);
}

// Montgomery affine point <-> packed words (x0 x1 y0 y1, 8 words each, canonical).
__device__ __forceinline__ void st_aff(uint32_t* p, const g2aff& a) {
  uint32_t w[32];
  pack(a.x.c0, w);
  pack(a.x.c1, w + 8);
  pack(a.y.c0, w + 16);
  pack(a.y.c1, w + 24);
  stw(p, w, 8);
}

__device__ __forceinline__ bool ld_aff(const uint32_t* p, g2aff& a) {
  uint32_t w[32];
  ldw(p, w, 8);
  uint32_t o = 0;
  for (int i = 0; i < 32; i++) o |= w[i];
  a.x.c0 = unpack(w);
  a.x.c1 = unpack(w + 8);
  a.y.c0 = unpack(w + 16);
  a.y.c1 = unpack(w + 24);
  return o != 0;
}

__device__ __forceinline__ void st_xyzz(uint32_t* p, const g2xyzz& a) {
  const f29* c[8] = {&a.X.c0, &a.X.c1, &a.Y.c0, &a.Y.c1, &a.ZZ.c0, &a.ZZ.c1, &a.ZZZ.c0, &a.ZZZ.c1};
  for (int k = 0; k < 8; k++)
    for (int i = 0; i < 9; i++) p[9 * k + i] = c[k]->l[i];
}

__device__ __forceinline__ g2xyzz ld_xyzz(const uint32_t* p) {
  g2xyzz a;
  f29* c[8] = {&a.X.c0, &a.X.c1, &a.Y.c0, &a.Y.c1, &a.ZZ.c0, &a.ZZ.c1, &a.ZZZ.c0, &a.ZZZ.c1};
  for (int k = 0; k < 8; k++)
    for (int i = 0; i < 9; i++) c[k]->l[i] = p[9 * k + i];
  return a;
}

// Signed 8-bit digit of window w (carry from the lower windows): the caller
// walks w = 0, 1, ... keeping `carry`.
__device__ __forceinline__ int32_t next_digit(const uint32_t s[8], uint32_t w, uint32_t& carry) {
  const uint32_t v = ((s[w >> 2] >> (8 * (w & 3))) & 255u) + carry;
  if (v > 128u) {
    carry = 1;
    return (int32_t)v - 256;
  }
  carry = 0;
  return (int32_t)v;
}

// ---- setup ---------------------------------------------------------------------

// gtab[b] = 2^b H, b < 254
__global__ void g2_gen_table_kernel(uint32_t* gtab) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= 254) return;
  uint32_t w[32];
  for (int i = 0; i < 32; i++) w[i] = G2_GEN[i];
  g2aff h;
  g2_from_words(w, h);
  g2xyzz acc = g2_from_aff(h);
  for (uint32_t t = 0; t < b; t++) acc = g2_dbl(acc);
  g2aff a;
  g2_to_aff(acc, a);
  st_aff(gtab + (size_t)b * G2_AFF_WORDS, a);
}

__global__ void g2_srs_kernel(Words8x tw, const uint32_t* __restrict__ gtab, uint32_t* __restrict__ out,
                              uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const f29 tau = reduce_full<FrP>(to_mont<FrP>(unpack(tw.w)));
  uint32_t e[8] = {(uint32_t)i, (uint32_t)(i >> 32), 0, 0, 0, 0, 0, 0};
  const f29 ti = (i == 0) ? f29_from(FrP::ONE) : mont_pow<FrP>(tau, e);
  uint32_t s[8];
  pack(from_mont<FrP>(ti), s);
  g2xyzz acc = g2_inf();
  for (int b = 0; b < 254; b++) {
    if ((s[b >> 5] >> (b & 31)) & 1u) {
      g2aff g;
      ld_aff(gtab + (size_t)b * G2_AFF_WORDS, g);
      acc = g2_madd(acc, g);
    }
  }
  uint32_t o[32];
  g2_to_words(acc, o);
  stw(out + i * 32, o, 8);
}

__global__ void g2_table_kernel(const uint32_t* __restrict__ points, uint32_t* __restrict__ tab, uint64_t n) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t w[32];
  ldw(points + i * 32, w, 8);
  g2aff p;
  const bool fin = g2_from_words(w, p);
  g2xyzz acc = fin ? g2_from_aff(p) : g2_inf();
  for (uint32_t win = 0; win < G2_W; win++) {
    g2aff a;
    if (g2_to_aff(acc, a)) {
      st_aff(tab + ((uint64_t)win * n + i) * G2_AFF_WORDS, a);
    } else {
      for (int k = 0; k < 32; k++) w[k] = 0;
      stw(tab + ((uint64_t)win * n + i) * G2_AFF_WORDS, w, 8);
    }
    if (win + 1 < G2_W)
      for (uint32_t t = 0; t < G2_C; t++) acc = g2_dbl(acc);
  }
}

// ---- MSM -------------------------------------------------------------------------

__global__ __launch_bounds__(G2_NT) void g2_count_kernel(const uint32_t* __restrict__ scalars, uint64_t n,
                                                         uint32_t* __restrict__ blockhist) {
  __shared__ uint32_t hist[G2_K];
  for (uint32_t b = threadIdx.x; b < G2_K; b += G2_NT) hist[b] = 0;
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * G2_NT + threadIdx.x;
  if (i < n) {
    uint32_t s[8];
    ldw(scalars + i * 8, s, 2);
    uint32_t carry = 0;
    for (uint32_t w = 0; w < G2_W; w++) {
      const int32_t d = next_digit(s, w, carry);
      if (d) atomicAdd(&hist[(d < 0 ? -d : d) - 1], 1u);
    }
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < G2_K; b += G2_NT) blockhist[(size_t)blockIdx.x * G2_K + b] = hist[b];
}

// One workgroup per bucket b: blockhist[k][b] becomes workgroup k's position
// inside bucket b (an exclusive scan over the workgroups); tot[b] = the
// bucket's entry count.
__global__ __launch_bounds__(G2_NT) void g2_bucket_scan_kernel(uint32_t* __restrict__ blockhist, uint32_t nblk,
                                                               uint32_t* __restrict__ tot) {
  __shared__ uint32_t part[G2_NT];
  const uint32_t b = blockIdx.x;
  const uint32_t per = (nblk + G2_NT - 1) / G2_NT;
  const uint32_t k0 = threadIdx.x * per;
  uint32_t sum = 0;
  for (uint32_t k = k0; k < min(k0 + per, nblk); k++) sum += blockhist[(size_t)k * G2_K + b];
  part[threadIdx.x] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (uint32_t t = 0; t < G2_NT; t++) {
      const uint32_t c = part[t];
      part[t] = run;
      run += c;
    }
    tot[b] = run;
  }
  __syncthreads();
  uint32_t run = part[threadIdx.x];
  for (uint32_t k = k0; k < min(k0 + per, nblk); k++) {
    const uint32_t c = blockhist[(size_t)k * G2_K + b];
    blockhist[(size_t)k * G2_K + b] = run;
    run += c;
  }
}

// One workgroup of G2_K threads: off[b] = first entry of bucket b (off[G2_K]
// = total); tp[b] = first accumulation thread of bucket b (tp[G2_K] = total).
__global__ __launch_bounds__(G2_K) void g2_offsets_kernel(const uint32_t* __restrict__ tot, uint32_t L,
                                                          uint32_t* __restrict__ off, uint32_t* __restrict__ tp) {
  if (threadIdx.x == 0) {
    uint32_t a = 0, t = 0;
    for (uint32_t k = 0; k < G2_K; k++) {
      const uint32_t c = tot[k];
      off[k] = a;
      tp[k] = t;
      a += c;
      t += (c + L - 1) / L;
    }
    off[G2_K] = a;
    tp[G2_K] = t;
  }
}

__global__ __launch_bounds__(G2_NT) void g2_scatter_kernel(const uint32_t* __restrict__ scalars, uint64_t n,
                                                           uint64_t n_tab, const uint32_t* __restrict__ base,
                                                           const uint32_t* __restrict__ off,
                                                           uint32_t* __restrict__ entries) {
  __shared__ uint32_t cur[G2_K];
  for (uint32_t b = threadIdx.x; b < G2_K; b += G2_NT) cur[b] = off[b] + base[(size_t)blockIdx.x * G2_K + b];
  __syncthreads();
  const uint64_t i = (uint64_t)blockIdx.x * G2_NT + threadIdx.x;
  if (i < n) {
    uint32_t s[8];
    ldw(scalars + i * 8, s, 2);
    uint32_t carry = 0;
    for (uint32_t w = 0; w < G2_W; w++) {
      const int32_t d = next_digit(s, w, carry);
      if (d) {
        const uint32_t pos = atomicAdd(&cur[(d < 0 ? -d : d) - 1], 1u);
        entries[pos] = (uint32_t)((uint64_t)w * n_tab + i) | (d < 0 ? 0x80000000u : 0u);
      }
    }
  }
}

// A mixed G2 addition keeps about 300 registers live; held to 256 (two waves
// per SIMD, about 280 bytes per lane spilled to scratch) the accumulation
// runs 5% faster than with one wave per SIMD and no spills, because the
// second wave hides the first's dependent-chain and load latency.
__global__ __launch_bounds__(G2_NT) __attribute__((amdgpu_waves_per_eu(2, 2))) void g2_accumulate_kernel(const uint32_t* __restrict__ tab,
                                                              const uint32_t* __restrict__ entries,
                                                              const uint32_t* __restrict__ off,
                                                              const uint32_t* __restrict__ tp, uint32_t L,
                                                              uint32_t* __restrict__ partial) {
  __shared__ uint32_t t0[G2_K + 1];
  for (uint32_t b = threadIdx.x; b <= G2_K; b += G2_NT) t0[b] = tp[b];
  __syncthreads();
  const uint32_t t = blockIdx.x * G2_NT + threadIdx.x;
  if (t >= t0[G2_K]) return;
  // bucket of thread t: the last b with t0[b] <= t
  uint32_t lo = 0, hi = G2_K;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (t0[mid] <= t) lo = mid;
    else hi = mid;
  }
  const uint32_t b = lo;
  const uint32_t beg = off[b] + (t - t0[b]) * L;
  const uint32_t end = min(beg + L, off[b + 1]);
  g2xyzz acc = g2_inf();
  for (uint32_t e = beg; e < end; e++) {
    const uint32_t en = entries[e];
    g2aff p;
    if (!ld_aff(tab + (size_t)(en & 0x7fffffffu) * G2_AFF_WORDS, p)) continue;
    if (en >> 31) p = g2_aff_neg(p);
    acc = g2_madd(acc, p);
  }
  st_xyzz(partial + (size_t)t * G2_XYZZ_WORDS, acc);
}

// G2_SPLIT workgroups per bucket (so that the 128 buckets fill the compute
// units): workgroup (b, h) sums every G2_SPLIT-th block of the bucket's
// partials into bsum[G2_SPLIT b + h]; B_b is the sum of those.  Each quad of
// lanes carries one running sum (g2_quad.h), a chain of quad additions over
// the partials it owns, then a tree over the quads.
constexpr uint32_t G2_SPLIT = 2;

__global__ __launch_bounds__(G2_BUCKET_NT) void g2_bucket_kernel(const uint32_t* __restrict__ partial,
                                                                 const uint32_t* __restrict__ tp,
                                                                 uint32_t* __restrict__ bsum) {
  constexpr uint32_t NQ = G2_BUCKET_NT / 4;
  __shared__ uint32_t lds[NQ * G2_XYZZ_WORDS];
  const uint32_t b = blockIdx.x / G2_SPLIT, h0 = blockIdx.x % G2_SPLIT;
  const uint32_t q = threadIdx.x >> 2, c = threadIdx.x & 3u;
  const uint32_t first = tp[b], last = tp[b + 1];
  fp2 acc = fp2_zero();
  for (uint32_t t = first + h0 * NQ + q; t < last; t += G2_SPLIT * NQ)
    acc = g2q_add(acc, ldq2(partial + (size_t)t * G2_XYZZ_WORDS, c));
  stq2(lds + q * G2_XYZZ_WORDS, c, acc);
  __syncthreads();
  for (uint32_t h = NQ / 2; h > 0; h >>= 1) {
    if (q < h) {
      acc = g2q_add(acc, ldq2(lds + (q + h) * G2_XYZZ_WORDS, c));
      stq2(lds + q * G2_XYZZ_WORDS, c, acc);
    }
    __syncthreads();
  }
  if (q == 0) stq2(bsum + (size_t)blockIdx.x * G2_XYZZ_WORDS, c, acc);
}

// B_b from its G2_SPLIT workgroup sums.
__device__ __forceinline__ fp2 g2_bucket_sum(const uint32_t* bsum, uint32_t b, uint32_t c) {
  fp2 v = ldq2(bsum + (size_t)G2_SPLIT * b * G2_XYZZ_WORDS, c);
  for (uint32_t h = 1; h < G2_SPLIT; h++) v = g2q_add(v, ldq2(bsum + (size_t)(G2_SPLIT * b + h) * G2_XYZZ_WORDS, c));
  return v;
}

// sum_b (b + 1) B_b = sum_j 2^j T_j, where T_j is the sum of the B_b whose
// b + 1 has bit j set (j < 8; T_7 = B_127).  One workgroup per j, on its own
// compute unit: T_j as an LDS tree of quad additions over its 64 buckets
// (g2_quad.h), then j quad doublings.  The eight workgroups run side by side,
// so the dependent chain is 6 additions and at most 7 doublings instead of
// a 128-bucket suffix scan and tree on one compute unit.
constexpr uint32_t G2_BITS = 8;   // bits of b + 1 <= G2_K
static_assert((1u << (G2_BITS - 1)) == G2_K, "b + 1 <= G2_K needs G2_BITS bits");

__global__ __launch_bounds__(2 * G2_K) void g2_bitsum_kernel(const uint32_t* __restrict__ bsum,
                                                               uint32_t* __restrict__ tsum) {
  constexpr uint32_t NQ = G2_K / 2;  // buckets with bit j of b + 1 set, j < 7
  __shared__ uint32_t lds[NQ * G2_XYZZ_WORDS];
  const uint32_t j = blockIdx.x, q = threadIdx.x >> 2, c = threadIdx.x & 3u;
  fp2 v;
  if (j + 1 < G2_BITS) {
    // the q-th value in [1, 128) with bit j set: q with a one inserted at bit j
    const uint32_t val = ((q >> j) << (j + 1)) | (1u << j) | (q & ((1u << j) - 1));
    v = g2_bucket_sum(bsum, val - 1, c);
    stq2(lds + q * G2_XYZZ_WORDS, c, v);
    __syncthreads();
    for (uint32_t h = NQ / 2; h > 0; h >>= 1) {
      if (q < h) {
        v = g2q_add(v, ldq2(lds + (q + h) * G2_XYZZ_WORDS, c));
        stq2(lds + q * G2_XYZZ_WORDS, c, v);
      }
      __syncthreads();
    }
  } else {
    v = g2_bucket_sum(bsum, G2_K - 1, c);
  }
  if (q == 0) {
    for (uint32_t i = 0; i < j; i++) v = g2q_dbl(v);
    stq2(tsum + (size_t)j * G2_XYZZ_WORDS, c, v);
  }
}

// The eight 2^j T_j summed (one quad each, an LDS tree of three levels) and
// the result made affine.
__global__ __launch_bounds__(4 * G2_BITS) void g2_final_kernel(const uint32_t* __restrict__ tsum,
                                                               uint32_t* __restrict__ out) {
  __shared__ uint32_t lds[G2_BITS * G2_XYZZ_WORDS];
  const uint32_t q = threadIdx.x >> 2, c = threadIdx.x & 3u;
  fp2 v = ldq2(tsum + (size_t)q * G2_XYZZ_WORDS, c);
  stq2(lds + q * G2_XYZZ_WORDS, c, v);
  __syncthreads();
  for (uint32_t h = G2_BITS / 2; h > 0; h >>= 1) {
    if (q < h) {
      v = g2q_add(v, ldq2(lds + (q + h) * G2_XYZZ_WORDS, c));
      stq2(lds + q * G2_XYZZ_WORDS, c, v);
    }
    __syncthreads();
  }
  const g2xyzz r = g2q_gather(v);
  if (threadIdx.x == 0) {
    uint32_t o[32];
    g2_to_words(r, o);
    stw(out, o, 8);
  }
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

hipError_t g2_srs_from_tau(const uint32_t tau[8], uint32_t* out, uint64_t n, uint32_t* gtab, hipStream_t s) {
  hipLaunchKernelGGL(g2_gen_table_kernel, dim3(4), dim3(64), 0, s, gtab);
  if (n == 0) return hipGetLastError();
  Words8x t;
  for (int i = 0; i < 8; i++) t.w[i] = tau[i];
  hipLaunchKernelGGL(g2_srs_kernel, dim3(cdiv(n, 64)), dim3(64), 0, s, t, gtab, out, n);
  return hipGetLastError();
}

hipError_t g2_build_table(const uint32_t* points, uint32_t* tab, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(g2_table_kernel, dim3(cdiv(n, 64)), dim3(64), 0, s, points, tab, n);
  return hipGetLastError();
}

// Entries per accumulation thread: at least G2_L, more once the threads
// exceed about 2^17 (enough waves), which keeps the partial sums per bucket
// (summed by G2_SPLIT workgroups each) few.
uint32_t g2_entries_per_thread(uint64_t ent) {
  uint64_t L = ent >> 17;
  if (L < G2_L) L = G2_L;
  return (uint32_t)L;
}

size_t g2_msm_scratch_bytes(uint64_t n) {
  const uint64_t nblk = cdiv(n ? n : 1, G2_NT);
  const uint64_t ent = (uint64_t)G2_W * n;
  const uint64_t thr = ent / g2_entries_per_thread(ent) + G2_K + 1;
  return align256(nblk * G2_K * 4) + 3 * align256((G2_K + 1) * 4) + align256(ent * 4) +
         align256(thr * G2_XYZZ_WORDS * 4) + align256((size_t)G2_SPLIT * G2_K * G2_XYZZ_WORDS * 4) +
         align256((size_t)G2_BITS * G2_XYZZ_WORDS * 4);
}

hipError_t g2_msm(const uint32_t* tab, uint64_t n_tab, const uint32_t* scalars, uint64_t n, uint32_t* out,
                  void* scratch, hipStream_t s) {
  const uint32_t nblk = cdiv(n ? n : 1, G2_NT);
  const uint64_t ent = (uint64_t)G2_W * n;
  const uint32_t L = g2_entries_per_thread(ent);
  const uint64_t thr = ent / L + G2_K + 1;
  char* p = static_cast<char*>(scratch);
  uint32_t* blockhist = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)nblk * G2_K * 4);
  uint32_t* tot = reinterpret_cast<uint32_t*>(p);
  p += align256((G2_K + 1) * 4);
  uint32_t* off = reinterpret_cast<uint32_t*>(p);
  p += align256((G2_K + 1) * 4);
  uint32_t* tp = reinterpret_cast<uint32_t*>(p);
  p += align256((G2_K + 1) * 4);
  uint32_t* entries = reinterpret_cast<uint32_t*>(p);
  p += align256(ent * 4);
  uint32_t* partial = reinterpret_cast<uint32_t*>(p);
  p += align256(thr * G2_XYZZ_WORDS * 4);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(p);
  p += align256((size_t)G2_SPLIT * G2_K * G2_XYZZ_WORDS * 4);
  uint32_t* tsum = reinterpret_cast<uint32_t*>(p);

  const ProfToken tok = prof_begin("g2.msm", s);
  hipLaunchKernelGGL(g2_count_kernel, dim3(nblk), dim3(G2_NT), 0, s, scalars, n, blockhist);
  hipLaunchKernelGGL(g2_bucket_scan_kernel, dim3(G2_K), dim3(G2_NT), 0, s, blockhist, nblk, tot);
  hipLaunchKernelGGL(g2_offsets_kernel, dim3(1), dim3(G2_K), 0, s, tot, L, off, tp);
  hipLaunchKernelGGL(g2_scatter_kernel, dim3(nblk), dim3(G2_NT), 0, s, scalars, n, n_tab, blockhist, off, entries);
  const ProfToken acc = prof_begin("g2.accumulate", s);
  hipLaunchKernelGGL(g2_accumulate_kernel, dim3(cdiv(thr, G2_NT)), dim3(G2_NT), 0, s, tab, entries, off, tp, L,
                     partial);
  prof_end(acc, s);
  hipLaunchKernelGGL(g2_bucket_kernel, dim3(G2_SPLIT * G2_K), dim3(G2_BUCKET_NT), 0, s, partial, tp, bsum);
  hipLaunchKernelGGL(g2_bitsum_kernel, dim3(G2_BITS), dim3(2 * G2_K), 0, s, bsum, tsum);
  hipLaunchKernelGGL(g2_final_kernel, dim3(1), dim3(4 * G2_BITS), 0, s, tsum, out);
  prof_end(tok, s);
  return hipGetLastError();
}

}  // namespace zk
