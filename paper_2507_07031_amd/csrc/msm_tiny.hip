// Small commitments over a prepared SRS by a table of small multiples.
//
// The KZG commitment Q = sum_i s_i P_i (Polynomial Commitment preliminaries)
// with every scalar written in 64 signed 4-bit digits,
//   s_i = sum_w d_(i,w) 16^w,   |d_(i,w)| <= 8,
// is Q = sum_i sum_w d_(i,w) 16^w P_i.  The table holds m 16^w P_i for
// m = 1..8, w < 64 and the first TINY_MAX points, so every (i, w) term is one
// table point, negated for a negative digit.  The n * 64 terms are summed by
// trees on quads: no sort, no buckets and no bucket reduction, whose dependent
// chains set the latency of a Pippenger run of any size.
//
// Digits: with the negation trick (s > (r-1)/2 becomes r - s and the terms
// change sign) a scalar has at most 253 bits.  With v_w the 4-bit windows and
// b_w = [v_w >= 8], d_w = v_w + b_(w-1) - 16 b_w lies in [-8, 8], depends only
// on windows w and w-1, and sum_w d_w 16^w = s - b_63 16^64 = s (v_63 <= 1).
#include "curve.h"
#include "curve_quad.h"
#include "msm.h"
#include "msm_store.h"
#include "msm_tiny.h"

namespace zk {

namespace {

// Montgomery affine point from 16 packed words; false for (0, 0) = infinity.
__device__ __forceinline__ bool tiny_ld_aff(const uint32_t* p, aff& a) {
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

// XYZZ -> Montgomery canonical affine words, infinity -> zeros.
__device__ void tiny_st_aff(uint32_t* p, const xyzz& a) {
  uint32_t w[16];
  if (is_inf(a)) {
#pragma unroll
    for (int i = 0; i < 16; i++) w[i] = 0;
  } else {
    const f29 I = mont_inv<Fq>(mont_mul<Fq>(a.ZZ, a.ZZZ));  // 1 / (ZZ ZZZ)
    pack(reduce_full<Fq>(mont_mul<Fq>(a.X, mont_mul<Fq>(I, a.ZZZ))), w);
    pack(reduce_full<Fq>(mont_mul<Fq>(a.Y, mont_mul<Fq>(I, a.ZZ))), w + 8);
  }
#pragma unroll
  for (int q = 0; q < 4; q++)
    reinterpret_cast<uint4*>(p)[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

// One thread per (w, i): from row w/4 of the 16-bit table (16^(4 (w/4)) P_i),
// 4 (w mod 4) doublings give 16^w P_i, then its multiples 1..8.
__global__ void __launch_bounds__(256) tiny_build_kernel(const uint32_t* __restrict__ tab16, uint64_t tab_n, uint32_t nt,
                                                          uint32_t* __restrict__ tiny) {
  const uint64_t idx = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (uint64_t)TINY_WINDOWS * nt) return;
  const uint32_t w = (uint32_t)(idx / nt), i = (uint32_t)(idx % nt);
  aff b;
  const bool fin = tiny_ld_aff(tab16 + ((uint64_t)(w >> 2) * tab_n + i) * 16, b);
  xyzz p = fin ? from_aff(b) : xyzz_inf();
  for (uint32_t t = 0; t < 4 * (w & 3u); t++) p = dbl(p);
  xyzz m = p;
  for (uint32_t k = 0; k < TINY_MULTS; k++) {
    tiny_st_aff(tiny + ((uint64_t)(w * TINY_MULTS + k) * nt + i) * 16, m);
    if (k + 1 < TINY_MULTS) m = add(m, p);
  }
}

// Sum of the TINY_NT points held in sm (36 words each) on the workgroup's 64
// quads: pair k combines slots k and k + half into slot k, so no quad reads a
// slot another quad writes in the same level.  The sum ends in slot 0.
__device__ __forceinline__ void tiny_tree(uint32_t* sm) {
  const uint32_t quad = threadIdx.x >> 2, c = threadIdx.x & 3u;
  for (uint32_t half = TINY_NT / 2; half >= 1; half >>= 1) {
    for (uint32_t k = quad; k < half; k += TINY_NT / 4) {  // quad-uniform
      const f29 a = ldq(sm + k * XYZZ_WORDS, c);
      const f29 b = ldq(sm + (k + half) * XYZZ_WORDS, c);
      stq(sm + k * XYZZ_WORDS, c, quad_add(a, b));
    }
    __syncthreads();
  }
}

// (r-1)/2 in 32-bit words, for the negation trick
__constant__ uint32_t TINY_FR_HALF[8] = {0xf8000000u, 0xa1f0fac9u, 0x3cdcb848u, 0x9419f424u,
                                         0x40c0ac2eu, 0xdc2822dbu, 0x7098d014u, 0x18322739u};

// Workgroup k takes the terms (i, w) = (4k + t / 64, t mod 64) and writes
// their sum to partial[k] (XYZZ).
__global__ void __launch_bounds__(TINY_NT)
tiny_terms_kernel(const uint32_t* __restrict__ scalars, uint32_t n, const uint32_t* __restrict__ tiny, uint32_t nt,
                  uint32_t* __restrict__ partial) {
  __shared__ uint32_t sm[TINY_NT * XYZZ_WORDS];
  const uint32_t t = threadIdx.x;
  const uint32_t g = blockIdx.x * TINY_NT + t;
  const uint32_t i = g / TINY_WINDOWS, w = g % TINY_WINDOWS;
  xyzz p = xyzz_inf();
  if (i < n) {
    uint32_t s[8];
#pragma unroll
    for (int q = 0; q < 2; q++) {
      const uint4 v = reinterpret_cast<const uint4*>(scalars + (size_t)i * 8)[q];
      s[4 * q] = v.x;
      s[4 * q + 1] = v.y;
      s[4 * q + 2] = v.z;
      s[4 * q + 3] = v.w;
    }
    unsigned br = 0;
#pragma unroll
    for (int q = 0; q < 8; q++) (void)__builtin_subc(TINY_FR_HALF[q], s[q], br, &br);
    const bool neg = br != 0;  // s > (r-1)/2
    if (neg) {
      unsigned b2 = 0;
#pragma unroll
      for (int q = 0; q < 8; q++) s[q] = __builtin_subc(FrP::M32[q], s[q], b2, &b2);
    }
    const uint32_t vw = (s[w >> 3] >> (4 * (w & 7u))) & 15u;
    const uint32_t vp = w ? (s[(w - 1) >> 3] >> (4 * ((w - 1) & 7u))) & 15u : 0u;
    const int d = (int)vw + (vp >= 8u ? 1 : 0) - (vw >= 8u ? 16 : 0);
    if (d != 0) {
      const uint32_t m = (uint32_t)(d < 0 ? -d : d);
      aff a;
      if (tiny_ld_aff(tiny + ((uint64_t)(w * TINY_MULTS + m - 1) * nt + i) * 16, a))
        p = from_aff(((d < 0) != neg) ? aff_neg(a) : a);
    }
  }
  st_xyzz(sm + t * XYZZ_WORDS, p);
  __syncthreads();
  tiny_tree(sm);
  const uint32_t quad = t >> 2, c = t & 3u;
  if (quad == 0) stq(partial + (size_t)blockIdx.x * XYZZ_WORDS, c, ldq(sm, c));
}

// Workgroup k sums in[256 k .. 256 k + 255] (fewer at the end of count) into
// out_xyzz[k]; with out_affine (one workgroup), the sum is written as
// canonical plain affine words instead.
__global__ void __launch_bounds__(TINY_NT)
tiny_sum_kernel(const uint32_t* __restrict__ in, uint32_t count, uint32_t* __restrict__ out_xyzz,
                uint32_t* __restrict__ out_affine) {
  __shared__ uint32_t sm[TINY_NT * XYZZ_WORDS];
  const uint32_t t = threadIdx.x;
  const uint32_t g = blockIdx.x * TINY_NT + t;
  uint4* dst = reinterpret_cast<uint4*>(sm + t * XYZZ_WORDS);
  if (g < count) {
    const uint4* src = reinterpret_cast<const uint4*>(in + (size_t)g * XYZZ_WORDS);
#pragma unroll
    for (int q = 0; q < 9; q++) dst[q] = src[q];
  } else {
#pragma unroll
    for (int q = 0; q < 9; q++) dst[q] = make_uint4(0, 0, 0, 0);
  }
  __syncthreads();
  tiny_tree(sm);
  const uint32_t quad = t >> 2, c = t & 3u;
  if (quad != 0) return;
  if (!out_affine) {
    stq(out_xyzz + (size_t)blockIdx.x * XYZZ_WORDS, c, ldq(sm, c));
    return;
  }
  xyzz r = quad_gather(ldq(sm, c));
  if (c != 0) return;
  force_vgpr(r);
  uint32_t o[16];
  to_affine_words(r, o);
#pragma unroll
  for (int q = 0; q < 4; q++)
    reinterpret_cast<uint4*>(out_affine)[q] = make_uint4(o[4 * q], o[4 * q + 1], o[4 * q + 2], o[4 * q + 3]);
}

}  // namespace

uint64_t msm_tiny_table_points(uint32_t nt) { return (uint64_t)TINY_WINDOWS * TINY_MULTS * nt; }

hipError_t msm_build_tiny_table(const uint32_t* tab16, uint32_t tab_c, uint32_t tab_W, uint64_t tab_n, uint32_t nt,
                                uint32_t* tiny, hipStream_t s) {
  if (nt == 0) return hipSuccess;
  // the build reads rows 0 .. 15 (16^(4 r) P_i) of a 16-bit-window table
  if (tab_c != 16 || tab_W < TINY_WINDOWS / 4 || nt > tab_n) return hipErrorInvalidValue;
  const uint64_t threads = (uint64_t)TINY_WINDOWS * nt;
  hipLaunchKernelGGL(tiny_build_kernel, dim3((uint32_t)((threads + 255) / 256)), dim3(256), 0, s, tab16, tab_n, nt,
                     tiny);
  return hipGetLastError();
}

size_t msm_tiny_workspace_bytes(uint32_t n) {
  const uint64_t b1 = ((uint64_t)n * TINY_WINDOWS + TINY_NT - 1) / TINY_NT;
  const uint64_t b2 = (b1 + TINY_NT - 1) / TINY_NT;
  return (size_t)(b1 + b2) * XYZZ_WORDS * 4;
}

hipError_t msm_tiny_run(const uint32_t* tiny, uint32_t nt, const uint32_t* scalars, uint32_t n, void* workspace,
                        uint32_t* out16, hipStream_t s, hipEvent_t after_terms) {
  if (n == 0 || n > nt || n > TINY_MAX) return hipErrorInvalidValue;
  uint32_t count = (uint32_t)(((uint64_t)n * TINY_WINDOWS + TINY_NT - 1) / TINY_NT);
  uint32_t* a = static_cast<uint32_t*>(workspace);
  uint32_t* b = a + (size_t)count * XYZZ_WORDS;
  hipLaunchKernelGGL(tiny_terms_kernel, dim3(count), dim3(TINY_NT), 0, s, scalars, n, tiny, nt, a);
  hipError_t e;
  if (after_terms && (e = hipEventRecord(after_terms, s))) return e;
  while (count > TINY_NT) {
    const uint32_t next = (count + TINY_NT - 1) / TINY_NT;
    hipLaunchKernelGGL(tiny_sum_kernel, dim3(next), dim3(TINY_NT), 0, s, a, count, b, nullptr);
    std::swap(a, b);
    count = next;
  }
  hipLaunchKernelGGL(tiny_sum_kernel, dim3(1), dim3(TINY_NT), 0, s, a, count, nullptr, out16);
  return hipGetLastError();
}

}  // namespace zk
