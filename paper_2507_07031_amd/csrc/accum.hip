// One step of the accumulation prover (Parallel Accumulation, prover steps
// 4-6) on the device parts of two accumulators acc (weighted by gamma) and
// acc':
//   C''_i = gamma C_i + C'_i                       (the k G1 commitments)
//   E''   = E' + sum_(j=1)^(d-1) gamma^j E_j + gamma^d E    (committed errors)
//   v''   = gamma v + v'                           (Fr parts: mu, pi, r_i, m_i)
//   e''   = e' + sum_j gamma^j e_j + gamma^d e     (Fr error vectors)
// and the challenge gamma derived from a transcript by hashing.
//
// The G1 outputs are short sums of scalar multiples by powers of one
// challenge, all independent: every scalar multiple other than by 1 runs in
// its own quad (curve_quad.h), split by the endomorphism into two 128-bit
// halves (glv.h) and computed by Straus's method with 4-bit windows over
// tables of 1..15 times the point and its image kept in scratch memory: 32
// window steps of four doublings and up to two additions.  The Fr parts are
// elementwise Horner combinations streamed through HBM.
#include "accum.h"
#include "curve.h"
#include "curve_quad.h"
#include "glv.h"
#include "msm_store.h"
#include "prof.h"

namespace zk {

namespace {

constexpr uint32_t ACC_NT = 64;        // threads per workgroup: 16 quads
constexpr uint32_t TAB_WORDS = 16 * 36;  // one term's table: multiples 0..15, 36 words each
constexpr uint32_t RLC_NT = 256;

__device__ __forceinline__ void ld8w(const uint32_t* p, uint32_t w[8]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
  w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}

__device__ __forceinline__ void st8w(uint32_t* p, const uint32_t w[8]) {
  reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

// Term t of output o: its point (scalar gamma^t).  Output o < k is
// gamma C[o] + C2[o] (terms C2[o], C[o]); output k is E'' (terms E2, Ej..., E).
__device__ __forceinline__ const uint32_t* term_point(const uint32_t* C, const uint32_t* C2, const uint32_t* E,
                                                      const uint32_t* E2, const uint32_t* Ej, uint32_t k,
                                                      uint32_t d, uint32_t o, uint32_t t) {
  if (o < k) return t == 0 ? C2 + (size_t)o * 16 : C + (size_t)o * 16;
  if (t == 0) return E2;
  if (t == d) return E;
  return Ej + (size_t)(t - 1) * 16;
}

// Lane c's coordinate of an affine point in XYZZ form on a quad (x, y, 1, 1;
// all zero for infinity), selected limb by limb so that no copy of the
// whole point is indexed by the lane number.
__device__ __forceinline__ f29 quad_aff_coord(const aff& a, bool fin, uint32_t c) {
  const f29 one = f29_from(Fq::ONE);
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = !fin ? 0u : c == 0 ? a.x.l[i] : c == 1 ? a.y.l[i] : one.l[i];
  return r;
}

// Coordinate c of a point held by a quad, negated when neg is set (the y
// coordinate, lane 1): 4q - Y keeps the coordinate bounds of the formulas.
__device__ __forceinline__ f29 quad_cneg(const f29& v, uint32_t c, bool neg) {
  return (neg && c == 1) ? sub_k(f29_zero(), v, Fq::K4) : v;
}

// k P on a quad for canonical k < r and a plain affine point P (words;
// (0, 0) = infinity): k is split by the endomorphism (glv.h),
// k = +-k1 +- k2 lambda with k1, k2 < 2^128, and k P = (+-k1) P + (+-k2) phi(P)
// runs as Straus over 32 windows of 4 bits with tables of 1..15 times +-P
// and +-phi(P) at T1 and T1 + TAB_WORDS, where
// phi(X, Y, ZZ, ZZZ) = (beta X, Y, ZZ, ZZZ).  Returns lane c's coordinate.
__device__ __forceinline__ f29 glv_quad_mul(const uint32_t (&sw)[8], const uint32_t* __restrict__ P,
                                            uint32_t* __restrict__ T1,
                            uint32_t c) {
  uint32_t k1[4], k2[4];
  bool n1, n2;
  glv_split(sw, k1, n1, k2, n2);
  uint32_t* T2 = T1 + TAB_WORDS;
  {
    uint32_t w[16];
    ld8w(P, w);
    ld8w(P + 8, w + 8);
    aff a;
    const bool fin = aff_from_plain_words(w, a);
    const f29 base = quad_cneg(quad_aff_coord(a, fin, c), c, fin && n1);
    stq(T1 + 36, c, base);
    f29 cur = quad_dbl(base);
    stq(T1 + 2 * 36, c, cur);
    for (uint32_t m = 3; m < 16; m++) {
      cur = quad_add(cur, base);
      stq(T1 + m * 36, c, cur);
    }
    uint32_t bw[8];
#pragma unroll
    for (int i = 0; i < 8; i++) bw[i] = GlvConst::BETA[i];
    const f29 beta = reduce_full<Fq>(to_mont<Fq>(unpack(bw)));
    for (uint32_t m = 1; m < 16; m++) {
      f29 v = ldq(T1 + m * 36, c);
      if (c == 0) v = mont_mul<Fq>(v, beta);
      stq(T2 + m * 36, c, quad_cneg(v, c, fin && n1 != n2));
    }
  }
  // windows from the top: word wi of each half (constant after unrolling,
  // so the halves stay in registers), eight 4-bit digits per word
  f29 acc = f29_zero();
#pragma unroll
  for (int wi = 3; wi >= 0; --wi) {
    const uint32_t w1 = k1[wi], w2 = k2[wi];
    for (int sub = 7; sub >= 0; --sub) {
      if (wi != 3 || sub != 7) {
        acc = quad_dbl(acc);
        acc = quad_dbl(acc);
        acc = quad_dbl(acc);
        acc = quad_dbl(acc);
      }
      const uint32_t d1 = (w1 >> (sub * 4)) & 15u;
      const uint32_t d2 = (w2 >> (sub * 4)) & 15u;
      if (d1) acc = quad_add(acc, ldq(T1 + d1 * 36, c));
      if (d2) acc = quad_add(acc, ldq(T2 + d2 * 36, c));
    }
  }
  return acc;
}

// One quad per (output, term) whose scalar gamma^t is not 1, all at once:
// quad q of wave w < nwc computes gamma C[16 w + q] for output 16 w + q < k,
// and quad q of the last wave gamma^(q+1) P_(q+1) of the error output for
// q < d (glv_quad_mul).  The term of scalar 1 is added to the result; the
// error output's quads first sum their terms in LDS.
__global__ __launch_bounds__(ACC_NT) void acc_fold_g1_kernel(const uint32_t* __restrict__ C,
                                                             const uint32_t* __restrict__ C2, uint32_t k,
                                                             const uint32_t* __restrict__ E,
                                                             const uint32_t* __restrict__ E2,
                                                             const uint32_t* __restrict__ Ej, uint32_t d,
                                                             const uint32_t* __restrict__ gamma, uint32_t nwc,
                                                             uint32_t* __restrict__ C_out,
                                                             uint32_t* __restrict__ E_out,
                                                             uint32_t* __restrict__ scratch) {
  __shared__ uint32_t sm[16 * 36];
  const uint32_t wave = blockIdx.x, q = threadIdx.x >> 2, c = quad_lane();
  const bool err = wave == nwc;
  const uint32_t o = err ? k : wave * 16 + q;  // output
  const uint32_t t = err ? q + 1 : 1;          // term
  const bool active = err ? t <= d : o < k;    // uniform over each quad
  f29 acc = f29_zero();
  if (active) {
    // scalar gamma^t, canonical words, computed alike by the lanes of the quad
    uint32_t sw[8];
    {
      uint32_t gw[8];
      ld8w(gamma, gw);
      const f29 gm = reduce_full<FrP>(to_mont<FrP>(unpack(gw)));
      f29 p = gm;
      for (uint32_t i = 1; i < t; i++) p = reduce_full<FrP>(mont_mul<FrP>(p, gm));
      pack(from_mont<FrP>(p), sw);
    }
    acc = glv_quad_mul(sw, term_point(C, C2, E, E2, Ej, k, d, o, t),
                       scratch + ((size_t)wave * 16 + q) * 2 * TAB_WORDS, c);
  }
  if (!err) {
    if (!active) return;  // whole quads leave together
  } else {
    // the error output: the terms of quads 0 .. d-1 (zero elsewhere) summed by a tree
    stq(sm + q * 36, c, acc);
    __syncthreads();
    for (uint32_t h = 8; h > 0; h >>= 1) {
      if (q < h) {
        acc = quad_add(acc, ldq(sm + (q + h) * 36, c));
        stq(sm + q * 36, c, acc);
      }
      __syncthreads();
    }
    if (q != 0) return;
  }
  // plus the term of scalar 1 (C2[o], or E2)
  {
    uint32_t w[16];
    const uint32_t* P = term_point(C, C2, E, E2, Ej, k, d, o, 0);
    ld8w(P, w);
    ld8w(P + 8, w + 8);
    aff a;
    if (aff_from_plain_words(w, a)) acc = quad_add(acc, quad_aff_coord(a, true, c));
  }
  xyzz r = quad_gather(acc);
  if (c == 0) {
    force_vgpr(r);
    uint32_t out[16];
    to_affine_words(r, out);
    uint32_t* dst = err ? E_out : C_out + (size_t)o * 16;
    st8w(dst, out);
    st8w(dst + 8, out + 8);
  }
}

// Linear combination of m points per component by per-term scalar multiples:
// block (b, j) computes sigma_i P_(i, j) for its 64 terms i = 64 b + q on
// quads q (glv_quad_mul) and sums them by an LDS tree into partial (b, j),
// or, with one workgroup per component, writes the sum affine itself; the
// finishing kernel sums a component's partials and writes it affine.
constexpr uint32_t RLC_TERMS_NT = 256;  // 64 quads
__global__ __launch_bounds__(RLC_TERMS_NT) void g1_rlc_terms_kernel(const uint32_t* __restrict__ pts,
                                                                    const uint32_t* __restrict__ sigma, uint32_t m,
                                                                    uint32_t k, uint32_t* __restrict__ tabs,
                                                                    uint32_t* __restrict__ partial,
                                                                    uint32_t* __restrict__ out) {
  __shared__ uint32_t sm[64 * 36];
  const uint32_t b = blockIdx.x, j = blockIdx.y, q = threadIdx.x >> 2, c = quad_lane();
  const uint32_t i = b * 64 + q;
  const size_t slot = (size_t)j * gridDim.x + b;
  f29 acc = f29_zero();
  if (i < m) {  // uniform over each quad
    uint32_t sw[8];
    ld8w(sigma + (size_t)i * 8, sw);
    acc = glv_quad_mul(sw, pts + ((size_t)i * k + j) * 16, tabs + (slot * 64 + q) * 2 * TAB_WORDS, c);
  }
  stq(sm + q * 36, c, acc);
  __syncthreads();
  for (uint32_t h = 32; h > 0; h >>= 1) {
    if (q < h) {
      acc = quad_add(acc, ldq(sm + (q + h) * 36, c));
      stq(sm + q * 36, c, acc);
    }
    __syncthreads();
  }
  if (q != 0) return;
  if (!out) {
    stq(partial + slot * 36, c, acc);
    return;
  }
  // a single workgroup per component: the sum is final, written affine here
  xyzz r = quad_gather(acc);
  if (c == 0) {
    force_vgpr(r);
    uint32_t o[16];
    to_affine_words(r, o);
    st8w(out + (size_t)j * 16, o);
    st8w(out + (size_t)j * 16 + 8, o + 8);
  }
}

__global__ __launch_bounds__(64) void g1_rlc_finish_kernel(const uint32_t* __restrict__ partial, uint32_t nblk,
                                                          uint32_t* __restrict__ out) {
  __shared__ uint32_t sm[16 * 36];
  const uint32_t j = blockIdx.x, q = threadIdx.x >> 2, c = quad_lane();
  f29 acc = f29_zero();
  for (uint32_t b = q; b < nblk; b += 16) acc = quad_add(acc, ldq(partial + ((size_t)j * nblk + b) * 36, c));
  stq(sm + q * 36, c, acc);
  __syncthreads();
  for (uint32_t h = 8; h > 0; h >>= 1) {
    if (q < h) {
      acc = quad_add(acc, ldq(sm + (q + h) * 36, c));
      stq(sm + q * 36, c, acc);
    }
    __syncthreads();
  }
  if (q != 0) return;
  xyzz r = quad_gather(acc);
  if (c == 0) {
    force_vgpr(r);
    uint32_t o[16];
    to_affine_words(r, o);
    st8w(out + (size_t)j * 16, o);
    st8w(out + (size_t)j * 16 + 8, o + 8);
  }
}

__global__ __launch_bounds__(RLC_NT) void fr_rlc_kernel(const uint32_t* __restrict__ v0,
                                                        const uint32_t* __restrict__ vmid,
                                                        const uint32_t* __restrict__ vlast, uint32_t d,
                                                        uint64_t len, const uint32_t* __restrict__ gamma,
                                                        uint32_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * RLC_NT + threadIdx.x;
  if (i >= len) return;
  uint32_t w[8];
  ld8w(gamma, w);
  const f29 gm = reduce_full<FrP>(to_mont<FrP>(unpack(w)));
  ld8w(vlast + i * 8, w);
  f29 acc = unpack(w);
  for (int32_t t = (int32_t)d - 1; t >= 1; --t) {
    ld8w(vmid + ((uint64_t)(t - 1) * len + i) * 8, w);
    acc = add_n(unpack(w), mont_mul<FrP>(acc, gm));
  }
  ld8w(v0 + i * 8, w);
  acc = add_n(unpack(w), mont_mul<FrP>(acc, gm));
  pack(reduce_full<FrP>(acc), w);
  st8w(out + i * 8, w);
}

// ---- SHA-256 (FIPS 180-4) ---------------------------------------------------
// Round constants: the first 32 bits of the fractional parts of the cube
// roots of the first 64 primes; initial value: the same of the square roots
// of the first 8 primes (FIPS 180-4, 4.2.2 and 5.3.3).
__constant__ uint32_t SHA_K[64] = {
    0x428a2f98u, 0x71374491u, 0xb5c0fbcfu, 0xe9b5dba5u, 0x3956c25bu, 0x59f111f1u, 0x923f82a4u, 0xab1c5ed5u,
    0xd807aa98u, 0x12835b01u, 0x243185beu, 0x550c7dc3u, 0x72be5d74u, 0x80deb1feu, 0x9bdc06a7u, 0xc19bf174u,
    0xe49b69c1u, 0xefbe4786u, 0x0fc19dc6u, 0x240ca1ccu, 0x2de92c6fu, 0x4a7484aau, 0x5cb0a9dcu, 0x76f988dau,
    0x983e5152u, 0xa831c66du, 0xb00327c8u, 0xbf597fc7u, 0xc6e00bf3u, 0xd5a79147u, 0x06ca6351u, 0x14292967u,
    0x27b70a85u, 0x2e1b2138u, 0x4d2c6dfcu, 0x53380d13u, 0x650a7354u, 0x766a0abbu, 0x81c2c92eu, 0x92722c85u,
    0xa2bfe8a1u, 0xa81a664bu, 0xc24b8b70u, 0xc76c51a3u, 0xd192e819u, 0xd6990624u, 0xf40e3585u, 0x106aa070u,
    0x19a4c116u, 0x1e376c08u, 0x2748774cu, 0x34b0bcb5u, 0x391c0cb3u, 0x4ed8aa4au, 0x5b9cca4fu, 0x682e6ff3u,
    0x748f82eeu, 0x78a5636fu, 0x84c87814u, 0x8cc70208u, 0x90befffau, 0xa4506cebu, 0xbef9a3f7u, 0xc67178f2u};
__constant__ uint32_t SHA_H0[8] = {0x6a09e667u, 0xbb67ae85u, 0x3c6ef372u, 0xa54ff53au,
                                   0x510e527fu, 0x9b05688cu, 0x1f83d9abu, 0x5be0cd19u};

__device__ __forceinline__ uint32_t rotr(uint32_t x, uint32_t n) { return (x >> n) | (x << (32 - n)); }

// Byte b of the message prefix || data || padding || 64-bit bit length.
__device__ __forceinline__ uint32_t msg_byte(const uint8_t* data, uint64_t bytes, uint8_t prefix, uint64_t total,
                                             uint64_t b) {
  const uint64_t L = bytes + 1;
  if (b == 0) return prefix;
  if (b < L) return data[b - 1];
  if (b == L) return 0x80u;
  if (b >= total - 8) {
    const uint64_t bits = L * 8;
    return (uint32_t)(bits >> (8 * (total - 1 - b))) & 0xffu;
  }
  return 0;
}

// One compression of a 64-byte block (FIPS 180-4, 6.2.2), schedule kept in a
// rolling window of 16 registers.
__device__ __forceinline__ void sha256_block(uint32_t h[8], const uint32_t blk[16]) {
  uint32_t W[16];
#pragma unroll
  for (int t = 0; t < 16; t++) W[t] = blk[t];
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll
  for (int t = 0; t < 64; t++) {
    uint32_t wt;
    if (t < 16) {
      wt = W[t];
    } else {
      const uint32_t w15 = W[(t - 15) & 15], w2 = W[(t - 2) & 15];
      const uint32_t s0 = rotr(w15, 7) ^ rotr(w15, 18) ^ (w15 >> 3);
      const uint32_t s1 = rotr(w2, 17) ^ rotr(w2, 19) ^ (w2 >> 10);
      wt = W[t & 15] + s0 + W[(t - 7) & 15] + s1;
      W[t & 15] = wt;
    }
    const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    const uint32_t ch = (e & f) ^ (~e & g);
    const uint32_t t1 = hh + S1 + ch + SHA_K[t] + wt;
    const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    const uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
    hh = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + S0 + mj;
  }
  h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

// Compression of one block from its full 64-word message schedule.
__device__ __forceinline__ void sha256_rounds(uint32_t h[8], const uint32_t* __restrict__ W) {
  uint32_t a = h[0], b = h[1], c = h[2], d = h[3], e = h[4], f = h[5], g = h[6], hh = h[7];
#pragma unroll
  for (int t = 0; t < 64; t++) {
    const uint32_t S1 = rotr(e, 6) ^ rotr(e, 11) ^ rotr(e, 25);
    const uint32_t ch = (e & f) ^ (~e & g);
    const uint32_t t1 = hh + S1 + ch + SHA_K[t] + W[t];
    const uint32_t S0 = rotr(a, 2) ^ rotr(a, 13) ^ rotr(a, 22);
    const uint32_t mj = (a & b) ^ (a & c) ^ (b & c);
    hh = g;
    g = f;
    f = e;
    e = d + t1;
    d = c;
    c = b;
    b = a;
    a = t1 + S0 + mj;
  }
  h[0] += a; h[1] += b; h[2] += c; h[3] += d; h[4] += e; h[5] += f; h[6] += g; h[7] += hh;
}

// Both messages 0x00 || data and 0x01 || data have the same padded layout
// and differ only in their first byte.  For 64 blocks at a time, lane b
// gathers block b's big-endian words and expands its message schedule into
// LDS; lanes 0 and 1 then run the rounds for prefix 0 and 1, the sequential
// part.  Block 0 is compressed inline by each of the two lanes with its own
// first byte.  Lane 0 then reduces the 512-bit little-endian concatenation
// of the two digests modulo r.
constexpr uint32_t TR_CHUNK = 64;  // blocks prepared per round of the 64 lanes
__global__ void transcript_kernel(const uint8_t* __restrict__ data, uint64_t bytes, f29 c_2_256,
                                  uint32_t* __restrict__ out) {
  __shared__ uint32_t Wsh[TR_CHUNK * 64];
  __shared__ uint32_t dig[2][8];
  const uint32_t lane = threadIdx.x;
  const uint64_t L = bytes + 1;
  const uint64_t total = ((L + 8) / 64 + 1) * 64;
  const uint64_t nblk = total / 64;
  uint32_t h[8];
  for (int i = 0; i < 8; i++) h[i] = SHA_H0[i];
  for (uint64_t c0 = 0; c0 < nblk; c0 += TR_CHUNK) {
    const uint64_t bi = c0 + lane;
    if (lane < TR_CHUNK && bi < nblk) {
      uint32_t* W = Wsh + lane * 64;
      for (int t = 0; t < 16; t++) {
        uint32_t v = 0;
        for (int q = 0; q < 4; q++) v = (v << 8) | msg_byte(data, bytes, 0, total, bi * 64 + 4 * t + q);
        W[t] = v;
      }
      for (int t = 16; t < 64; t++) {
        const uint32_t w15 = W[t - 15], w2 = W[t - 2];
        const uint32_t s0 = rotr(w15, 7) ^ rotr(w15, 18) ^ (w15 >> 3);
        const uint32_t s1 = rotr(w2, 17) ^ rotr(w2, 19) ^ (w2 >> 10);
        W[t] = W[t - 16] + s0 + W[t - 7] + s1;
      }
    }
    __syncthreads();
    if (lane < 2) {
      const uint64_t n = min((uint64_t)TR_CHUNK, nblk - c0);
      for (uint64_t b = 0; b < n; b++) {
        if (c0 + b == 0) {
          uint32_t w[16];
          for (int t = 0; t < 16; t++) w[t] = Wsh[t];
          w[0] = (w[0] & 0x00ffffffu) | (lane << 24);
          sha256_block(h, w);
        } else {
          sha256_rounds(h, Wsh + b * 64);
        }
      }
    }
    __syncthreads();
  }
  if (lane < 2)
    for (int i = 0; i < 8; i++) dig[lane][i] = __builtin_bswap32(h[i]);  // digest bytes as little-endian words
  __syncthreads();
  if (lane == 0) {
    const f29 lo = unpack(dig[0]);
    const f29 hi = unpack(dig[1]);
    // lo + hi 2^256 mod r: hi times 2^256 2^261 by a Montgomery product
    const f29 v = add_n(lo, mont_mul<FrP>(hi, c_2_256));
    uint32_t w[8];
    pack(reduce_full<FrP>(v), w);
    st8w(out, w);
  }
}

}  // namespace

// Waves of the commitment outputs (16 quads each); the error output takes one more.
static uint32_t acc_commit_waves(uint32_t k) { return (k + 15) / 16; }

size_t acc_fold_g1_scratch_bytes(uint32_t k, uint32_t d) {
  (void)d;
  return (size_t)(acc_commit_waves(k) + 1) * 16 * 2 * TAB_WORDS * 4;
}

hipError_t acc_fold_g1(const uint32_t* C, const uint32_t* C2, uint32_t k, const uint32_t* E, const uint32_t* E2,
                       const uint32_t* Ej, uint32_t d, const uint32_t* gamma, uint32_t* C_out, uint32_t* E_out,
                       void* scratch, hipStream_t s) {
  const uint32_t nwc = acc_commit_waves(k);
  const ProfToken tok = prof_begin("acc.fold_g1", s);
  hipLaunchKernelGGL(acc_fold_g1_kernel, dim3(nwc + 1), dim3(ACC_NT), 0, s, C, C2, k, E, E2, Ej, d, gamma, nwc,
                     C_out, E_out, static_cast<uint32_t*>(scratch));
  prof_end(tok, s);
  return hipGetLastError();
}

size_t g1_rlc_scratch_bytes(uint32_t m, uint32_t k) {
  const size_t nblk = (m + 63) / 64;
  return (size_t)k * nblk * 64 * 2 * TAB_WORDS * 4 + (size_t)k * nblk * 36 * 4;
}

hipError_t g1_rlc(const uint32_t* pts, const uint32_t* sigma, uint32_t m, uint32_t k, uint32_t* out, void* scratch,
                  hipStream_t s) {
  if (m == 0 || k == 0 || m > G1_RLC_TERMS_MAX) return hipErrorInvalidValue;
  const uint32_t nblk = (m + 63) / 64;
  uint32_t* tabs = static_cast<uint32_t*>(scratch);
  uint32_t* partial = tabs + (size_t)k * nblk * 64 * 2 * TAB_WORDS;
  const ProfToken tok = prof_begin("fold.terms", s);
  hipLaunchKernelGGL(g1_rlc_terms_kernel, dim3(nblk, k), dim3(RLC_TERMS_NT), 0, s, pts, sigma, m, k, tabs, partial,
                     nblk == 1 ? out : nullptr);
  if (nblk > 1) hipLaunchKernelGGL(g1_rlc_finish_kernel, dim3(k), dim3(64), 0, s, partial, nblk, out);
  prof_end(tok, s);
  return hipGetLastError();
}

hipError_t fr_rlc(const uint32_t* v0, const uint32_t* vmid, const uint32_t* vlast, uint32_t d, uint64_t len,
                  const uint32_t* gamma, uint32_t* out, hipStream_t s) {
  if (len == 0) return hipSuccess;
  const ProfToken tok = prof_begin("acc.fr_rlc", s);
  hipLaunchKernelGGL(fr_rlc_kernel, dim3((uint32_t)((len + RLC_NT - 1) / RLC_NT)), dim3(RLC_NT), 0, s, v0, vmid,
                     vlast, d, len, gamma, out);
  prof_end(tok, s);
  return hipGetLastError();
}

hipError_t transcript_challenge(const uint8_t* data, uint64_t bytes, const f29& c_2_256, uint32_t* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(transcript_kernel, dim3(1), dim3(64), 0, s, data, bytes, c_2_256, out);
  return hipGetLastError();
}

}  // namespace zk
