// BN254 prime-field arithmetic for gfx950 (and host builds of the same code).
//
// Working form: nine 29-bit limbs, value = sum l[i] * 2^(29 i).  Products use
// Montgomery reduction with R = 2^261: every limb product is one
// v_mad_u64_u32 accumulating into a 64-bit column sum, and the 29-bit radix
// leaves enough headroom that the column sums never overflow, so a full
// Montgomery product needs no carry propagation until the end (162 mads plus
// about 64 other VALU instructions).
//
// Reduction is lazy.  A Montgomery product of a and b is only guaranteed to be
// < a*b/2^261 + q; a subtraction a - b is computed as a + c*q - b with c*q
// written in limbs raised by 2^31 ("borrowed"), then carry-normalised.  The
// multiples c used by each point formula come from an interval analysis
// (bounds.py) showing every intermediate value stays bounded and no limb or
// column accumulator overflows.
//
// Storage form: the 256-bit little-endian value in eight 32-bit words
// (values < 2^256 only).  Coordinates in memory are kept in Montgomery form
// x * 2^261 mod p, canonical (< p); scalars and NTT data are plain canonical
// integers (the NTT multiplies plain values by Montgomery-form twiddles,
// which yields plain products).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field_constants.h"

#define ZK_HD __host__ __device__ __forceinline__

namespace zk {

constexpr uint32_t MASK29 = 0x1fffffffu;

struct f29 {
  uint32_t l[9];
};

template <int N>
ZK_HD f29 f29_from(const uint32_t (&c)[N]) {
  static_assert(N == 9, "29-bit constant tables have nine limbs");
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = c[i];
  return r;
}

ZK_HD f29 f29_zero() {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = 0;
  return r;
}

ZK_HD bool f29_is_zero_limbs(const f29& a) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) o |= a.l[i];
  return o == 0;
}

// 8 x 32-bit words -> nine 29-bit limbs.
ZK_HD f29 unpack(const uint32_t w[8]) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    const int bit = 29 * i, j = bit >> 5, s = bit & 31;
    uint64_t two = (uint64_t)w[j];
    if (j + 1 < 8) two |= (uint64_t)w[j + 1] << 32;
    r.l[i] = (uint32_t)(two >> s) & MASK29;
  }
  return r;
}

// Nine normalised limbs (each < 2^29) of a value < 2^256 -> 8 words.
ZK_HD void pack(const f29& a, uint32_t w[8]) {
#pragma unroll
  for (int j = 0; j < 8; j++) w[j] = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    const int bit = 29 * i, j = bit >> 5, s = bit & 31;
    w[j] |= a.l[i] << s;
    if (s > 3 && j + 1 < 8) w[j + 1] |= a.l[i] >> (32 - s);
  }
}

// Carry-propagate so limbs 0..7 are < 2^29 (value unchanged).
ZK_HD f29 normalize(f29 a) {
#pragma unroll
  for (int i = 0; i < 8; i++) {
    a.l[i + 1] += a.l[i] >> 29;
    a.l[i] &= MASK29;
  }
  return a;
}

// Limb-wise sum, not normalised.
ZK_HD f29 add(const f29& a, const f29& b) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = a.l[i] + b.l[i];
  return r;
}

ZK_HD f29 add_n(const f29& a, const f29& b) { return normalize(add(a, b)); }

// a - b + K where K is a multiple of q in borrowed limbs; normalised.
template <int N>
ZK_HD f29 sub_k(const f29& a, const f29& b, const uint32_t (&k)[N]) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = a.l[i] + k[i] - b.l[i];
  return normalize(r);
}

// Montgomery product a * b * 2^-261 mod q (lazily reduced, normalised limbs).
template <class F>
ZK_HD f29 mont_mul(const f29& a, const f29& b) {
  uint64_t acc[18];
#pragma unroll
  for (int k = 0; k < 18; k++) acc[k] = 0;
#pragma unroll
  for (int i = 0; i < 9; i++)
#pragma unroll
    for (int j = 0; j < 9; j++) acc[i + j] += (uint64_t)a.l[i] * b.l[j];
#pragma unroll
  for (int k = 0; k < 9; k++) {
    const uint32_t m = ((uint32_t)acc[k] * F::INV) & MASK29;
#pragma unroll
    for (int j = 0; j < 9; j++) acc[k + j] += (uint64_t)m * F::M[j];
    acc[k + 1] += acc[k] >> 29;
  }
  f29 r;
#pragma unroll
  for (int k = 9; k < 17; k++) {
    r.l[k - 9] = (uint32_t)acc[k] & MASK29;
    acc[k + 1] += acc[k] >> 29;
  }
  r.l[8] = (uint32_t)acc[17];
  return r;
}

// Squaring: cross products once, doubled, plus the diagonal.
template <class F>
ZK_HD f29 mont_sqr(const f29& a) {
  uint64_t acc[18];
#pragma unroll
  for (int k = 0; k < 18; k++) acc[k] = 0;
#pragma unroll
  for (int i = 0; i < 9; i++)
#pragma unroll
    for (int j = i + 1; j < 9; j++) acc[i + j] += (uint64_t)a.l[i] * a.l[j];
#pragma unroll
  for (int k = 0; k < 18; k++) acc[k] <<= 1;
#pragma unroll
  for (int i = 0; i < 9; i++) acc[2 * i] += (uint64_t)a.l[i] * a.l[i];
#pragma unroll
  for (int k = 0; k < 9; k++) {
    const uint32_t m = ((uint32_t)acc[k] * F::INV) & MASK29;
#pragma unroll
    for (int j = 0; j < 9; j++) acc[k + j] += (uint64_t)m * F::M[j];
    acc[k + 1] += acc[k] >> 29;
  }
  f29 r;
#pragma unroll
  for (int k = 9; k < 17; k++) {
    r.l[k - 9] = (uint32_t)acc[k] & MASK29;
    acc[k + 1] += acc[k] >> 29;
  }
  r.l[8] = (uint32_t)acc[17];
  return r;
}

// If a >= c*q (normalised limbs, c*q given normalised) return a - c*q else a.
template <int N>
ZK_HD f29 cond_sub(const f29& a, const uint32_t (&cq)[N]) {
  int32_t d[9];
#pragma unroll
  for (int i = 0; i < 9; i++) d[i] = (int32_t)a.l[i] - (int32_t)cq[i];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    d[i + 1] += d[i] >> 29;  // arithmetic shift: floor division by 2^29
    d[i] &= (int32_t)MASK29;
  }
  const bool keep = d[8] < 0;
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = keep ? a.l[i] : (uint32_t)d[i];
  return r;
}

// Normalised a with value < 32 q  ->  canonical value in [0, q).
template <class F>
ZK_HD f29 reduce_full(f29 a) {
  a = normalize(a);
  a = cond_sub(a, F::C16);
  a = cond_sub(a, F::C8);
  a = cond_sub(a, F::C4);
  a = cond_sub(a, F::C2);
  a = cond_sub(a, F::C1);
  return a;
}

// Is the normalised value a (< 32 q) a multiple of q?  A multiple k*q with
// k < 32 has k = a mod 2^29 * q^-1 mod 2^29, so one multiply rejects almost
// every nonzero input; the rare candidate is compared exactly.
template <class F>
ZK_HD bool is_zero_mod(const f29& a) {
  const uint32_t qinv = (0u - F::INV) & MASK29;  // q^-1 mod 2^29
  const uint32_t k = (a.l[0] * qinv) & MASK29;
  if (k >= 32u) return false;
  uint64_t c = 0;
  uint32_t diff = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    c += (uint64_t)k * F::M[i];
    diff |= ((uint32_t)c & (i < 8 ? MASK29 : 0xffffffffu)) ^ a.l[i];
    c >>= 29;
  }
  return diff == 0;
}

template <class F>
ZK_HD f29 to_mont(const f29& a) {
  return mont_mul<F>(a, f29_from(F::R2));
}

// Montgomery form -> canonical plain value.
template <class F>
ZK_HD f29 from_mont(const f29& a) {
  f29 one = f29_zero();
  one.l[0] = 1;
  return reduce_full<F>(mont_mul<F>(a, one));
}

// a^e for a 256-bit exponent given as 8 little-endian words (Montgomery form in and out).
template <class F>
ZK_HD f29 mont_pow(const f29& a, const uint32_t e[8]) {
  f29 r = f29_from(F::ONE);
  bool started = false;
  for (int i = 255; i >= 0; --i) {
    if (started) r = mont_sqr<F>(r);
    if ((e[i >> 5] >> (i & 31)) & 1u) {
      r = started ? mont_mul<F>(r, a) : a;
      started = true;
    }
  }
  return r;
}

// Inverse by Fermat: a^(q-2); a must be nonzero mod q.
template <class F>
ZK_HD f29 mont_inv_fermat(const f29& a) {
  uint32_t e[8];
#pragma unroll
  for (int i = 0; i < 8; i++) e[i] = F::M32[i];
  e[0] -= 2u;  // q is odd and its low word exceeds 2
  return mont_pow<F>(a, e);
}

// ---- 32-bit-word canonical arithmetic (values in [0, q)) -------------------



// r = a + b mod q for canonical a, b (2q < 2^256, so the sum never carries out).
template <class F>
ZK_HD void add_mod32(const uint32_t a[8], const uint32_t b[8], uint32_t r[8]) {
  uint32_t s[8], d[8];
  unsigned c = 0, br = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) s[i] = __builtin_addc(a[i], b[i], c, &c);
#pragma unroll
  for (int i = 0; i < 8; i++) d[i] = __builtin_subc(s[i], F::M32[i], br, &br);
#pragma unroll
  for (int i = 0; i < 8; i++) r[i] = br ? s[i] : d[i];
}

// r = a - b mod q for canonical a, b.
template <class F>
ZK_HD void sub_mod32(const uint32_t a[8], const uint32_t b[8], uint32_t r[8]) {
  uint32_t d[8];
  unsigned br = 0, c = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) d[i] = __builtin_subc(a[i], b[i], br, &br);
  const uint32_t mask = 0u - br;
#pragma unroll
  for (int i = 0; i < 8; i++) r[i] = __builtin_addc(d[i], F::M32[i] & mask, c, &c);
}

// a in [0, 2q) -> a mod q.
template <class F>
ZK_HD void canon32(uint32_t a[8]) {
  uint32_t d[8];
  unsigned br = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) d[i] = __builtin_subc(a[i], F::M32[i], br, &br);
#pragma unroll
  for (int i = 0; i < 8; i++) a[i] = br ? a[i] : d[i];
}

// Plain canonical a (words) times a Montgomery-form constant w: the plain
// product a*w_plain mod q, canonical words.  (mont_mul(a, w*2^261) = a*w.)
template <class F>
ZK_HD void mul_plain_by_mont(const uint32_t a[8], const f29& w, uint32_t r[8]) {
  pack(mont_mul<F>(unpack(a), w), r);  // < q*q/2^261 + q < 2q
  canon32<F>(r);
}

// ---- inversion -------------------------------------------------------------

ZK_HD bool w8_is_one(const uint32_t a[8]) {
  uint32_t o = a[0] ^ 1u;
#pragma unroll
  for (int i = 1; i < 8; i++) o |= a[i];
  return o == 0;
}

// a >>= 1 over 8 words (with `top` shifted into bit 255).
ZK_HD void w8_shr1(uint32_t a[8], uint32_t top) {
#pragma unroll
  for (int i = 0; i < 7; i++) a[i] = (a[i] >> 1) | (a[i + 1] << 31);
  a[7] = (a[7] >> 1) | (top << 31);
}

// x / 2 mod q for canonical x (q odd): x even -> x >> 1, else (x + q) >> 1.
template <class F>
ZK_HD void half_mod32(uint32_t x[8]) {
  const uint32_t mask = 0u - (x[0] & 1u);
  unsigned c = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) x[i] = __builtin_addc(x[i], F::M32[i] & mask, c, &c);
  w8_shr1(x, c);
}

// Plain inverse x^-1 mod q of a canonical nonzero x by the binary extended
// Euclidean algorithm (invariants: x1 * x = u, x2 * x = v mod q).
template <class F>
ZK_HD void inv_binary32(const uint32_t x[8], uint32_t out[8]) {
  uint32_t u[8], v[8], x1[8], x2[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    u[i] = x[i];
    v[i] = F::M32[i];
    x1[i] = 0;
    x2[i] = 0;
  }
  x1[0] = 1;
  while (!w8_is_one(u) && !w8_is_one(v)) {
    while ((u[0] & 1u) == 0) {
      w8_shr1(u, 0);
      half_mod32<F>(x1);
    }
    while ((v[0] & 1u) == 0) {
      w8_shr1(v, 0);
      half_mod32<F>(x2);
    }
    uint32_t d[8];
    unsigned br = 0;
#pragma unroll
    for (int i = 0; i < 8; i++) d[i] = __builtin_subc(u[i], v[i], br, &br);
    if (!br) {  // u >= v
#pragma unroll
      for (int i = 0; i < 8; i++) u[i] = d[i];
      sub_mod32<F>(x1, x2, x1);
    } else {
      unsigned b2 = 0;
#pragma unroll
      for (int i = 0; i < 8; i++) v[i] = __builtin_subc(v[i], u[i], b2, &b2);
      sub_mod32<F>(x2, x1, x2);
    }
  }
  const bool uone = w8_is_one(u);
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = uone ? x1[i] : x2[i];
}

// Inverse in Montgomery form: (a R)^-1 by the binary algorithm, times R^3
// through one Montgomery product gives a^-1 R.  a must be nonzero mod q.
template <class F>
ZK_HD f29 mont_inv(const f29& a) {
  uint32_t w[8], iw[8];
  pack(reduce_full<F>(a), w);
  inv_binary32<F>(w, iw);
  return mont_mul<F>(unpack(iw), f29_from(F::R3));
}

}  // namespace zk
