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

// a - b + K limb-wise without carry normalisation, for K a multiple of q in
// limbs raised by 2^30 (the H tables): for normalised a, b every limb stays
// below 2^31, small enough for one operand of a product whose other
// operand is normalised (bounds.py checks each use).
template <int N>
ZK_HD f29 sub_raw(const f29& a, const f29& b, const uint32_t (&k)[N]) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = a.l[i] + k[i] - b.l[i];
  return r;
}

// Column sums of a * b: acc[i + j] += a_i b_j (one v_mad_u64_u32 each).
ZK_HD void mul_cols(uint64_t (&acc)[18], const f29& a, const f29& b) {
#pragma unroll
  for (int i = 0; i < 9; i++)
#pragma unroll
    for (int j = 0; j < 9; j++) acc[i + j] += (uint64_t)a.l[i] * b.l[j];
}

// Montgomery reduction of 18 column sums: value * 2^-261 mod q (lazily
// reduced, normalised limbs).
template <class F>
ZK_HD f29 mont_reduce(uint64_t (&acc)[18]) {
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

// Montgomery product a * b * 2^-261 mod q (lazily reduced, normalised limbs).
template <class F>
ZK_HD f29 mont_mul(const f29& a, const f29& b) {
  uint64_t acc[18];
#pragma unroll
  for (int k = 0; k < 18; k++) acc[k] = 0;
  mul_cols(acc, a, b);
  return mont_reduce<F>(acc);
}

// (a * b + c * d) * 2^-261 mod q with one reduction: the two products'
// column sums share the accumulators (18 terms per column, still far below
// 2^64 for normalised limbs), which saves a whole reduction where a formula
// subtracts one product from another (pass the subtrahend's negation, a
// multiple of q minus it, as c).
template <class F>
ZK_HD f29 mont_mul2(const f29& a, const f29& b, const f29& c, const f29& d) {
  uint64_t acc[18];
#pragma unroll
  for (int k = 0; k < 18; k++) acc[k] = 0;
  mul_cols(acc, a, b);
  mul_cols(acc, c, d);
  return mont_reduce<F>(acc);
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
  return mont_reduce<F>(acc);
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

// ---- inversion by the binary GCD with word-sized approximations ----------
// The binary GCD keeps (a, b) with b odd; a step subtracts the smaller from
// the larger when a is odd (swapping so that a - b >= 0) and halves a, while
// coefficients u, v with a = u x, b = v x (mod q) follow along; it ends with
// a = 0, b = gcd = 1, v = x^-1.  Thirty steps depend only on the low 30 bits
// of a and b (their parities) and on comparisons, which the top bits decide
// almost always.  So thirty steps run on 64-bit stand-ins (top 34 and low
// 30 bits), recording a 2x2 integer matrix [f0 g0; f1 g1] (rows scaled so
// that halving a becomes doubling the other row); one exact update
// (a, b) <- ((f0 a + g0 b), (f1 a + g1 b)) / 2^30 then applies them to the
// full values (and to u, v modulo q).  A misjudged comparison can make a new
// value negative; it is negated together with its matrix row.  This is the
// batched binary GCD of T. Pornin, "Optimized Binary GCD for Modular
// Inversion" (IACR ePrint 2020/972); the loop runs until a = 0, and a
// Fermat inversion backs it up should the iteration bound ever be reached.
constexpr int BGCD_STEPS = 30;
static_assert(BGCD_STEPS <= 30, "a round's matrix entries must fit in 32-bit words");

ZK_HD bool w8_is_zero(const uint32_t a[8]) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) o |= a[i];
  return o == 0;
}

// Bit length of a (0 for a = 0).
ZK_HD uint32_t w8_bitlen(const uint32_t a[8]) {
  uint32_t n = 0;
#pragma unroll
  for (int i = 0; i < 8; i++)
    if (a[i]) n = 32u * i + 32u - (uint32_t)__builtin_clz(a[i]);
  return n;
}

// floor(a / 2^p) mod 2^64 for 0 <= p < 256.
ZK_HD uint64_t w8_bits_at(const uint32_t a[8], uint32_t p) {
  const uint32_t k = p >> 5, sh = p & 31u;
  uint32_t w0 = 0, w1 = 0, w2 = 0;
#pragma unroll
  for (uint32_t i = 0; i < 8; i++) {
    if (i == k) w0 = a[i];
    if (i == k + 1) w1 = a[i];
    if (i == k + 2) w2 = a[i];
  }
  const uint64_t lo = (uint64_t)w0 | ((uint64_t)w1 << 32);
  return sh ? (lo >> sh) | ((uint64_t)w2 << (64u - sh)) : lo;
}

// r = a * m (8 words times a 32-bit word) into 9 words.
ZK_HD void w8_mul_u32(const uint32_t a[8], uint32_t m, uint32_t r[9]) {
  uint64_t c = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    c += (uint64_t)a[i] * m;
    r[i] = (uint32_t)c;
    c >>= 32;
  }
  r[8] = (uint32_t)c;
}

// Two's complement negation of a 9-word value when neg is set.
ZK_HD void w9_cneg(uint32_t r[9], bool neg) {
  const uint32_t mask = neg ? 0xffffffffu : 0u;
  unsigned c = neg ? 1u : 0u;
#pragma unroll
  for (int i = 0; i < 9; i++) r[i] = __builtin_addc(r[i] ^ mask, 0u, c, &c);
}

// (f a + g b) / 2^30 for |f| + |g| <= 2^30 and a, b < 2^254 (the division is
// exact by construction).  Returns the magnitude in out and whether the
// result is negative.
ZK_HD bool bgcd_update(const uint32_t a[8], const uint32_t b[8], int64_t f, int64_t g, uint32_t out[8]) {
  uint32_t pa[9], pb[9], s[9];
  w8_mul_u32(a, (uint32_t)(f < 0 ? -f : f), pa);
  w8_mul_u32(b, (uint32_t)(g < 0 ? -g : g), pb);
  w9_cneg(pa, f < 0);
  w9_cneg(pb, g < 0);
  unsigned c = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) s[i] = __builtin_addc(pa[i], pb[i], c, &c);
  const bool neg = (s[8] >> 31) != 0;
  w9_cneg(s, neg);
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = (s[i] >> BGCD_STEPS) | (s[i + 1] << (32 - BGCD_STEPS));
  return neg;
}

// (f u + g v) / 2^30 mod q for canonical u, v and |f| + |g| <= 2^30: negative
// coefficients use q - u (= -u), and the division is a Montgomery step with
// 2^30 (add the multiple of q that clears the low 30 bits).
template <class F>
ZK_HD void bgcd_update_mod(const uint32_t u[8], const uint32_t v[8], int64_t f, int64_t g, uint32_t out[8]) {
  uint32_t us[8], vs[8], pu[9], pv[9], t[10];
  unsigned bu = 0, bv = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) {
    const uint32_t du = __builtin_subc(F::M32[i], u[i], bu, &bu);
    const uint32_t dv = __builtin_subc(F::M32[i], v[i], bv, &bv);
    us[i] = f < 0 ? du : u[i];
    vs[i] = g < 0 ? dv : v[i];
  }
  w8_mul_u32(us, (uint32_t)(f < 0 ? -f : f), pu);
  w8_mul_u32(vs, (uint32_t)(g < 0 ? -g : g), pv);
  unsigned c = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) t[i] = __builtin_addc(pu[i], pv[i], c, &c);
  t[9] = c;
  // -q^-1 mod 2^32 by Newton's iteration from the low word (q odd)
  uint32_t qi = F::M32[0];
#pragma unroll
  for (int k = 0; k < 5; k++) qi *= 2u - F::M32[0] * qi;
  const uint32_t m = (t[0] * (0u - qi)) & ((1u << BGCD_STEPS) - 1u);
  uint32_t mq[9];
  w8_mul_u32(F::M32, m, mq);
  c = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) t[i] = __builtin_addc(t[i], mq[i], c, &c);
  t[9] += c;
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = (t[i] >> BGCD_STEPS) | (t[i + 1] << (32 - BGCD_STEPS));
  canon32<F>(out);  // the quotient is < 2q
}

// x^-1 mod q for canonical nonzero x.  Returns false (out unspecified) if the
// iteration bound was reached without finishing.
template <class F>
ZK_HD bool inv_bgcd32(const uint32_t x[8], uint32_t out[8]) {
  uint32_t a[8], b[8], u[8], v[8];
#pragma unroll
  for (int i = 0; i < 8; i++) {
    a[i] = x[i];
    b[i] = F::M32[i];
    u[i] = 0;
    v[i] = 0;
  }
  u[0] = 1;
  // 2 log2(q) single steps suffice for the exact algorithm; allow slack
  for (int it = 0; it < 40 && !w8_is_zero(a); it++) {
    uint32_t ab[8];
#pragma unroll
    for (int i = 0; i < 8; i++) ab[i] = a[i] | b[i];
    const uint32_t n = w8_bitlen(ab);
    uint64_t xa, xb;
    if (n <= 64) {
      xa = (uint64_t)a[0] | ((uint64_t)a[1] << 32);
      xb = (uint64_t)b[0] | ((uint64_t)b[1] << 32);
    } else {
      const uint32_t p = n - (64 - BGCD_STEPS);
      const uint64_t lowmask = (1ull << BGCD_STEPS) - 1ull;
      xa = (w8_bits_at(a, p) << BGCD_STEPS) | (a[0] & lowmask);
      xb = (w8_bits_at(b, p) << BGCD_STEPS) | (b[0] & lowmask);
    }
    // after k steps |f0| + |g0| <= 2^k and |f1| + |g1| <= 2^k, so the
    // matrix stays within 32-bit words for the 30 steps of a round
    int32_t f0 = 1, g0 = 0, f1 = 0, g1 = 1;
#pragma unroll
    for (int k = 0; k < BGCD_STEPS; k++) {
      const bool odd = (xa & 1u) != 0;
      const bool sw = odd && xa < xb;
      const uint64_t ta = sw ? xb : xa, tb = sw ? xa : xb;
      const int32_t tf0 = sw ? f1 : f0, tg0 = sw ? g1 : g0;
      const int32_t tf1 = sw ? f0 : f1, tg1 = sw ? g0 : g1;
      xa = (odd ? ta - tb : ta) >> 1;
      xb = tb;
      f0 = odd ? tf0 - tf1 : tf0;
      g0 = odd ? tg0 - tg1 : tg0;
      f1 = tf1 * 2;
      g1 = tg1 * 2;
    }
    uint32_t na[8], nb[8];
    if (bgcd_update(a, b, f0, g0, na)) {
      f0 = -f0;
      g0 = -g0;
    }
    if (bgcd_update(a, b, f1, g1, nb)) {
      f1 = -f1;
      g1 = -g1;
    }
    uint32_t nu[8], nv[8];
    bgcd_update_mod<F>(u, v, f0, g0, nu);
    bgcd_update_mod<F>(u, v, f1, g1, nv);
#pragma unroll
    for (int i = 0; i < 8; i++) {
      a[i] = na[i];
      b[i] = nb[i];
      u[i] = nu[i];
      v[i] = nv[i];
    }
  }
#pragma unroll
  for (int i = 0; i < 8; i++) out[i] = v[i];
  return w8_is_zero(a) && w8_is_one(b);
}

// Inverse in Montgomery form: (a R)^-1 by the batched binary GCD, times R^3
// through one Montgomery product gives a^-1 R.  a must be nonzero mod q.
template <class F>
ZK_HD f29 mont_inv(const f29& a) {
  uint32_t w[8], iw[8];
  pack(reduce_full<F>(a), w);
  if (!inv_bgcd32<F>(w, iw)) return mont_inv_fermat<F>(a);
  return mont_mul<F>(unpack(iw), f29_from(F::R3));
}

}  // namespace zk
