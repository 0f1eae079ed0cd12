// BN254 G2 arithmetic: Fq2 = Fq[u] / (u^2 + 1) and XYZZ points on the twist
// y^2 = x^3 + 3 / (9 + u) (the curve constant is not needed by the formulas).
//
// Every Fq2 operation returns both components reduced below 2q with
// normalised limbs, so inputs of every Montgomery product stay below 4q (sums
// of two reduced values), comfortably inside the product's 16q input bound;
// a product of two values below 4q is below 1.1q.  Each operation then needs
// only the conditional subtractions its own output bound calls for (stated
// at each one).  Coordinates are in Montgomery form.
// The point formulas are the XYZZ ones of curve.h with Fq2 coefficients.
#pragma once
#include "curve.h"

namespace zk {

struct fp2 {
  f29 c0, c1;
};

struct g2xyzz {
  fp2 X, Y, ZZ, ZZZ;
};

struct g2aff {
  fp2 x, y;
};

// The generator H of G2 (plain canonical words: x0, x1, y0, y1).
__constant__ static const uint32_t G2_GEN[32] = {
    0xd992f6edu, 0x46debd5cu, 0xf75edaddu, 0x674322d4u, 0x5e5c4479u, 0x426a0066u, 0x121f1e76u, 0x1800deefu,
    0xaef312c2u, 0x97e485b7u, 0x35a9e712u, 0xf1aa4933u, 0x31fb5d25u, 0x7260bfb7u, 0x920d483au, 0x198e9393u,
    0x66fa7daau, 0x4ce6cc01u, 0x0c43d37bu, 0xe3d1e769u, 0x8dcb408fu, 0x4aab7180u, 0xdb8c6debu, 0x12c85ea5u,
    0xd122975bu, 0x55acdadcu, 0x70b38ef3u, 0xbc4b3133u, 0x690c3395u, 0xec9e99adu, 0x585ff075u, 0x090689d0u};

// The twist's constant 3 / (9 + u) (plain canonical words: c0, c1).
static constexpr uint32_t G2_TWIST_B[16] = {
    0x24a138e5u, 0x3267e6dcu, 0x59dbefa3u, 0xb5b4c5e5u, 0x1be06ac3u, 0x81be1899u, 0xceb8aaaeu, 0x2b149d40u,
    0x85c315d2u, 0xe4a2bd06u, 0xe52d1852u, 0xa74fa084u, 0xeed8fdf4u, 0xcd2cafadu, 0x3af0fed4u, 0x009713b0u};

// normalised value < 4q -> < 2q
ZK_HD f29 red_lt4(const f29& a) { return cond_sub(a, Fq::C2); }

// normalised value < 8q -> < 2q
ZK_HD f29 red_lt8(const f29& a) { return cond_sub(cond_sub(a, Fq::C4), Fq::C2); }

ZK_HD fp2 fp2_zero() { return fp2{f29_zero(), f29_zero()}; }

ZK_HD bool fp2_is_zero_limbs(const fp2& a) { return f29_is_zero_limbs(a.c0) && f29_is_zero_limbs(a.c1); }

ZK_HD bool fp2_is_zero_mod(const fp2& a) { return is_zero_mod<Fq>(a.c0) && is_zero_mod<Fq>(a.c1); }

// a + b < 4q
ZK_HD fp2 fp2_add(const fp2& a, const fp2& b) { return fp2{red_lt4(add_n(a.c0, b.c0)), red_lt4(add_n(a.c1, b.c1))}; }

// a - b + 2q < 4q
ZK_HD fp2 fp2_sub(const fp2& a, const fp2& b) {
  return fp2{red_lt4(sub_k(a.c0, b.c0, Fq::K2)), red_lt4(sub_k(a.c1, b.c1, Fq::K2))};
}

ZK_HD fp2 fp2_neg(const fp2& a) { return fp2_sub(fp2_zero(), a); }

// (a0 + a1 u)(b0 + b1 u) = (a0 b0 - a1 b1) + (a0 b1 + a1 b0) u, each
// component one Montgomery reduction of two products' column sums
// (mont_mul2; -a1 b1 as (2q - a1) b1).  For components below 2q both sums
// are below 8q^2, so each component is below 8q^2 / 2^261 + q < 1.05q (no
// correction), and a column holds at most 18 limb products below 2^58.  The
// four products cost the same word mads as Karatsuba's three, with two
// reductions instead of three and none of its sums and corrections.
ZK_HD fp2 fp2_mul(const fp2& a, const fp2& b) {
  return fp2{mont_mul2<Fq>(a.c0, b.c0, sub_k(f29_zero(), a.c1, Fq::K2), b.c1),
             mont_mul2<Fq>(a.c0, b.c1, a.c1, b.c0)};
}

// a b - c d, each component one Montgomery reduction of four limb products'
// column sums (the subtracted terms as (2q - x) operands):
//   re: a0 b0 + (2q - a1) b1 + (2q - c0) d0 + c1 d1
//   im: a0 b1 + a1 b0 + (2q - c0) d1 + (2q - c1) d0.
// For components below 2q a column holds at most 36 limb products below
// 2^58 (below 2^63.2, and below 2^64 with the reduction's terms), and each
// sum is below 16 q^2, so a component is below 16 q^2 / 2^261 + q < 1.1q.
ZK_HD fp2 fp2_mul_sub(const fp2& a, const fp2& b, const fp2& c, const fp2& d) {
  const f29 na1 = sub_k(f29_zero(), a.c1, Fq::K2);
  const f29 nc0 = sub_k(f29_zero(), c.c0, Fq::K2);
  const f29 nc1 = sub_k(f29_zero(), c.c1, Fq::K2);
  uint64_t re[18], im[18];
#pragma unroll
  for (int k = 0; k < 18; k++) re[k] = im[k] = 0;
  mul_cols(re, a.c0, b.c0);
  mul_cols(re, na1, b.c1);
  mul_cols(re, nc0, d.c0);
  mul_cols(re, c.c1, d.c1);
  const f29 r0 = mont_reduce<Fq>(re);
  mul_cols(im, a.c0, b.c1);
  mul_cols(im, a.c1, b.c0);
  mul_cols(im, nc0, d.c1);
  mul_cols(im, nc1, d.c0);
  return fp2{r0, mont_reduce<Fq>(im)};
}

// (a0 + a1 u)^2 = (a0 + a1)(a0 - a1) + 2 a0 a1 u
// both factors of s below 4q, so s < 1.1q; 2 t < 2.1q.
ZK_HD fp2 fp2_sqr(const fp2& a) {
  const f29 s = mont_mul<Fq>(add_n(a.c0, a.c1), sub_k(a.c0, a.c1, Fq::K2));
  const f29 t = mont_mul<Fq>(a.c0, a.c1);
  return fp2{s, red_lt4(add_n(t, t))};
}

ZK_HD fp2 fp2_from_mont_one() { return fp2{f29_from(Fq::ONE), f29_zero()}; }

// 1 / a = conj(a) / (a0^2 + a1^2), a nonzero; Montgomery form in and out.
ZK_HD fp2 fp2_inv(const fp2& a) {
  const f29 nrm = reduce_full<Fq>(add_n(mont_mul<Fq>(a.c0, a.c0), mont_mul<Fq>(a.c1, a.c1)));
  const f29 ni = mont_inv<Fq>(nrm);
  const fp2 conj{a.c0, red_lt4(sub_k(f29_zero(), a.c1, Fq::K2))};
  return fp2{red_lt4(mont_mul<Fq>(conj.c0, ni)), red_lt4(mont_mul<Fq>(conj.c1, ni))};
}

ZK_HD bool g2_is_inf(const g2xyzz& a) { return fp2_is_zero_limbs(a.ZZ); }

ZK_HD g2xyzz g2_inf() { return g2xyzz{fp2_zero(), fp2_zero(), fp2_zero(), fp2_zero()}; }

ZK_HD g2xyzz g2_from_aff(const g2aff& p) { return g2xyzz{p.x, p.y, fp2_from_mont_one(), fp2_from_mont_one()}; }

ZK_HD g2aff g2_aff_neg(const g2aff& p) { return g2aff{p.x, fp2_neg(p.y)}; }

ZK_HD g2xyzz g2_dbl(const g2xyzz& a) {
  if (g2_is_inf(a)) return a;
  const fp2 U = fp2_add(a.Y, a.Y);
  const fp2 V = fp2_sqr(U);
  const fp2 W = fp2_mul(U, V);
  const fp2 S = fp2_mul(a.X, V);
  const fp2 x2 = fp2_sqr(a.X);
  const fp2 M = fp2_add(fp2_add(x2, x2), x2);
  g2xyzz r;
  r.X = fp2_sub(fp2_sqr(M), fp2_add(S, S));
  r.Y = fp2_sub(fp2_mul(M, fp2_sub(S, r.X)), fp2_mul(W, a.Y));
  r.ZZ = fp2_mul(V, a.ZZ);
  r.ZZZ = fp2_mul(W, a.ZZZ);
  return r;
}

ZK_HD g2xyzz g2_add(const g2xyzz& a, const g2xyzz& b) {
  if (g2_is_inf(a)) return b;
  if (g2_is_inf(b)) return a;
  const fp2 U1 = fp2_mul(a.X, b.ZZ);
  const fp2 U2 = fp2_mul(b.X, a.ZZ);
  const fp2 S1 = fp2_mul(a.Y, b.ZZZ);
  const fp2 S2 = fp2_mul(b.Y, a.ZZZ);
  const fp2 P = fp2_sub(U2, U1);
  const fp2 R = fp2_sub(S2, S1);
  if (fp2_is_zero_mod(P)) {
    if (fp2_is_zero_mod(R)) return g2_dbl(a);
    return g2_inf();
  }
  const fp2 PP = fp2_sqr(P);
  const fp2 PPP = fp2_mul(P, PP);
  const fp2 Q = fp2_mul(U1, PP);
  g2xyzz r;
  r.X = fp2_sub(fp2_sqr(R), fp2_add(fp2_add(PPP, Q), Q));
  r.Y = fp2_sub(fp2_mul(R, fp2_sub(Q, r.X)), fp2_mul(S1, PPP));
  r.ZZ = fp2_mul(fp2_mul(a.ZZ, b.ZZ), PP);
  r.ZZZ = fp2_mul(fp2_mul(a.ZZZ, b.ZZZ), PPP);
  return r;
}

// a + p, p affine (not infinity)
ZK_HD g2xyzz g2_madd(const g2xyzz& a, const g2aff& p) {
  if (g2_is_inf(a)) return g2_from_aff(p);
  const fp2 U2 = fp2_mul(p.x, a.ZZ);
  const fp2 S2 = fp2_mul(p.y, a.ZZZ);
  const fp2 P = fp2_sub(U2, a.X);
  const fp2 R = fp2_sub(S2, a.Y);
  if (fp2_is_zero_mod(P)) {
    if (fp2_is_zero_mod(R)) return g2_dbl(g2_from_aff(p));
    return g2_inf();
  }
  const fp2 PP = fp2_sqr(P);
  const fp2 PPP = fp2_mul(P, PP);
  const fp2 Q = fp2_mul(a.X, PP);
  g2xyzz r;
  r.X = fp2_sub(fp2_sqr(R), fp2_add(fp2_add(PPP, Q), Q));
  r.Y = fp2_mul_sub(R, fp2_sub(Q, r.X), a.Y, PPP);
  r.ZZ = fp2_mul(a.ZZ, PP);
  r.ZZZ = fp2_mul(a.ZZZ, PPP);
  return r;
}

// Canonical plain words of one Fq value (Montgomery form in).
ZK_HD void fq_words(const f29& a, uint32_t w[8]) { pack(from_mont<Fq>(a), w); }

// Affine Montgomery form of a; false for infinity.
ZK_HD bool g2_to_aff(const g2xyzz& a, g2aff& o) {
  if (g2_is_inf(a)) return false;
  const fp2 I = fp2_inv(fp2_mul(a.ZZ, a.ZZZ));   // 1 / Z^5
  o.x = fp2_mul(a.X, fp2_mul(I, a.ZZZ));          // X / Z^2
  o.y = fp2_mul(a.Y, fp2_mul(I, a.ZZ));           // Y / Z^3
  o.x = fp2{reduce_full<Fq>(o.x.c0), reduce_full<Fq>(o.x.c1)};
  o.y = fp2{reduce_full<Fq>(o.y.c0), reduce_full<Fq>(o.y.c1)};
  return true;
}

// Canonical plain words x0, x1, y0, y1; infinity -> zeros.
ZK_HD void g2_to_words(const g2xyzz& a, uint32_t out[32]) {
  g2aff o;
  if (!g2_to_aff(a, o)) {
    for (int i = 0; i < 32; i++) out[i] = 0;
    return;
  }
  fq_words(o.x.c0, out);
  fq_words(o.x.c1, out + 8);
  fq_words(o.y.c0, out + 16);
  fq_words(o.y.c1, out + 24);
}

// Canonical plain words -> Montgomery affine; false for (0, 0, 0, 0).
ZK_HD bool g2_from_words(const uint32_t w[32], g2aff& p) {
  uint32_t o = 0;
  for (int i = 0; i < 32; i++) o |= w[i];
  p.x.c0 = reduce_full<Fq>(to_mont<Fq>(unpack(w)));
  p.x.c1 = reduce_full<Fq>(to_mont<Fq>(unpack(w + 8)));
  p.y.c0 = reduce_full<Fq>(to_mont<Fq>(unpack(w + 16)));
  p.y.c1 = reduce_full<Fq>(to_mont<Fq>(unpack(w + 24)));
  return o != 0;
}

ZK_HD bool words_below(const uint32_t* w, const uint32_t (&m)[8]) {
  unsigned br = 0;
  for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], m[i], br, &br);
  return br != 0;
}

ZK_HD bool fp2_equal(const fp2& a, const fp2& b) {
  const f29 a0 = reduce_full<Fq>(a.c0), a1 = reduce_full<Fq>(a.c1);
  const f29 b0 = reduce_full<Fq>(b.c0), b1 = reduce_full<Fq>(b.c1);
  uint32_t d = 0;
  for (int k = 0; k < 9; k++) d |= (a0.l[k] ^ b0.l[k]) | (a1.l[k] ^ b1.l[k]);
  return d == 0;
}

// Is w (x0 x1 y0 y1, plain words) all zeros or a canonical point of order r
// on the twist?  G2 has cofactor > 1, so on top of the curve equation the
// point must satisfy r P = O (double-and-add over the bits of r).
ZK_HD bool g2_words_valid(const uint32_t w[32]) {
  uint32_t o = 0;
  for (int k = 0; k < 32; k++) o |= w[k];
  if (o == 0) return true;
  for (int c = 0; c < 4; c++)
    if (!words_below(w + 8 * c, Fq::M32)) return false;
  g2aff p;
  g2_from_words(w, p);
  const fp2 b{reduce_full<Fq>(to_mont<Fq>(unpack(G2_TWIST_B))), reduce_full<Fq>(to_mont<Fq>(unpack(G2_TWIST_B + 8)))};
  if (!fp2_equal(fp2_sqr(p.y), fp2_add(fp2_mul(fp2_sqr(p.x), p.x), b))) return false;
  g2xyzz acc = g2_inf();
  for (int bit = 253; bit >= 0; --bit) {
    acc = g2_dbl(acc);
    if ((FrP::M32[bit >> 5] >> (bit & 31)) & 1u) acc = g2_madd(acc, p);
  }
  return g2_is_inf(acc);
}

}  // namespace zk
