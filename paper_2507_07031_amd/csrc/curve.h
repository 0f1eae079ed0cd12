// BN254 G1 (y^2 = x^3 + 3 over Fq) in extended Jacobian "XYZZ" coordinates:
// (X, Y, ZZ, ZZZ) represents the affine point (X/ZZ, Y/ZZZ) with ZZ^3 = ZZZ^2.
// The point at infinity is ZZ = 0 (all limbs zero); every formula below
// produces it only through its explicit special cases, so a nonzero ZZ never
// becomes a multiple of p by accident.
//
// Formulas: mixed addition madd-2008-s, addition add-2008-s and doubling
// dbl-2008-s-1 of the Explicit-Formulas Database for XYZZ coordinates
// (a = 0).  The subtraction multiples (K2/K4/K8) are the ones bounds.py
// proves safe.  Both additions form Y3 = R (Q - X3) - S PPP (S = Y1, or
// S1 = Y1 ZZZ2) as one Montgomery reduction of both products' column sums
// (mont_mul2), with -S written as 8q - S and Q - X3 left unnormalised
// (sub_raw with the 2^30-raised 8q).
#pragma once
#include "field.h"

namespace zk {

using Fq = FqP;

struct xyzz {
  f29 X, Y, ZZ, ZZZ;
};

// Affine point, coordinates in Montgomery form, normalised limbs (< p).
struct aff {
  f29 x, y;
};

ZK_HD bool is_inf(const xyzz& a) { return f29_is_zero_limbs(a.ZZ); }

ZK_HD xyzz xyzz_inf() {
  xyzz r;
  r.X = f29_zero();
  r.Y = f29_zero();
  r.ZZ = f29_zero();
  r.ZZZ = f29_zero();
  return r;
}

ZK_HD xyzz from_aff(const aff& p) {
  xyzz r;
  r.X = p.x;
  r.Y = p.y;
  r.ZZ = f29_from(Fq::ONE);
  r.ZZZ = f29_from(Fq::ONE);
  return r;
}

// -P for an affine P with canonical y: y -> p - y (in (0, p] for y < p).
ZK_HD aff aff_neg(const aff& p) {
  aff r;
  r.x = p.x;
  r.y = sub_k(f29_zero(), p.y, Fq::K1);
  return r;
}

// 2P for an affine P (y != 0 always: BN254 G1 has odd prime order).
ZK_HD xyzz mdbl(const aff& p) {
  const f29 U = add(p.y, p.y);
  const f29 V = mont_sqr<Fq>(U);
  const f29 W = mont_mul<Fq>(U, V);
  const f29 S = mont_mul<Fq>(p.x, V);
  const f29 x2 = mont_sqr<Fq>(p.x);
  const f29 M = add_n(add(x2, x2), x2);
  xyzz r;
  r.X = sub_k(mont_sqr<Fq>(M), add(S, S), Fq::K4);
  r.Y = sub_k(mont_mul<Fq>(M, sub_k(S, r.X, Fq::K8)), mont_mul<Fq>(W, p.y), Fq::K2);
  r.ZZ = V;
  r.ZZZ = W;
  return r;
}

ZK_HD xyzz dbl(const xyzz& a) {
  if (is_inf(a)) return a;
  const f29 U = add(a.Y, a.Y);
  const f29 V = mont_sqr<Fq>(U);
  const f29 W = mont_mul<Fq>(U, V);
  const f29 S = mont_mul<Fq>(a.X, V);
  const f29 x2 = mont_sqr<Fq>(a.X);
  const f29 M = add_n(add(x2, x2), x2);
  xyzz r;
  r.X = sub_k(mont_sqr<Fq>(M), add(S, S), Fq::K4);
  r.Y = sub_k(mont_mul<Fq>(M, sub_k(S, r.X, Fq::K8)), mont_mul<Fq>(W, a.Y), Fq::K2);
  r.ZZ = mont_mul<Fq>(V, a.ZZ);
  r.ZZZ = mont_mul<Fq>(W, a.ZZZ);
  return r;
}

// a + p with p affine and not infinity.
ZK_HD xyzz madd(const xyzz& a, const aff& p) {
  if (is_inf(a)) return from_aff(p);
  const f29 U2 = mont_mul<Fq>(p.x, a.ZZ);
  const f29 S2 = mont_mul<Fq>(p.y, a.ZZZ);
  const f29 P = sub_k(U2, a.X, Fq::K8);
  const f29 R = sub_k(S2, a.Y, Fq::K8);
  if (is_zero_mod<Fq>(P)) {
    if (is_zero_mod<Fq>(R)) return mdbl(p);
    return xyzz_inf();
  }
  const f29 PP = mont_sqr<Fq>(P);
  const f29 PPP = mont_mul<Fq>(P, PP);
  const f29 Q = mont_mul<Fq>(a.X, PP);
  xyzz r;
  r.X = sub_k(mont_sqr<Fq>(R), add(add(PPP, Q), Q), Fq::K4);
  // Y3 = R (Q - X3) - Y1 PPP with one reduction: -Y1 as 8q - Y1, and Q - X3
  // left unnormalised (limbs below 2^31)
  r.Y = mont_mul2<Fq>(R, sub_raw(Q, r.X, Fq::H8), sub_k(f29_zero(), a.Y, Fq::K8), PPP);
  r.ZZ = mont_mul<Fq>(a.ZZ, PP);
  r.ZZZ = mont_mul<Fq>(a.ZZZ, PPP);
  return r;
}

// a + (neg ? -p : p) with p affine and not infinity: the sign enters only
// R = +-S2 - Y1 (for -p, R = 8q - (S2 + Y1)), so no negated copy of p is
// formed except on the rare doubling path.
ZK_HD xyzz madd_signed(const xyzz& a, const aff& p, bool neg) {
  if (is_inf(a)) return from_aff(neg ? aff_neg(p) : p);
  const f29 U2 = mont_mul<Fq>(p.x, a.ZZ);
  const f29 S2 = mont_mul<Fq>(p.y, a.ZZZ);
  const f29 P = sub_k(U2, a.X, Fq::K8);
  f29 ra, rb;
  const f29 s2y = add(S2, a.Y);
#pragma unroll
  for (int i = 0; i < 9; i++) {
    ra.l[i] = neg ? 0u : S2.l[i];
    rb.l[i] = neg ? s2y.l[i] : a.Y.l[i];
  }
  const f29 R = sub_k(ra, rb, Fq::K8);
  if (is_zero_mod<Fq>(P)) {
    if (is_zero_mod<Fq>(R)) return mdbl(neg ? aff_neg(p) : p);
    return xyzz_inf();
  }
  const f29 PP = mont_sqr<Fq>(P);
  const f29 PPP = mont_mul<Fq>(P, PP);
  const f29 Q = mont_mul<Fq>(a.X, PP);
  xyzz r;
  r.X = sub_k(mont_sqr<Fq>(R), add(add(PPP, Q), Q), Fq::K4);
  r.Y = mont_mul2<Fq>(R, sub_raw(Q, r.X, Fq::H8), sub_k(f29_zero(), a.Y, Fq::K8), PPP);
  r.ZZ = mont_mul<Fq>(a.ZZ, PP);
  r.ZZZ = mont_mul<Fq>(a.ZZZ, PPP);
  return r;
}

ZK_HD xyzz add(const xyzz& a, const xyzz& b) {
  if (is_inf(a)) return b;
  if (is_inf(b)) return a;
  const f29 U1 = mont_mul<Fq>(a.X, b.ZZ);
  const f29 U2 = mont_mul<Fq>(b.X, a.ZZ);
  const f29 S1 = mont_mul<Fq>(a.Y, b.ZZZ);
  const f29 S2 = mont_mul<Fq>(b.Y, a.ZZZ);
  const f29 P = sub_k(U2, U1, Fq::K8);
  const f29 R = sub_k(S2, S1, Fq::K8);
  if (is_zero_mod<Fq>(P)) {
    if (is_zero_mod<Fq>(R)) return dbl(a);
    return xyzz_inf();
  }
  const f29 PP = mont_sqr<Fq>(P);
  const f29 PPP = mont_mul<Fq>(P, PP);
  const f29 Q = mont_mul<Fq>(U1, PP);
  xyzz r;
  r.X = sub_k(mont_sqr<Fq>(R), add(add(PPP, Q), Q), Fq::K4);
  // Y3 = R (Q - X3) - S1 PPP with one reduction: -S1 as 8q - S1, and Q - X3
  // left unnormalised (limbs below 2^31)
  r.Y = mont_mul2<Fq>(R, sub_raw(Q, r.X, Fq::H8), sub_k(f29_zero(), S1, Fq::K8), PPP);
  r.ZZ = mont_mul<Fq>(mont_mul<Fq>(a.ZZ, b.ZZ), PP);
  r.ZZZ = mont_mul<Fq>(mont_mul<Fq>(a.ZZZ, b.ZZZ), PPP);
  return r;
}

// k * a for a small non-negative integer k (double-and-add, MSB first).
ZK_HD xyzz mul_small(const xyzz& a, uint32_t k) {
  if (k == 0) return xyzz_inf();
  xyzz r = a;
  for (int i = 30 - __builtin_clz(k); i >= 0; --i) {
    r = dbl(r);
    if ((k >> i) & 1u) r = add(r, a);
  }
  return r;
}

// Canonical affine output words (x, y plain integers < p); infinity -> (0, 0).
ZK_HD void to_affine_words(const xyzz& a, uint32_t out[16]) {
  if (is_inf(a)) {
#pragma unroll
    for (int i = 0; i < 16; i++) out[i] = 0;
    return;
  }
  const f29 I = mont_inv<Fq>(mont_mul<Fq>(a.ZZ, a.ZZZ));   // 1 / Z^5
  const f29 izz = mont_mul<Fq>(I, a.ZZZ);                   // 1 / Z^2
  const f29 izzz = mont_mul<Fq>(I, a.ZZ);                   // 1 / Z^3
  pack(from_mont<Fq>(mont_mul<Fq>(a.X, izz)), out);
  pack(from_mont<Fq>(mont_mul<Fq>(a.Y, izzz)), out + 8);
}

// Load a canonical plain affine point (x, y words; (0,0) = infinity) into
// Montgomery affine form.  Returns false for infinity.
ZK_HD bool aff_from_plain_words(const uint32_t w[16], aff& p) {
  uint32_t o = 0;
#pragma unroll
  for (int i = 0; i < 16; i++) o |= w[i];
  p.x = reduce_full<Fq>(to_mont<Fq>(unpack(w)));
  p.y = reduce_full<Fq>(to_mont<Fq>(unpack(w + 8)));
  return o != 0;
}

// Keep a value in vector registers.  Work done by one lane on wave-uniform
// data would otherwise be moved to the scalar unit, whose 32x32 multiplies
// and carry chains are several times slower for this arithmetic.
ZK_HD void force_vgpr(f29& a) {
#if defined(__HIP_DEVICE_COMPILE__)
#pragma unroll
  for (int i = 0; i < 9; i++) asm volatile("" : "+v"(a.l[i]));
#else
  (void)a;
#endif
}
ZK_HD void force_vgpr(xyzz& a) {
  force_vgpr(a.X);
  force_vgpr(a.Y);
  force_vgpr(a.ZZ);
  force_vgpr(a.ZZZ);
}

}  // namespace zk
