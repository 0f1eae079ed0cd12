// XYZZ addition and doubling spread over the four lanes of a quad, for code
// whose point operations form one dependent chain (a single lane would do all
// the products of a formula one after another).
//
// Lane c of a quad holds coordinate c of a point: X, Y, ZZ, ZZZ for c = 0..3.
// Each lane computes one Montgomery product per step; operands move between
// the lanes of the quad by DPP quad permutes.  The products, subtractions
// and their lazy-reduction multiples are exactly those of add() and dbl() in
// curve.h (a Montgomery product does not depend on operand order, and a
// square equals the product of a value with itself limb for limb), so the
// results are bit-identical to the one-lane formulas:
//   addition: 4 product steps instead of 14 products in sequence,
//   doubling: 3 product steps instead of 9.
// All four lanes of every quad must be active.
#pragma once
#include "curve.h"

namespace zk {

constexpr int qp(int a, int b, int c, int d) { return a | (b << 2) | (c << 4) | (d << 6); }

template <int CTRL>
__device__ __forceinline__ uint32_t qperm_u32(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xF, 0xF, false);
}

template <int CTRL>
__device__ __forceinline__ f29 qperm(const f29& v) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = qperm_u32<CTRL>(v.l[i]);
  return r;
}

__device__ __forceinline__ f29 fsel(bool c, const f29& a, const f29& b) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = c ? a.l[i] : b.l[i];
  return r;
}

__device__ __forceinline__ uint32_t quad_lane() { return __lane_id() & 3u; }

// One coordinate of a point per lane.
__device__ __forceinline__ f29 quad_coord(const xyzz& p, uint32_t c) {
  return c == 0 ? p.X : c == 1 ? p.Y : c == 2 ? p.ZZ : p.ZZZ;
}

// Gather the four coordinates of the quad's point into every lane.
__device__ __forceinline__ xyzz quad_gather(const f29& v) {
  xyzz p;
  p.X = qperm<qp(0, 0, 0, 0)>(v);
  p.Y = qperm<qp(1, 1, 1, 1)>(v);
  p.ZZ = qperm<qp(2, 2, 2, 2)>(v);
  p.ZZZ = qperm<qp(3, 3, 3, 3)>(v);
  return p;
}

// 2A.  a: this lane's coordinate of A.
__device__ __forceinline__ f29 quad_dbl(const f29& a) {
  const uint32_t c = quad_lane();
  const bool inf = qperm_u32<qp(2, 2, 2, 2)>(f29_is_zero_limbs(a) ? 1u : 0u) != 0;
  // step 1: lane 0 x2 = X^2, lane 1 V = U^2 with U = 2Y
  const f29 u = add(a, a);
  const f29 s1 = c == 1 ? u : a;
  const f29 t1 = mont_mul<Fq>(s1, s1);
  const f29 x2 = qperm<qp(0, 0, 0, 0)>(t1);
  const f29 V = qperm<qp(1, 1, 1, 1)>(t1);
  const f29 M = add_n(add(x2, x2), x2);
  // step 2: lane 0 S = X V, lane 1 W = U V, lane 2 ZZ3 = ZZ V, lane 3 M^2
  const f29 x = c == 1 ? u : (c == 3 ? M : a);
  const f29 t2 = mont_mul<Fq>(x, c == 3 ? M : V);
  const f29 S = qperm<qp(0, 0, 0, 0)>(t2);
  const f29 W = qperm<qp(1, 1, 1, 1)>(t2);
  const f29 MM = qperm<qp(3, 3, 3, 3)>(t2);
  const f29 X3 = sub_k(MM, add(S, S), Fq::K4);
  const f29 SX = sub_k(S, X3, Fq::K8);
  // step 3: lane 0 M (S - X3), lane 1 W Y, lane 3 ZZZ3 = W ZZZ
  const f29 t3 = mont_mul<Fq>(c == 0 ? M : W, c == 0 ? SX : a);
  const f29 ya = qperm<qp(0, 0, 0, 0)>(t3);
  const f29 yb = qperm<qp(1, 1, 1, 1)>(t3);
  const f29 Y3 = sub_k(ya, yb, Fq::K2);
  const f29 r = c == 0 ? X3 : (c == 1 ? Y3 : (c == 2 ? t2 : t3));
  return fsel(inf, a, r);
}

// A + B.  a, b: this lane's coordinates of A and B.
__device__ __forceinline__ f29 quad_add(const f29& a, const f29& b) {
  const uint32_t c = quad_lane();
  const bool odd = (c & 1u) != 0;
  const bool inf_a = qperm_u32<qp(2, 2, 2, 2)>(f29_is_zero_limbs(a) ? 1u : 0u) != 0;
  const bool inf_b = qperm_u32<qp(2, 2, 2, 2)>(f29_is_zero_limbs(b) ? 1u : 0u) != 0;
  // step 1: U1 = X1 ZZ2, U2 = X2 ZZ1, S1 = Y1 ZZZ2, S2 = Y2 ZZZ1 (lanes 0..3)
  const f29 x1 = fsel(odd, qperm<qp(0, 0, 1, 1)>(b), qperm<qp(0, 0, 1, 1)>(a));
  const f29 y1 = fsel(odd, qperm<qp(2, 2, 3, 3)>(a), qperm<qp(2, 2, 3, 3)>(b));
  const f29 t1 = mont_mul<Fq>(x1, y1);
  // P = U2 - U1 (lanes 0, 1), R = S2 - S1 (lanes 2, 3)
  const f29 sw = qperm<qp(1, 0, 3, 2)>(t1);
  const f29 d = odd ? sub_k(t1, sw, Fq::K8) : sub_k(sw, t1, Fq::K8);
  const bool zd = is_zero_mod<Fq>(d);
  const bool p_zero = qperm_u32<qp(0, 0, 0, 0)>(zd ? 1u : 0u) != 0;
  const bool r_zero = qperm_u32<qp(2, 2, 2, 2)>(zd ? 1u : 0u) != 0;
  // step 2: lane 0 PP = P^2, lane 1 ZZ1 ZZ2, lane 2 R^2, lane 3 ZZZ1 ZZZ2
  const f29 x2 = fsel(odd, qperm<qp(0, 2, 2, 3)>(a), d);
  const f29 y2 = fsel(odd, qperm<qp(0, 2, 2, 3)>(b), d);
  const f29 t2 = mont_mul<Fq>(x2, y2);
  const f29 PP = qperm<qp(0, 0, 0, 0)>(t2);
  // step 3: lane 0 PPP = P PP, lane 1 Q = U1 PP, lane 2 ZZ3 = ZZ1ZZ2 PP
  const f29 u1 = qperm<qp(0, 0, 2, 3)>(t1);
  const f29 zz12 = qperm<qp(0, 1, 1, 3)>(t2);
  const f29 x3 = c == 0 ? d : (c == 1 ? u1 : zz12);
  const f29 t3 = mont_mul<Fq>(x3, PP);
  const f29 PPP = qperm<qp(0, 0, 0, 0)>(t3);
  const f29 Q = qperm<qp(1, 1, 1, 1)>(t3);
  const f29 RR = qperm<qp(2, 2, 2, 2)>(t2);
  const f29 X3 = sub_k(RR, add(add(PPP, Q), Q), Fq::K4);
  const f29 QX = sub_k(Q, X3, Fq::K8);
  // step 4: lane 0 R (Q - X3), lane 1 S1 PPP, lane 3 ZZZ3 = ZZZ1ZZZ2 PPP
  const f29 r_ = qperm<qp(2, 2, 2, 3)>(d);
  const f29 s1 = qperm<qp(2, 2, 2, 3)>(t1);
  const f29 x4 = c == 0 ? r_ : (c == 1 ? s1 : t2);
  const f29 t4 = mont_mul<Fq>(x4, c == 0 ? QX : PPP);
  const f29 ya = qperm<qp(0, 0, 0, 0)>(t4);
  const f29 yb = qperm<qp(1, 1, 1, 1)>(t4);
  const f29 Y3 = sub_k(ya, yb, Fq::K2);
  f29 r = c == 0 ? X3 : (c == 1 ? Y3 : (c == 2 ? t3 : t4));
  // special cases, decided per quad
  if (p_zero) r = r_zero ? quad_dbl(a) : f29_zero();
  if (inf_b) r = a;
  if (inf_a) r = b;
  return r;
}

}  // namespace zk
