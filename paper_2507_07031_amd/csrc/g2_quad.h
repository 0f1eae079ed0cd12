// G2 XYZZ addition and doubling spread over the four lanes of a quad, for
// the dependent chains of the G2 bucket sums (the quad scheme of
// curve_quad.h with Fq2 coordinates).
//
// Lane c of a quad holds coordinate c of a point (X, Y, ZZ, ZZZ for
// c = 0..3, each an Fq2 value); each lane computes one Fq2 product per step
// and operands move between the lanes of the quad by DPP quad permutes:
//   addition: 4 product steps instead of 14 Fq2 products in sequence,
//   doubling: 3 product steps instead of 9.
// The formulas are g2_add / g2_dbl of g2.h; squares are taken as products of
// a value with itself, so the XYZZ representatives can differ from the
// one-lane formulas while the points are the same.  All four lanes of every
// quad must be active.
#pragma once
#include "curve_quad.h"
#include "g2.h"

namespace zk {

template <int CTRL>
__device__ __forceinline__ fp2 qperm2(const fp2& v) {
  return fp2{qperm<CTRL>(v.c0), qperm<CTRL>(v.c1)};
}

__device__ __forceinline__ fp2 fsel2(bool c, const fp2& a, const fp2& b) { return fp2{fsel(c, a.c0, b.c0), fsel(c, a.c1, b.c1)}; }

// Coordinate c of a G2 XYZZ point stored as 72 words (X.c0 X.c1 Y.c0 ...,
// nine words each): words 18 c .. 18 c + 17.
__device__ __forceinline__ fp2 ldq2(const uint32_t* p, uint32_t c) {
  fp2 r;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    r.c0.l[i] = p[18 * c + i];
    r.c1.l[i] = p[18 * c + 9 + i];
  }
  return r;
}

__device__ __forceinline__ void stq2(uint32_t* p, uint32_t c, const fp2& v) {
#pragma unroll
  for (int i = 0; i < 9; i++) {
    p[18 * c + i] = v.c0.l[i];
    p[18 * c + 9 + i] = v.c1.l[i];
  }
}

// The quad's whole point in every lane.
__device__ __forceinline__ g2xyzz g2q_gather(const fp2& v) {
  return g2xyzz{qperm2<qp(0, 0, 0, 0)>(v), qperm2<qp(1, 1, 1, 1)>(v), qperm2<qp(2, 2, 2, 2)>(v),
                qperm2<qp(3, 3, 3, 3)>(v)};
}

// 2A.  a: this lane's coordinate of A.
__device__ __forceinline__ fp2 g2q_dbl(const fp2& a) {
  const uint32_t c = quad_lane();
  const bool inf = qperm_u32<qp(2, 2, 2, 2)>(fp2_is_zero_limbs(a) ? 1u : 0u) != 0;
  // step 1: lane 0 x2 = X^2, lane 1 V = U^2 with U = 2Y
  const fp2 u = fp2_add(a, a);
  const fp2 s1 = fsel2(c == 1, u, a);
  const fp2 t1 = fp2_mul(s1, s1);
  const fp2 x2 = qperm2<qp(0, 0, 0, 0)>(t1);
  const fp2 V = qperm2<qp(1, 1, 1, 1)>(t1);
  const fp2 M = fp2_add(fp2_add(x2, x2), x2);
  // step 2: lane 0 S = X V, lane 1 W = U V, lane 2 ZZ3 = ZZ V, lane 3 M^2
  const fp2 x = fsel2(c == 1, u, fsel2(c == 3, M, a));
  const fp2 t2 = fp2_mul(x, fsel2(c == 3, M, V));
  const fp2 S = qperm2<qp(0, 0, 0, 0)>(t2);
  const fp2 W = qperm2<qp(1, 1, 1, 1)>(t2);
  const fp2 MM = qperm2<qp(3, 3, 3, 3)>(t2);
  const fp2 X3 = fp2_sub(MM, fp2_add(S, S));
  const fp2 SX = fp2_sub(S, X3);
  // step 3: lane 0 M (S - X3), lane 1 W Y, lane 3 ZZZ3 = W ZZZ
  const fp2 t3 = fp2_mul(fsel2(c == 0, M, W), fsel2(c == 0, SX, a));
  const fp2 Y3 = fp2_sub(qperm2<qp(0, 0, 0, 0)>(t3), qperm2<qp(1, 1, 1, 1)>(t3));
  const fp2 r = fsel2(c == 0, X3, fsel2(c == 1, Y3, fsel2(c == 2, t2, t3)));
  return fsel2(inf, a, r);
}

// A + B.  a, b: this lane's coordinates of A and B.
__device__ __forceinline__ fp2 g2q_add(const fp2& a, const fp2& b) {
  const uint32_t c = quad_lane();
  const bool odd = (c & 1u) != 0;
  const bool inf_a = qperm_u32<qp(2, 2, 2, 2)>(fp2_is_zero_limbs(a) ? 1u : 0u) != 0;
  const bool inf_b = qperm_u32<qp(2, 2, 2, 2)>(fp2_is_zero_limbs(b) ? 1u : 0u) != 0;
  // step 1: U1 = X1 ZZ2, U2 = X2 ZZ1, S1 = Y1 ZZZ2, S2 = Y2 ZZZ1 (lanes 0..3)
  const fp2 x1 = fsel2(odd, qperm2<qp(0, 0, 1, 1)>(b), qperm2<qp(0, 0, 1, 1)>(a));
  const fp2 y1 = fsel2(odd, qperm2<qp(2, 2, 3, 3)>(a), qperm2<qp(2, 2, 3, 3)>(b));
  const fp2 t1 = fp2_mul(x1, y1);
  // P = U2 - U1 (lanes 0, 1), R = S2 - S1 (lanes 2, 3)
  const fp2 sw = qperm2<qp(1, 0, 3, 2)>(t1);
  const fp2 d = odd ? fp2_sub(t1, sw) : fp2_sub(sw, t1);
  const bool zd = fp2_is_zero_mod(d);
  const bool p_zero = qperm_u32<qp(0, 0, 0, 0)>(zd ? 1u : 0u) != 0;
  const bool r_zero = qperm_u32<qp(2, 2, 2, 2)>(zd ? 1u : 0u) != 0;
  // step 2: lane 0 PP = P^2, lane 1 ZZ1 ZZ2, lane 2 R^2, lane 3 ZZZ1 ZZZ2
  const fp2 x2 = fsel2(odd, qperm2<qp(0, 2, 2, 3)>(a), d);
  const fp2 y2 = fsel2(odd, qperm2<qp(0, 2, 2, 3)>(b), d);
  const fp2 t2 = fp2_mul(x2, y2);
  const fp2 PP = qperm2<qp(0, 0, 0, 0)>(t2);
  // step 3: lane 0 PPP = P PP, lane 1 Q = U1 PP, lane 2 ZZ3 = ZZ1ZZ2 PP
  const fp2 u1 = qperm2<qp(0, 0, 2, 3)>(t1);
  const fp2 zz12 = qperm2<qp(0, 1, 1, 3)>(t2);
  const fp2 x3 = fsel2(c == 0, d, fsel2(c == 1, u1, zz12));
  const fp2 t3 = fp2_mul(x3, PP);
  const fp2 PPP = qperm2<qp(0, 0, 0, 0)>(t3);
  const fp2 Q = qperm2<qp(1, 1, 1, 1)>(t3);
  const fp2 RR = qperm2<qp(2, 2, 2, 2)>(t2);
  const fp2 X3 = fp2_sub(RR, fp2_add(fp2_add(PPP, Q), Q));
  const fp2 QX = fp2_sub(Q, X3);
  // step 4: lane 0 R (Q - X3), lane 1 S1 PPP, lane 3 ZZZ3 = ZZZ1ZZZ2 PPP
  const fp2 r_ = qperm2<qp(2, 2, 2, 3)>(d);
  const fp2 s1 = qperm2<qp(2, 2, 2, 3)>(t1);
  const fp2 x4 = fsel2(c == 0, r_, fsel2(c == 1, s1, t2));
  const fp2 t4 = fp2_mul(x4, fsel2(c == 0, QX, PPP));
  const fp2 Y3 = fp2_sub(qperm2<qp(0, 0, 0, 0)>(t4), qperm2<qp(1, 1, 1, 1)>(t4));
  fp2 r = fsel2(c == 0, X3, fsel2(c == 1, Y3, fsel2(c == 2, t3, t4)));
  // special cases, decided per quad
  if (p_zero) r = r_zero ? g2q_dbl(a) : fp2_zero();
  if (inf_b) r = a;
  if (inf_a) r = b;
  return r;
}

}  // namespace zk
