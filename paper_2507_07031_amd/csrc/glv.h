// Scalar splitting by the BN254 G1 endomorphism (Gallant, Lambert and
// Vanstone, CRYPTO 2001).
//
// G1 has an efficiently computable endomorphism phi(x, y) = (beta x, y),
// beta a primitive cube root of unity in Fq; on the order-r group it acts as
// multiplication by lambda, a primitive cube root of unity mod r.  A scalar
// k < r is rewritten as k = k1 + k2 lambda (mod r) with |k1|, |k2| < 2^128,
// so k P = k1 P + k2 phi(P): two half-length multiplications that share one
// chain of doublings.
//
// The split rounds k against a reduced basis of the lattice
// {(x, y) : x + y lambda = 0 mod r}: v1 = (a1, b1), v2 = (a2, b2), found by
// the extended Euclidean algorithm on (r, lambda) and stopped at sqrt(r):
//   c1 = round(b2 k / r),  c2 = round(-b1 k / r),
//   k1 = k - c1 a1 - c2 a2,  k2 = -c1 b1 - c2 b2.
// The quotients use g1 = round(2^256 b2 / r) and g2 = round(2^256 (-b1) / r):
// c = floor((k g + 2^255) / 2^256).  Here b1 < 0 and -b1 = a2.  Over all
// k < r the halves stay below 2^128 (the basis vectors are below 2^127).
//
// Integers are little-endian 32-bit words; the functions run on host and
// device so that a host build can be checked against exact integers.
#pragma once
#include <stdint.h>

#include "field.h"

namespace zk {

struct GlvConst {
  // lambda mod r with lambda^2 + lambda + 1 = 0 and lambda (x, y) = (beta x, y)
  static constexpr uint32_t LAMBDA[8] = {0x36636f23u, 0xb8ca0b2du, 0xec2bc5e9u, 0xcc37a73fu,
                                         0x3fd84104u, 0x048b6e19u, 0xe131a029u, 0x30644e72u};
  // beta mod q, the matching cube root of unity in the base field
  static constexpr uint32_t BETA[8] = {0x607cfd48u, 0xe4bd44e5u, 0xbb966e3du, 0xc28f069fu,
                                       0xe0acccb0u, 0x5e6dd9e7u, 0xe131a029u, 0x30644e72u};
  static constexpr uint32_t A1[4] = {0x7d4f1128u, 0x8211bbebu, 0xeeb859fcu, 0x6f4d8248u};
  static constexpr uint32_t A2[2] = {0x94d213e3u, 0x89d32568u};  // = -b1
  static constexpr uint32_t B2[4] = {0x1221250bu, 0x0be4e154u, 0xeeb859fdu, 0x6f4d8248u};
  static constexpr uint32_t G1[5] = {0x00ff6565u, 0x5398fd03u, 0xa773d2d2u, 0x4ccef014u, 0x2u};
  static constexpr uint32_t G2[3] = {0xc7e0b3d7u, 0xd91d232eu, 0x2u};
};

// out[0 .. NA+NB) = a * b (schoolbook, 64-bit column products).
template <int NA, int NB>
ZK_HD void glv_mulw(const uint32_t (&a)[NA], const uint32_t (&b)[NB], uint32_t (&out)[NA + NB]) {
#pragma unroll
  for (int i = 0; i < NA + NB; i++) out[i] = 0;
#pragma unroll
  for (int i = 0; i < NA; i++) {
    uint64_t carry = 0;
#pragma unroll
    for (int j = 0; j < NB; j++) {
      const uint64_t t = (uint64_t)a[i] * b[j] + out[i + j] + carry;
      out[i + j] = (uint32_t)t;
      carry = t >> 32;
    }
    out[i + NB] = (uint32_t)carry;
  }
}

// floor((k g + 2^255) / 2^256) for k < 2^256: the rounded quotient, NC words.
template <int NG, int NC>
ZK_HD void glv_round_quot(const uint32_t (&k)[8], const uint32_t (&g)[NG], uint32_t (&c)[NC]) {
  uint32_t p[8 + NG];
  glv_mulw<8, NG>(k, g, p);
  uint64_t s = (uint64_t)p[7] + 0x80000000u;
  p[7] = (uint32_t)s;
#pragma unroll
  for (int i = 8; i < 8 + NG; i++) {
    s = (uint64_t)p[i] + (s >> 32);
    p[i] = (uint32_t)s;
  }
#pragma unroll
  for (int i = 0; i < NC; i++) c[i] = p[8 + i];
}

// Two's complement of an N-word value in place when neg is set.
template <int N>
ZK_HD void glv_cneg(uint32_t (&r)[N], bool neg) {
  uint64_t c = neg ? 1u : 0u;
  const uint32_t mask = neg ? 0xffffffffu : 0u;
#pragma unroll
  for (int i = 0; i < N; i++) {
    c += (uint64_t)(r[i] ^ mask);
    r[i] = (uint32_t)c;
    c >>= 32;
  }
}

// k = (-1)^n1 k1 + (-1)^n2 k2 lambda (mod r) for canonical k < r, with
// k1, k2 < 2^128 (four words each).
ZK_HD void glv_split(const uint32_t (&k)[8], uint32_t (&k1)[4], bool& n1, uint32_t (&k2)[4], bool& n2) {
  uint32_t c1[4], c2[2];
  glv_round_quot<5, 4>(k, GlvConst::G1, c1);
  glv_round_quot<3, 2>(k, GlvConst::G2, c2);
  // k1 = k - c1 a1 - c2 a2 over nine words
  uint32_t t1[8], t2[4];
  glv_mulw<4, 4>(c1, GlvConst::A1, t1);
  glv_mulw<2, 2>(c2, GlvConst::A2, t2);
  uint32_t r[9];
  int64_t b = 0;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    int64_t v = (int64_t)(i < 8 ? k[i] : 0u) - (int64_t)(i < 8 ? t1[i] : 0u) - (int64_t)(i < 4 ? t2[i] : 0u) + b;
    r[i] = (uint32_t)v;
    b = v >> 32;  // arithmetic shift: the borrow, -2 .. 0
  }
  n1 = (r[8] >> 31) != 0;
  glv_cneg<9>(r, n1);
#pragma unroll
  for (int i = 0; i < 4; i++) k1[i] = r[i];
  // k2 = c1 a2 - c2 b2 over seven words (-b1 = a2)
  uint32_t u1[6], u2[6];
  glv_mulw<4, 2>(c1, GlvConst::A2, u1);
  glv_mulw<2, 4>(c2, GlvConst::B2, u2);
  uint32_t s[7];
  b = 0;
#pragma unroll
  for (int i = 0; i < 7; i++) {
    int64_t v = (int64_t)(i < 6 ? u1[i] : 0u) - (int64_t)(i < 6 ? u2[i] : 0u) + b;
    s[i] = (uint32_t)v;
    b = v >> 32;
  }
  n2 = (s[6] >> 31) != 0;
  glv_cneg<7>(s, n2);
#pragma unroll
  for (int i = 0; i < 4; i++) k2[i] = s[i];
}

}  // namespace zk
