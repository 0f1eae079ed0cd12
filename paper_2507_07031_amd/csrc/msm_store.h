// XYZZ points in device memory (internal to the MSM kernels): 36 words,
// the nine limbs of X, Y, ZZ, ZZZ in that order.
#pragma once
#include "curve.h"

namespace zk {

__device__ __forceinline__ xyzz ld_xyzz(const uint32_t* p) {
  uint32_t w[36];
#pragma unroll
  for (int q = 0; q < 9; q++) {
    const uint4 v = reinterpret_cast<const uint4*>(p)[q];
    w[4 * q] = v.x;
    w[4 * q + 1] = v.y;
    w[4 * q + 2] = v.z;
    w[4 * q + 3] = v.w;
  }
  xyzz a;
#pragma unroll
  for (int i = 0; i < 9; i++) {
    a.X.l[i] = w[i];
    a.Y.l[i] = w[9 + i];
    a.ZZ.l[i] = w[18 + i];
    a.ZZZ.l[i] = w[27 + i];
  }
  return a;
}

// Coordinate c (X, Y, ZZ, ZZZ for c = 0..3) of a point stored as 36 words:
// the quad form of ld_xyzz / st_xyzz (the four lanes of a quad together
// move the same 36 words).
__device__ __forceinline__ f29 ldq(const uint32_t* p, uint32_t c) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = p[9 * c + i];
  return r;
}

__device__ __forceinline__ void stq(uint32_t* p, uint32_t c, const f29& v) {
#pragma unroll
  for (int i = 0; i < 9; i++) p[9 * c + i] = v.l[i];
}

__device__ __forceinline__ void st_xyzz(uint32_t* p, const xyzz& a) {
  uint32_t w[36];
#pragma unroll
  for (int i = 0; i < 9; i++) {
    w[i] = a.X.l[i];
    w[9 + i] = a.Y.l[i];
    w[18 + i] = a.ZZ.l[i];
    w[27 + i] = a.ZZZ.l[i];
  }
#pragma unroll
  for (int q = 0; q < 9; q++)
    reinterpret_cast<uint4*>(p)[q] = make_uint4(w[4 * q], w[4 * q + 1], w[4 * q + 2], w[4 * q + 3]);
}

}  // namespace zk
