// Input checks behind zk_set_validate: Fr inputs are canonical (< r), G1
// inputs are canonical affine points on y^2 = x^3 + 3 or (0, 0), G2 inputs
// canonical points of order r on the twist y^2 = x^3 + 3/(9 + u) or all
// zeros.  Each launch ORs its findings into a device flag word.
#include "g2.h"
#include "validate.h"

namespace zk {

namespace {

__device__ __forceinline__ bool below(const uint32_t* w, const uint32_t (&m)[8]) {
  unsigned br = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], m[i], br, &br);
  return br != 0;
}

__global__ void check_fr_kernel(const uint32_t* __restrict__ v, uint64_t n, uint32_t* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t w[8];
#pragma unroll
  for (int k = 0; k < 8; k++) w[k] = v[i * 8 + k];
  if (!below(w, FrP::M32)) atomicOr(flag, VALIDATE_FR);
}

__global__ void check_g1_kernel(const uint32_t* __restrict__ pts, uint64_t n, uint32_t* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t w[16];
  uint32_t o = 0;
#pragma unroll
  for (int k = 0; k < 16; k++) {
    w[k] = pts[i * 16 + k];
    o |= w[k];
  }
  if (o == 0) return;  // (0, 0) is the point at infinity
  if (!below(w, FqP::M32) || !below(w + 8, FqP::M32)) {
    atomicOr(flag, VALIDATE_G1);
    return;
  }
  // y^2 = x^3 + 3 in Montgomery form
  const f29 x = to_mont<FqP>(unpack(w));
  const f29 y = to_mont<FqP>(unpack(w + 8));
  f29 three = f29_zero();
  three.l[0] = 3;
  const f29 lhs = reduce_full<FqP>(mont_sqr<FqP>(y));
  const f29 rhs = reduce_full<FqP>(add_n(mont_mul<FqP>(mont_sqr<FqP>(x), x), to_mont<FqP>(three)));
  uint32_t d = 0;
#pragma unroll
  for (int k = 0; k < 9; k++) d |= lhs.l[k] ^ rhs.l[k];
  if (d) atomicOr(flag, VALIDATE_G1);
}

__global__ void check_g2_kernel(const uint32_t* __restrict__ pts, uint64_t n, uint32_t* flag) {
  const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t w[32];
  for (int k = 0; k < 32; k++) w[k] = pts[i * 32 + k];
  if (!g2_words_valid(w)) atomicOr(flag, VALIDATE_G2);
}

inline uint32_t blocks_for(uint64_t n) { return (uint32_t)((n + 255) / 256); }

}  // namespace

hipError_t validate_fr(const uint32_t* v, uint64_t n, uint32_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(check_fr_kernel, dim3(blocks_for(n)), dim3(256), 0, s, v, n, flag);
  return hipGetLastError();
}

hipError_t validate_g1(const uint32_t* pts, uint64_t n, uint32_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(check_g1_kernel, dim3(blocks_for(n)), dim3(256), 0, s, pts, n, flag);
  return hipGetLastError();
}

hipError_t validate_g2(const uint32_t* pts, uint64_t n, uint32_t* flag, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(check_g2_kernel, dim3((uint32_t)((n + 63) / 64)), dim3(64), 0, s, pts, n, flag);
  return hipGetLastError();
}

}  // namespace zk
