// Quotient by the vanishing polynomial X^n - 1 on a coset (Mul block:
// t = (f h - g) / (X^n - 1); Poly-IOP blocks: Q = R(f(x), f(omega x)) /
// (X^n - 1) for a constraint R given as monomial terms).  With f, h, g evaluated on s H_(B n), t's
// evaluations there are the pointwise (f h - g) / Z, Z = X^n - 1 taking only
// B distinct values on that coset; an inverse transform of size B n and the
// scaling of coefficient i by s^-i return t's coefficients.
//
// Both kernels stream plain canonical Fr values once through HBM.
#include "prof.h"
#include "quotient.h"

namespace zk {

namespace {

constexpr uint32_t QUOT_NT = 256;

__device__ __forceinline__ f29 ld_fr(const uint32_t* p) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  const uint32_t w[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  return unpack(w);
}

__device__ __forceinline__ void st_fr(uint32_t* p, const f29& v) {
  uint32_t w[8];
  pack(reduce_full<FrP>(v), w);
  reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

// e <- (e f - g) / Z: P = e f / 2^261 and g / 2^261 by Montgomery products,
// then one product with Z^-1 2^522 restores the plain value.
__global__ __launch_bounds__(QUOT_NT) void quot_mul_kernel(uint32_t* __restrict__ e, const uint32_t* __restrict__ f,
                                                           const uint32_t* __restrict__ g, uint64_t big,
                                                           uint32_t log_b, QuotZinv z) {
  __shared__ f29 zl[1u << QUOT_MAX_LOG_BLOWUP];
  if (threadIdx.x < (1u << log_b)) {
#pragma unroll
    for (uint32_t k = 0; k < (1u << QUOT_MAX_LOG_BLOWUP); k++)
      if (k == threadIdx.x) zl[k] = z.zinv_r2[k];
  }
  __syncthreads();
  const uint64_t j = (uint64_t)blockIdx.x * QUOT_NT + threadIdx.x;
  if (j >= big) return;
  f29 one = f29_zero();
  one.l[0] = 1;
  const f29 P = mont_mul<FrP>(ld_fr(e + j * 8), ld_fr(f + j * 8));
  const f29 G = mont_mul<FrP>(ld_fr(g + j * 8), one);
  const f29 D = sub_k(P, G, FrP::K2);
  st_fr(e + j * 8, mont_mul<FrP>(D, zl[j & ((1u << log_b) - 1)]));
}

// One point of a Poly-IOP constraint.  Operands are re-read per factor
// (the repeats hit in cache) and never converted: the term's Montgomery
// chain and its pre-scaled coefficient give the plain term value; plain
// terms (each < 1.02 r) are summed lazily (< 17 r for 16 terms) and one
// product with Z^-1 in Montgomery form divides by the vanishing polynomial.
__global__ __launch_bounds__(QUOT_NT) void quot_polyiop_kernel(const uint32_t* __restrict__ E, uint64_t big,
                                                               uint32_t log_b, PolyIopTerms T, QuotZinv z,
                                                               uint32_t* __restrict__ out) {
  const uint64_t j = (uint64_t)blockIdx.x * QUOT_NT + threadIdx.x;
  if (j >= big) return;
  const uint64_t js = (j + (1u << log_b)) & (big - 1);
  f29 total = f29_zero();
  for (uint32_t t = 0; t < T.nterms; t++) {
    const uint32_t d = T.nfac[t];
    f29 v = f29_zero();
    if (d == 0) {
      v = T.coeff[t];
    } else {
      for (uint32_t i = 0; i < d; i++) {
        const uint32_t a = (T.fac[t] >> (8 * i)) & 0xffu;
        const uint32_t k = a < T.N ? a : a - T.N;
        const f29 x = ld_fr(E + ((uint64_t)k * big + (a < T.N ? j : js)) * 8);
        v = i == 0 ? x : mont_mul<FrP>(v, x);
      }
      if (!T.ident[t]) v = mont_mul<FrP>(v, T.coeff[t]);
    }
    total = add_n(total, v);
  }
  st_fr(out + j * 8, mont_mul<FrP>(total, z.zinv_r2[j & ((1u << log_b) - 1)]));
}

__global__ __launch_bounds__(QUOT_NT) void quot_scale_kernel(const uint32_t* __restrict__ u, uint64_t n,
                                                             const f29* __restrict__ lo, const f29* __restrict__ hi,
                                                             uint32_t* __restrict__ out) {
  const uint64_t i = (uint64_t)blockIdx.x * QUOT_NT + threadIdx.x;
  if (i >= n) return;
  const uint32_t a = (uint32_t)i & 0x3fffu, b = (uint32_t)(i >> 14);
  const f29 w = mont_mul<FrP>(lo[a], hi[b]);
  st_fr(out + i * 8, mont_mul<FrP>(ld_fr(u + i * 8), w));
}

}  // namespace

hipError_t quot_mul_pointwise(uint32_t* e, const uint32_t* f, const uint32_t* g, uint64_t big, uint32_t log_b,
                              const QuotZinv& z, hipStream_t s) {
  if (big == 0) return hipSuccess;
  const ProfToken t = prof_begin("quot.pointwise", s);
  hipLaunchKernelGGL(quot_mul_kernel, dim3((uint32_t)((big + QUOT_NT - 1) / QUOT_NT)), dim3(QUOT_NT), 0, s, e, f, g,
                     big, log_b, z);
  prof_end(t, s);
  return hipGetLastError();
}

hipError_t quot_polyiop_pointwise(const uint32_t* evals, uint64_t big, uint32_t log_b, const PolyIopTerms& terms,
                                  const QuotZinv& z, uint32_t* out, hipStream_t s) {
  if (big == 0) return hipSuccess;
  const ProfToken t = prof_begin("quot.pointwise", s);
  hipLaunchKernelGGL(quot_polyiop_kernel, dim3((uint32_t)((big + QUOT_NT - 1) / QUOT_NT)), dim3(QUOT_NT), 0, s, evals,
                     big, log_b, terms, z, out);
  prof_end(t, s);
  return hipGetLastError();
}

hipError_t quot_scale_powers(const uint32_t* u, uint64_t n, const f29* lo, const f29* hi, uint32_t* out,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(quot_scale_kernel, dim3((uint32_t)((n + QUOT_NT - 1) / QUOT_NT)), dim3(QUOT_NT), 0, s, u, n, lo,
                     hi, out);
  return hipGetLastError();
}

}  // namespace zk
