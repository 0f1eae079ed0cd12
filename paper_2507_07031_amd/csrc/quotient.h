// Internal interface of the quotient kernels (quotient.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.h"

namespace zk {

constexpr uint32_t QUOT_MAX_LOG_BLOWUP = 4;

// On the coset s H_(B n), B = 2^log_b: the vanishing polynomial X^n - 1 takes
// the B values s^n omega_B^k - 1 (k = j mod B at point j).  zinv_r2[k] is
// the inverse of value k times 2^522 mod r (so that a Montgomery product
// with a value divided by 2^261 yields the plain quotient).
struct QuotZinv {
  f29 zinv_r2[1u << QUOT_MAX_LOG_BLOWUP];
};

// e[j] = (e[j] * f[j] - g[j]) / Z(point j), j < big, for plain canonical
// evaluations (in place into e).
hipError_t quot_mul_pointwise(uint32_t* e, const uint32_t* f, const uint32_t* g, uint64_t big, uint32_t log_b,
                              const QuotZinv& z, hipStream_t s);

// A Poly-IOP constraint R over 2N operands (N witness polynomials at x and
// at omega x), as a sum of terms c * x_a * x_b * ...  Factor index a < N is
// f_a(x), N <= a < 2N is f_(a-N)(omega x).  coeff[t] holds c * 2^(261 d_t)
// mod r in limbs (d_t = nfac[t] factors), so that a chain of d_t - 1
// Montgomery products of plain operands followed by one with coeff[t]
// gives the plain term; for d_t = 0 it is c itself.  ident[t] marks c = 1
// with one factor (the term is the operand, no product).
constexpr uint32_t POLYIOP_MAX_N = 8;
constexpr uint32_t POLYIOP_MAX_TERMS = 16;
constexpr uint32_t POLYIOP_MAX_DEG = 4;

struct PolyIopTerms {
  f29 coeff[POLYIOP_MAX_TERMS];
  uint32_t nfac[POLYIOP_MAX_TERMS];
  uint32_t fac[POLYIOP_MAX_TERMS];    // factor i in bits 8i .. 8i+7
  uint32_t ident[POLYIOP_MAX_TERMS];
  uint32_t nterms;
  uint32_t N;
};

// On the coset of B n points (B = 2^log_b, big = B n): out[j] =
// R(E_0[j], .., E_(N-1)[j], E_0[j + B], .., E_(N-1)[j + B]) / Z(point j),
// indices mod big (the omega-shifted operand of point j is point j + B of
// the same coset).  E_k = evals + k * big * 8 words, plain canonical.
// z.zinv_r2 here holds Z^-1 * 2^261 (Montgomery form of the inverse).
hipError_t quot_polyiop_pointwise(const uint32_t* evals, uint64_t big, uint32_t log_b, const PolyIopTerms& terms,
                                  const QuotZinv& z, uint32_t* out, hipStream_t s);

// out[i] = u[i] * w^i for i < n, w^e read from split power tables
// (lo[e mod 2^14] * hi[e / 2^14], Montgomery form).
hipError_t quot_scale_powers(const uint32_t* u, uint64_t n, const f29* lo, const f29* hi, uint32_t* out,
                             hipStream_t s);

}  // namespace zk
