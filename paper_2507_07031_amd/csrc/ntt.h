// Internal interface of the NTT pass kernel (see ntt.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "field.h"

namespace zk {

// One pass: a batch of M = 2^m point transforms held in LDS.
//   input  element (batch b, point i) at in[(b + i*s_in)]          (words x8)
//   output element (batch b, point k) at out[(b*b_out + k*s_out)], or, with
//   b_hi_log > 0, at out[(b mod 2^b_hi_log)*b_out + (b >> b_hi_log)*b_out_hi + k*s_out]
// Elements with input index >= valid_n read as zero.
struct NttPass {
  const uint32_t* in;
  uint32_t* out;
  uint32_t m;          // log2 points per transform (<= 12)
  uint32_t G;          // transforms per workgroup (M * G <= 4096)
  uint32_t nbatch;     // number of transforms
  uint32_t s_in;       // input stride between points
  uint32_t s_out;      // output stride between points
  uint32_t b_out;      // output stride between transforms
  uint32_t valid_n;
  const f29* tw_lo;    // omega^e, e < 2^14 (forward or inverse root)
  const f29* tw_hi;    // omega^(e 2^14)
  const f29* ladder;   // in-tile twiddles: ladder[2^(k-1) + j] = omega_(2^k)^j
  uint32_t post_tw_L;  // 0: none; else multiply (b, k) by omega_(2^L)^((b >> tw_shift) k)
  uint32_t tw_scaled;  // tw_lo holds omega^e times a constant c (every (b, k) is then multiplied by c
                       // times its twiddle, exponent 0 included)
  uint32_t tw_shift;
  uint32_t b_hi_log;   // 0: plain batch stride b_out
  uint32_t b_out_hi;
  const f29* pre_lo;   // coset: multiply input i by g^i (nullptr: none)
  const f29* pre_hi;
  const f29* post_scale;  // multiply every output by this constant (nullptr: none)
  uint32_t unit_log;   // stages per LDS round trip at most: 3 (8 points a thread) or 2 (4 points)
  uint32_t zero_log;   // points i >= 2^(m - zero_log) of every transform are zero padding (input index
                       // >= valid_n): the first zero_log stages only copy, and are not run
  const uint32_t* tw_full;  // nullptr, or the post twiddle (scale included) of every (b, k) at entry
                            // ((b >> tw_shift) << m) + k, as nine limb planes of 2^post_tw_L words
                            // (ntt_full_twiddles with mA = m); replaces tw_lo / tw_hi
};

hipError_t ntt_pass_setup();
hipError_t ntt_launch_pass(const NttPass& p, hipStream_t s);
struct Words8 {
  uint32_t w[8];
};

// lo[e] = base^e, hi[e] = base^(e 2^14), e < 2^14 (Montgomery form); base canonical.
hipError_t ntt_make_pow_tables(Words8 base, f29* lo, f29* hi, hipStream_t s);
size_t ntt_pass_lds_bytes();
// ladder[2^(k-1) + j] = omega_(2^k)^j (k <= tile log) from a "hi" table; entries: ntt_ladder_entries()
size_t ntt_ladder_entries();
hipError_t ntt_make_ladder(const f29* hi, f29* ladder, hipStream_t s);
// out[l 2^14 + e] = lo[e] * scales[l] (canonical Montgomery form), l < nscales.
hipError_t ntt_scale_tables(const f29* lo, const f29* scales, uint32_t nscales, f29* out, hipStream_t s);
uint32_t ntt_tile_log();
// The post twiddles of the first pass of a two-pass transform of 2^L points
// whose first pass runs 2^mA-point transforms: entry i1 2^mA + k2 (limb l at
// out[l 2^L + i1 2^mA + k2]) is omega_(2^L)^(i1 k2) from the split tables lo /
// hi (times the constant of a scaled lo table).  out holds 9 * 2^L words; L <= 28.
hipError_t ntt_full_twiddles(const f29* lo, const f29* hi, uint32_t scaled, uint32_t L, uint32_t mA, uint32_t* out,
                             hipStream_t s);

}  // namespace zk
