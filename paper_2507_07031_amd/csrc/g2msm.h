// Internal interface of the G2 multi-scalar multiplication (g2msm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

constexpr uint32_t G2_C = 8;                          // window bits
constexpr uint32_t G2_W = 32;                         // windows (8 * 32 >= 254 + 1 for signed digits)
constexpr uint32_t G2_K = 1u << (G2_C - 1);           // buckets: |digit| = 1..128
constexpr uint32_t G2_AFF_WORDS = 32;                 // Montgomery affine point: x0 x1 y0 y1, 8 words each

// out[i] = [tau^i] H (canonical plain words x0 x1 y0 y1), i < n.  gtab: 254 *
// G2_AFF_WORDS words of scratch (the table 2^b H).
hipError_t g2_srs_from_tau(const uint32_t tau[8], uint32_t* out, uint64_t n, uint32_t* gtab, hipStream_t s);

// Pre-shifted table: tab[w * n + i] = 2^(8 w) P_i, Montgomery affine, w < G2_W
// (infinity stored as zeros).  points: canonical plain words.
hipError_t g2_build_table(const uint32_t* points, uint32_t* tab, uint64_t n, hipStream_t s);

// Scratch bytes of one n-point MSM.
size_t g2_msm_scratch_bytes(uint64_t n);

// *out = sum_i scalars[i] P_i over the table of n_tab points (first n used);
// out: canonical plain words x0 x1 y0 y1.
hipError_t g2_msm(const uint32_t* tab, uint64_t n_tab, const uint32_t* scalars, uint64_t n, uint32_t* out,
                  void* scratch, hipStream_t s);

}  // namespace zk
