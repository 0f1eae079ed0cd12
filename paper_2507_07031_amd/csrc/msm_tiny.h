// Small commitments over a prepared SRS by a table of small multiples
// (msm_tiny.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace zk {

// A table of m 16^w P_i (m = 1..8, w < 64) over the first nt <= TINY_MAX
// points of a prepared SRS, and a run that sums one table point per nonzero
// signed 4-bit digit by trees.
constexpr uint32_t TINY_WINDOWS = 64;
constexpr uint32_t TINY_MULTS = 8;
constexpr uint32_t TINY_MAX = 4096;
constexpr uint32_t TINY_NT = 256;
// Points in the table of nt points (64 B each).
uint64_t msm_tiny_table_points(uint32_t nt);
// tab16: the 16-bit-window pre-shifted table (rows w < 16, row stride tab_n);
// hipErrorInvalidValue unless tab_c = 16, tab_W >= 16 and nt <= tab_n.
hipError_t msm_build_tiny_table(const uint32_t* tab16, uint32_t tab_c, uint32_t tab_W, uint64_t tab_n, uint32_t nt,
                                uint32_t* tiny, hipStream_t s);
size_t msm_tiny_workspace_bytes(uint32_t n);
// 0 < n <= min(nt, TINY_MAX); workspace of msm_tiny_workspace_bytes(n);
// out16: canonical affine.  after_terms: if not null, recorded after the
// terms kernel (the rest is a short latency-bound tree).
hipError_t msm_tiny_run(const uint32_t* tiny, uint32_t nt, const uint32_t* scalars, uint32_t n, void* workspace,
                        uint32_t* out16, hipStream_t s, hipEvent_t after_terms = nullptr);

}  // namespace zk
