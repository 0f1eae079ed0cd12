// Internal interface of the multi-scalar-multiplication kernels (msm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

constexpr uint32_t MSM_NT = 256;          // threads per workgroup (accumulate / reduce)
constexpr uint32_t MSM_SLOTS = 2 * MSM_NT; // records combined per workgroup
constexpr uint32_t KEY_SENTINEL = 0xfffffffeu;
constexpr uint32_t XYZZ_WORDS = 36;       // four 9-limb coordinates

// Geometry of one Pippenger run.
struct MsmPlan {
  uint32_t n;          // points / scalars
  uint32_t c;          // window bits; digits are signed in [-2^(c-1), 2^(c-1)]
  uint32_t W;          // windows = ceil(254 / c)
  uint32_t K;          // buckets per window = 2^(c-1)
  uint32_t shared;     // 1: all windows share K buckets (bases pre-shifted by 2^(cw))
  uint32_t nbins;      // shared ? K : W*K
  uint32_t tab_stride; // shared: point index of window w = w*tab_stride + i
  uint32_t chunk;      // digits per histogram / scatter workgroup
  uint32_t L;          // sorted entries per accumulating thread
  uint32_t acc_blocks; // accumulate workgroups
  uint32_t LB;         // buckets per thread in the running-sum reduction
  uint32_t J;          // LB-chunks per window = K / LB
};

MsmPlan msm_plan(uint32_t n, uint32_t c, bool shared, uint32_t tab_stride);
uint32_t msm_default_c(uint32_t n);

// Scratch buffers of one run (device pointers), sizes from msm_workspace_layout.
struct MsmBuffers {
  uint32_t* digits;    // W*n
  uint32_t* counts;    // nbins
  uint32_t* offsets;   // nbins + 1
  uint32_t* cursor;    // nbins
  uint32_t* scan_tmp;  // scan block sums
  uint32_t* keys;      // W*n
  uint32_t* vals;      // W*n
  uint32_t* buckets;   // nbins * 36
  uint32_t* rec_keys[2];
  uint32_t* rec_flags[2];
  uint32_t* rec_pts[2];
  uint32_t* vbuf;      // (shared ? 1 : W) * J * 36
  uint32_t* wsum;      // (shared ? 1 : W) * 36
};

size_t msm_workspace_bytes(const MsmPlan& p);
MsmBuffers msm_carve(const MsmPlan& p, void* base);

// Full pipeline: scalars (canonical, 8 words each) against Montgomery-form
// affine points (16 words each) -> canonical affine result (16 words, device).
hipError_t msm_run(const MsmPlan& p, const uint32_t* mont_points, const uint32_t* scalars,
                   const MsmBuffers& b, uint32_t* out16, hipStream_t s);

// Canonical plain affine points -> Montgomery-form affine points (count n).
hipError_t msm_points_to_mont(const uint32_t* plain, uint32_t* mont, uint64_t n, hipStream_t s);

// Pre-shifted table: tab[w*n + i] = 2^(c w) * P_i (Montgomery affine), w < W.
hipError_t msm_build_table(const uint32_t* plain_points, uint32_t* tab, uint64_t n, uint32_t c,
                           uint32_t W, hipStream_t s);

// out[i] = [tau^i] G (canonical plain affine), i < n.
struct Tau8 {
  uint32_t w[8];
};
hipError_t srs_from_tau(Tau8 tau, uint32_t* out, uint64_t n, uint32_t* gtab_dev, hipStream_t s);
size_t srs_gtab_words();

// sigma_i of the tree fold (instance i's product of left-operand challenges).
hipError_t fold_sigmas(const uint32_t* gammas, uint32_t m, uint32_t* sigma, hipStream_t s);
// Gather component c of m instances (each k points) into a contiguous array.
hipError_t gather_component(const uint32_t* inst, uint32_t m, uint32_t k, uint32_t comp, uint32_t* out,
                            hipStream_t s);

// Exclusive scan of n u32 values; out has n + 1 entries (out[n] = total).
hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp, hipStream_t s);
size_t scan_tmp_words(uint32_t n);

}  // namespace zk
