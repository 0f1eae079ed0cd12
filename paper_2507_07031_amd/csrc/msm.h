// Internal interface of the multi-scalar-multiplication kernels (msm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace zk {

constexpr uint32_t MSM_NT = 256;           // threads per workgroup
constexpr uint32_t MSM_SLOTS = 2 * MSM_NT; // records combined per workgroup
constexpr uint32_t KEY_SENTINEL = 0xfffffffeu;
constexpr uint32_t XYZZ_WORDS = 36;        // four 9-limb coordinates
constexpr uint32_t REC_WORDS = 40;         // key, flag, pad, pad, point (36): 160 bytes

// Geometry of one Pippenger run over one or several independent sums.
//  generic: one MSM over arbitrary (Montgomery) bases; one set of K buckets
//           per window, window sums Horner-combined at the end.
//  table:   `nseg` MSMs over one pre-shifted table (tab[w*tab_stride + i] =
//           2^(c w) P_i), every MSM with its own output.  Window w's digit of
//           s_i selects table point (w, i), so window sums are simply added
//           and all windows of an MSM share one set of K buckets (Wb = 1).
struct MsmPlan {
  uint32_t n;          // scalars in total (all segments)
  uint32_t c;          // window bits; digits are signed in [-2^(c-1), 2^(c-1)]
  uint32_t W;          // windows = ceil(254 / c)
  uint32_t K;          // buckets per bucket set = 2^(c-1)
  uint32_t table;      // 1: pre-shifted table layout
  uint32_t nseg;       // outputs: 1 (generic) or the number of MSMs (table)
  uint32_t Wb;         // bucket sets per output: W or 1
  uint32_t groups;     // nseg * Wb bucket sets
  uint32_t nbins;      // groups * K
  uint32_t tab_stride;
  uint32_t S;          // fine bits of the two-level sort: coarse bin = bin >> S
  uint32_t ncoarse;    // nbins >> S
  uint32_t chunk;      // scalars per coarse-sort item
  uint32_t nitems;     // items per window
  uint32_t L;          // least sorted entries per accumulating thread
  uint32_t acc_blocks; // accumulate workgroups
  uint32_t LB;         // buckets per chunk in the running-sum reduction
  uint32_t lgLB;       // log2 LB
  uint32_t J;          // chunks per bucket set = K / LB
  uint32_t nbits;      // log2 J: bit slices of the chunk index
  uint32_t parts;      // partial sums per bit slice
};

MsmPlan msm_plan_generic(uint32_t n, uint32_t c);
// offsets: nmsm + 1 scalar offsets (host), offsets[0] = 0.
MsmPlan msm_plan_table(const uint64_t* offsets, uint32_t nmsm, uint32_t c, uint32_t tab_stride);
uint32_t msm_default_c(uint32_t n);

// Scratch buffers of one run (device pointers), carved from one allocation.
struct MsmBuffers {
  uint2* pairs;        // W*n (entry, bin), sorted by coarse bin
  uint32_t* ccounts;   // ncoarse
  uint32_t* coff;      // ncoarse + 1
  uint32_t* ccursor;   // ncoarse
  uint32_t* counts;    // nbins
  uint32_t* offsets;   // nbins + 1
  uint32_t* cursor;    // nbins
  uint32_t* scan_tmp;  // scan block sums
  uint32_t* entries;   // W*n point index | sign << 31, sorted by bucket (ranges from offsets)
  uint32_t* buckets;   // nbins * 36
  uint32_t* rec[2];    // records (REC_WORDS each), ping-pong between levels
  uint32_t* vbuf;      // groups * J * 2 * 36: chunk totals S_j and weighted sums T_j
  uint32_t* partial;   // groups * (nbits + 1) * parts * 36: bit-slice partial sums
  uint32_t* wsum;      // groups * 36 (generic: window sums)
  uint32_t* seg_off;   // nseg + 1 (shared) / 2 (generic)
  uint4* items;        // nitems: (segment, first scalar, end scalar, 0)
};

size_t msm_workspace_bytes(const MsmPlan& p);
MsmBuffers msm_carve(const MsmPlan& p, void* base);

// Full pipeline.  Scalars: canonical, 8 words each, concatenated per segment.
// points: Montgomery affine (16 words each) -- the bases (generic) or the
// pre-shifted table (table layout).  offsets: host segment offsets (table),
// or nullptr (generic).  out: 16 words per output (nseg), canonical affine.
// after_accumulate: if not null, recorded on s right after the accumulation
// kernel (the rest of the run is latency-bound reduction; work that waits on
// this event can fill the idle compute units).  before_accumulate: if not
// null, s waits for it before the accumulation kernel (work overlapped with
// the sort then does not compete with the accumulation).
hipError_t msm_run(const MsmPlan& p, const uint64_t* offsets, const uint32_t* points, const uint32_t* scalars,
                   const MsmBuffers& b, uint32_t* out, hipStream_t s, hipEvent_t after_accumulate = nullptr,
                   hipEvent_t before_accumulate = nullptr);

// The bucket-accumulation kernel of msm_run (msm_accumulate.hip): sorted
// entries -> complete buckets and two boundary records per thread.
hipError_t msm_launch_accumulate(const MsmPlan& p, const MsmBuffers& b, const uint32_t* points, hipStream_t s);

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
// copy (if not null) receives out[0..n) as well.
hipError_t scan_exclusive(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* tmp, hipStream_t s,
                          uint32_t* copy = nullptr);
size_t scan_tmp_words(uint32_t n);

}  // namespace zk
