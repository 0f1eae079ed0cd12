// Bucket accumulation of the multi-scalar multiplication (see msm.hip for
// the whole pipeline): the dominant kernel, kept in a file of its own so that
// its measured memory traffic is tied to exactly this code.
#include "msm.h"
#include "msm_store.h"

namespace zk {

namespace {

// The next gathered point travels straight to LDS (global_load_lds, no VGPRs
// held while it is in flight).  Each wave owns a 4 KiB stage: 16-byte chunk k
// of lane l's point lands at chunk k * 64 + l (the instruction writes its 64
// lanes' 16 bytes contiguously from the wave-uniform base it is given).
constexpr uint32_t STAGE_CHUNKS = MSM_NT / 64 * 4 * 64;

typedef __attribute__((address_space(3))) void lds_void;

__device__ __forceinline__ void stage_pt(const uint32_t* __restrict__ points, uint32_t v, uint4* wave_stage) {
  const uint4* src = reinterpret_cast<const uint4*>(points + (size_t)(v & 0x7fffffffu) * 16);
#pragma unroll
  for (int k = 0; k < 4; k++)
    __builtin_amdgcn_global_load_lds(src + k, (lds_void*)(wave_stage + k * 64), 16, 0, 0);
}

// s_waitcnt immediates (gfx9 encoding): vmcnt(0) alone, lgkmcnt(0) alone
constexpr int WAIT_VM0 = 0x0F70;
constexpr int WAIT_LGKM0 = 0xC07F;

__device__ __forceinline__ void st_rec_xyzz(uint32_t* rec, uint32_t key, uint32_t flag, const xyzz& a) {
  reinterpret_cast<uint4*>(rec)[0] = make_uint4(key, flag, 0, 0);
  st_xyzz(rec + 4, a);
}

// Each thread sums L consecutive sorted entries (L from the sorted total).  An entry is only its point
// index and sign; its bucket is the one whose offset range contains the
// entry's position (found once by binary search, then followed).  Runs of
// one bucket strictly inside the range are complete and go straight to HBM;
// the first and last run of the range become the thread's two records,
// finished by the record levels.  The next point is staged in LDS one step
// ahead, the entry after it two steps ahead.
__global__ void __launch_bounds__(MSM_NT) __attribute__((amdgpu_waves_per_eu(3, 3)))
accumulate_kernel(const uint32_t* __restrict__ entries, const uint32_t* __restrict__ offsets, uint32_t nbins,
                  const uint32_t* __restrict__ points, uint32_t lmin, uint32_t* __restrict__ buckets,
                  uint32_t* __restrict__ rec) {
  const uint64_t t = (uint64_t)blockIdx.x * MSM_NT + threadIdx.x;
  const uint32_t total = offsets[nbins];
  // slice length from the sorted total, which zero digits (skipped) can put
  // far below the n * W the grid was planned for: the real entries are spread
  // over the whole grid, at least lmin per thread
  const uint64_t nthreads = (uint64_t)gridDim.x * MSM_NT;
  uint64_t L = (total + nthreads - 1) / nthreads;
  if (L < lmin) L = lmin;
  const uint64_t tb = t * L;
  uint32_t* r0 = rec + (2 * t) * REC_WORDS;
  uint32_t* r1 = r0 + REC_WORDS;
  if (tb >= total) {
    st_rec_xyzz(r0, KEY_SENTINEL, 0, xyzz_inf());
    st_rec_xyzz(r1, KEY_SENTINEL, 0, xyzz_inf());
    return;
  }
  const uint32_t te = (uint32_t)min(tb + L, (uint64_t)total);
  // bucket of entry tb: the largest b with offsets[b] <= tb
  uint32_t lo = 0, hi = nbins;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= (uint32_t)tb) lo = mid; else hi = mid - 1;
  }
  uint32_t cur = lo;
  uint32_t bend = offsets[cur + 1];
  __shared__ uint4 stage[STAGE_CHUNKS];
  const uint32_t lane = threadIdx.x & 63;
  uint4* wave_stage = stage + (threadIdx.x >> 6) * 256;
  uint32_t v = entries[tb];
  uint32_t nv = tb + 1 < te ? entries[tb + 1] : v;
  stage_pt(points, v, wave_stage);
  bool first_done = false;
  xyzz acc = xyzz_inf();
  for (uint32_t e = (uint32_t)tb; e < te; e++) {
    if (e == bend) {
      if (!first_done) {
        st_rec_xyzz(r0, cur, 1, acc);
        first_done = true;
      } else {
        st_xyzz(buckets + (size_t)cur * XYZZ_WORDS, acc);
      }
      do {
        cur++;
        bend = offsets[cur + 1];
      } while (bend == e);
      acc = xyzz_inf();
    }
    // this entry's point, staged one entry ago
    __builtin_amdgcn_s_waitcnt(WAIT_VM0);
    uint32_t w[16];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const uint4 c = wave_stage[k * 64 + lane];
      w[4 * k] = c.x;
      w[4 * k + 1] = c.y;
      w[4 * k + 2] = c.z;
      w[4 * k + 3] = c.w;
    }
    // the stage is read before the next point overwrites it
    __builtin_amdgcn_s_waitcnt(WAIT_LGKM0);
    uint32_t nnv = nv;
    if (e + 1 < te) {
      stage_pt(points, nv, wave_stage);
      if (e + 2 < te) nnv = entries[e + 2];
    }
    uint32_t o = 0;
#pragma unroll
    for (int k = 0; k < 16; k++) o |= w[k];
    if (o) {
      aff pt;
      pt.x = unpack(w);
      pt.y = unpack(w + 8);
      acc = madd_signed(acc, pt, (v >> 31) != 0);
    }
    v = nv;
    nv = nnv;
  }
  if (!first_done) {
    st_rec_xyzz(r0, cur, 1, acc);
    st_rec_xyzz(r1, cur, 0, xyzz_inf());
  } else {
    st_rec_xyzz(r1, cur, 1, acc);
  }
}

}  // namespace

hipError_t msm_launch_accumulate(const MsmPlan& p, const MsmBuffers& b, const uint32_t* points, hipStream_t s) {
  hipLaunchKernelGGL(accumulate_kernel, dim3(p.acc_blocks), dim3(MSM_NT), 0, s, b.entries, b.offsets, p.nbins,
                     points, p.L, b.buckets, b.rec[0]);
  return hipGetLastError();
}

}  // namespace zk
