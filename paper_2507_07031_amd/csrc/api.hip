// C-ABI entry points (include/zk.h): argument checks, per-device tables,
// stream-ordered scratch, and the launch sequences of each operation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <initializer_list>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/zk.h"
#include "accum.h"
#include "device.h"
#include "field.h"
#include "g2msm.h"
#include "msm.h"
#include "msm_tiny.h"
#include "ntt.h"
#include "open.h"
#include "prof.h"
#include "quotient.h"
#include "setup.h"
#include "validate.h"

using namespace zk;

namespace {

thread_local std::string g_err;

zk_status fail(zk_status code, const std::string& msg) {
  g_err = msg;
  return code;
}

zk_status hip_fail(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? ZK_ENOMEM : ZK_EDEVICE,
              std::string(where) + ": " + hipGetErrorString(e));
}

// zk_set_validate: when on, calls check their Fr and G1 inputs on the device
// before any work and return ZK_EINVAL if one is out of range (the check
// waits for the stream: validated calls are synchronous).
std::atomic<bool> g_validate{false};

struct InputCheck {
  const void* p;
  uint64_t n;
  int kind;  // 0: Fr, 1: G1, 2: G2
};


#define ZK_HIP(call, where)                 \
  do {                                      \
    hipError_t _e = (call);                 \
    if (_e != hipSuccess) return hip_fail(_e, where); \
  } while (0)

// ---------------------------------------------------------------- device context
// Scratch of zk_msm_srs_noalloc: a fixed device array, one copy per GPU the
// library runs on, held until the process ends.  Host code never uses the
// array's name as a device address: ctx_get looks up each device's copy with
// hipGetSymbolAddress and the entry point passes that address to the kernels.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(128) << 20;
}  // namespace
static __device__ __align__(256) uint8_t scratch[NOALLOC_SCRATCH_BYTES];
namespace {

// Clears the validation finding word of a zk_msm_srs_noalloc call (a kernel
// rather than a memset, so the call's work stays capturable).
__global__ void noalloc_zero_kernel(uint32_t* w) {
  if (threadIdx.x == 0) w[0] = 0;
}

// Two-pass transforms of 2^13 .. 2^FULL_TW_MAX_LOG points read their first
// pass's four-step twiddles from per-size tables (36 B per point and
// direction: 0.6 GB per device in all) rather than forming each one by a
// Montgomery product of two split-table entries; three-pass transforms do
// the same in their second pass (B1), whose twiddles range over only 2^mB
// entries (2^16 .. 2^18: 52 MB for both directions and the four sizes).
constexpr uint32_t FULL_TW_MAX_LOG = 22;
constexpr uint32_t NTT_MAX_LOG = 28;
static_assert(NTT_MAX_LOG == ZK_MAX_LOG_NTT, "pass B1 tables cover every three-pass size");

// pass shapes of the three-pass form (the factors of ntt_prepare)
inline uint32_t three_pass_mA(uint32_t L) { return (L + 2) / 3; }
inline uint32_t three_pass_mB(uint32_t L) { return L - three_pass_mA(L); }
inline uint32_t three_pass_p2(uint32_t L) { return (three_pass_mB(L) + 1) / 2; }

struct DeviceCtx {
  bool ready = false;
  f29* tw[4] = {nullptr, nullptr, nullptr, nullptr};   // fwd lo, fwd hi, inv lo, inv hi
  f29* ladder[2] = {nullptr, nullptr};                  // in-tile twiddles, fwd / inv
  f29* coset5[2] = {nullptr, nullptr};                  // 5^e lo / hi
  f29* coset5inv[2] = {nullptr, nullptr};               // 5^-e lo / hi
  f29* ninv = nullptr;                                  // 2^-L, L = 0..28
  f29* tw_inv_n = nullptr;                              // inverse lo table times 2^-L, L = 13..28
  uint32_t* tw_full[2][FULL_TW_MAX_LOG + 1] = {};       // first-pass twiddles of two-pass transforms, fwd / inv
  uint32_t* tw_b1[2][NTT_MAX_LOG + 1] = {};              // pass B1 twiddles of three-pass transforms, fwd / inv
  uint32_t* gtab = nullptr;                             // 2^j G table for the setup
  uint8_t* noalloc = nullptr;                           // this device's copy of `scratch`
};

std::mutex g_mu;
DeviceCtx g_ctx[64];

void host_words(const f29& a, uint32_t w[8]) { pack(a, w); }

zk_status ctx_get(DeviceCtx** out) {
  int dev = 0;
  ZK_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ZK_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_mu);
  DeviceCtx& c = g_ctx[dev];
  if (c.ready) {
    *out = &c;
    return ZK_OK;
  }
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  ZK_HIP(ntt_pass_setup(), "ntt setup");
  const size_t tsz = sizeof(f29) << 14;
  for (int i = 0; i < 4; i++) ZK_HIP(hipMalloc(&c.tw[i], tsz), "hipMalloc(twiddles)");
  for (int i = 0; i < 2; i++) ZK_HIP(hipMalloc(&c.ladder[i], sizeof(f29) * ntt_ladder_entries()), "hipMalloc(ladder)");
  for (int i = 0; i < 2; i++) ZK_HIP(hipMalloc(&c.coset5[i], tsz), "hipMalloc(coset)");
  for (int i = 0; i < 2; i++) ZK_HIP(hipMalloc(&c.coset5inv[i], tsz), "hipMalloc(coset)");
  ZK_HIP(hipMalloc(&c.ninv, sizeof(f29) * 29), "hipMalloc(ninv)");
  ZK_HIP(hipMalloc(&c.gtab, srs_gtab_words() * 4), "hipMalloc(gtab)");
  // this device's copy of the no-allocation scratch (the device is current)
  ZK_HIP(hipGetSymbolAddress(reinterpret_cast<void**>(&c.noalloc), HIP_SYMBOL(scratch)),
         "hipGetSymbolAddress(scratch)");
  // roots omega_(2^28), its inverse, and the coset shift 5 (host arithmetic, same field code)
  Words8 wf, wi, w5;
  std::memcpy(wf.w, FR_OMEGA_2_28, 32);
  {
    const f29 w = reduce_full<FrP>(to_mont<FrP>(unpack(FR_OMEGA_2_28)));
    host_words(from_mont<FrP>(mont_inv<FrP>(w)), wi.w);
  }
  std::memset(w5.w, 0, 32);
  w5.w[0] = 5;
  ZK_HIP(ntt_make_pow_tables(wf, c.tw[0], c.tw[1], 0), "twiddle tables");
  ZK_HIP(ntt_make_pow_tables(wi, c.tw[2], c.tw[3], 0), "twiddle tables");
  ZK_HIP(ntt_make_ladder(c.tw[1], c.ladder[0], 0), "twiddle ladder");
  ZK_HIP(ntt_make_ladder(c.tw[3], c.ladder[1], 0), "twiddle ladder");
  ZK_HIP(ntt_make_pow_tables(w5, c.coset5[0], c.coset5[1], 0), "coset tables");
  {
    Words8 w5i;
    host_words(from_mont<FrP>(mont_inv<FrP>(reduce_full<FrP>(to_mont<FrP>(unpack(w5.w))))), w5i.w);
    ZK_HIP(ntt_make_pow_tables(w5i, c.coset5inv[0], c.coset5inv[1], 0), "coset tables");
  }
  // 2^-L in Montgomery form; 2^-1 = (r + 1) / 2
  f29 ninv[29];
  {
    uint32_t rp1[8], half[8];
    uint64_t acc = 1;
    for (int i = 0; i < 8; i++) {
      acc += FrP::M32[i];
      rp1[i] = (uint32_t)acc;
      acc >>= 32;
    }
    for (int i = 0; i < 8; i++) half[i] = (rp1[i] >> 1) | (i < 7 ? (rp1[i + 1] << 31) : 0u);
    const f29 h = reduce_full<FrP>(to_mont<FrP>(unpack(half)));
    ninv[0] = f29_from(FrP::ONE);
    for (int L = 1; L < 29; L++) ninv[L] = reduce_full<FrP>(mont_mul<FrP>(ninv[L - 1], h));
  }
  ZK_HIP(hipMemcpy(c.ninv, ninv, sizeof(ninv), hipMemcpyHostToDevice), "hipMemcpy");
  // multi-pass inverse transforms fold 2^-L into their first pass's twiddles
  ZK_HIP(hipMalloc(&c.tw_inv_n, tsz * (28 - ntt_tile_log())), "hipMalloc(scaled twiddles)");
  ZK_HIP(ntt_scale_tables(c.tw[2], c.ninv + ntt_tile_log() + 1, 28 - ntt_tile_log(), c.tw_inv_n, 0),
         "scaled twiddle tables");
  // first-pass twiddles of the two-pass sizes (pass A runs 2^(L/2)-point
  // transforms); the inverse ones carry 2^-L like tw_inv_n
  for (uint32_t L = ntt_tile_log() + 1; L <= FULL_TW_MAX_LOG; L++) {
    for (int d = 0; d < 2; d++) {
      ZK_HIP(hipMalloc(&c.tw_full[d][L], (size_t)36 << L), "hipMalloc(first-pass twiddles)");
      const f29* lo = d ? c.tw_inv_n + ((size_t)(L - ntt_tile_log() - 1) << 14) : c.tw[0];
      ZK_HIP(ntt_full_twiddles(lo, d ? c.tw[3] : c.tw[1], (uint32_t)d, L, L / 2, c.tw_full[d][L], 0),
             "first-pass twiddles");
    }
  }
  for (uint32_t L = 2 * ntt_tile_log() + 1; L <= NTT_MAX_LOG; L++) {
    const uint32_t mB = three_pass_mB(L);
    for (int d = 0; d < 2; d++) {
      ZK_HIP(hipMalloc(&c.tw_b1[d][L], (size_t)36 << mB), "hipMalloc(pass B1 twiddles)");
      ZK_HIP(ntt_full_twiddles(c.tw[2 * d], c.tw[2 * d + 1], 0, mB, three_pass_p2(L), c.tw_b1[d][L], 0),
             "pass B1 twiddles");
    }
  }
  ZK_HIP(hipDeviceSynchronize(), "table init");
  c.ready = true;
  *out = &c;
  return ZK_OK;
}

// ---------------------------------------------------------------- scratch
// Caching allocator for per-call scratch.  A freed block keeps its device
// memory and an event recorded on the stream that last used it; the next
// request that fits reuses it at once (same stream) or after making its
// stream wait on that event (another stream) -- no HIP allocation call on the
// hot path.  hipMalloc runs only when no cached block fits.
struct Block {
  void* p = nullptr;
  size_t size = 0;
  hipEvent_t done = nullptr;
  hipStream_t stream = nullptr;
  int device = 0;
};

std::mutex g_cache_mu;
std::vector<Block> g_free_blocks;
// Per device: scratch bytes the library holds (cached and in use), and the
// cap set by zk_set_scratch_budget (0: none).  Guarded by g_cache_mu.
uint64_t g_held[64] = {};
uint64_t g_budget[64] = {};

// Free this device's cached blocks (waiting for their last use); the caller
// holds no lock.
void drop_cached(int dev) {
  std::vector<Block> keep, drop;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (Block& b : g_free_blocks) (b.device == dev ? drop : keep).push_back(b);
    g_free_blocks.swap(keep);
  }
  for (Block& b : drop) {
    (void)hipEventSynchronize(b.done);
    (void)hipFree(b.p);
    (void)hipEventDestroy(b.done);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_held[dev] -= b.size;
  }
}

size_t round_up(size_t b) {
  const size_t g = b <= (size_t(1) << 20) ? 4096 : (size_t(2) << 20);
  return (b + g - 1) / g * g;
}

zk_status block_alloc(Block& out, size_t bytes, hipStream_t s) {
  int dev = 0;
  ZK_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ZK_EUNSUPPORTED, "device index out of range");
  bytes = round_up(bytes ? bytes : 256);
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    int best = -1;
    for (int i = 0; i < (int)g_free_blocks.size(); i++) {
      const Block& b = g_free_blocks[i];
      if (b.device != dev || b.size < bytes || b.size > bytes + bytes / 4) continue;
      if (best < 0 || b.size < g_free_blocks[best].size) best = i;
    }
    if (best >= 0) {
      out = g_free_blocks[best];
      g_free_blocks.erase(g_free_blocks.begin() + best);
    }
  }
  if (out.p) {
    if (out.stream != s) ZK_HIP(hipStreamWaitEvent(s, out.done, 0), "hipStreamWaitEvent(scratch)");
    out.stream = s;
    return ZK_OK;
  }
  static const bool log_alloc = std::getenv("ZK_LOG_ALLOC") != nullptr;
  if (log_alloc) {
    size_t cached = 0;
    {
      std::lock_guard<std::mutex> lk(g_cache_mu);
      for (const Block& b : g_free_blocks) cached += b.size;
    }
    std::fprintf(stderr, "[zk] scratch hipMalloc %zu bytes (cached %zu bytes in %zu blocks)\n", bytes, cached,
                 g_free_blocks.size());
  }
  // a budget counts cached blocks too: over it, drop the cache first
  auto over_budget = [&]() {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return g_budget[dev] != 0 && g_held[dev] + bytes > g_budget[dev];
  };
  if (over_budget()) {
    drop_cached(dev);
    if (over_budget()) {
      uint64_t held, cap;
      {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        held = g_held[dev];
        cap = g_budget[dev];
      }
      return fail(ZK_EBUDGET, "scratch of " + std::to_string(bytes) + " bytes exceeds the budget (" +
                                  std::to_string(held) + " of " + std::to_string(cap) + " bytes held)");
    }
  }
  hipError_t e = hipMalloc(&out.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    // drop cached blocks of this device and retry once
    drop_cached(dev);
    e = hipMalloc(&out.p, bytes);
    if (e != hipSuccess) {
      out.p = nullptr;
      (void)hipGetLastError();
      return fail(ZK_ENOMEM, "scratch allocation of " + std::to_string(bytes) + " bytes failed");
    }
  }
  out.size = bytes;
  out.device = dev;
  out.stream = s;
  {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    g_held[dev] += bytes;
  }
  ZK_HIP(hipEventCreateWithFlags(&out.done, hipEventDisableTiming), "hipEventCreate(scratch)");
  return ZK_OK;
}

void block_free(Block& b) {
  if (!b.p) return;
  (void)hipEventRecord(b.done, b.stream);
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_free_blocks.push_back(b);
  b.p = nullptr;
}

struct Scratch {
  Block blk;
  void* p = nullptr;
  ~Scratch() { block_free(blk); }
};

zk_status scratch_alloc(Scratch& sc, size_t bytes, hipStream_t s) {
  zk_status st = block_alloc(sc.blk, bytes, s);
  sc.p = sc.blk.p;
  return st;
}

// Input checks of one call.  Each validated call ORs its findings into a flag
// word of its own (a scratch block on its stream), so concurrent validated
// calls on other streams or threads neither clear nor read each other's.
zk_status check_inputs(DeviceCtx* c, hipStream_t s, std::initializer_list<InputCheck> checks, const char* who) {
  (void)c;
  if (!g_validate.load(std::memory_order_relaxed)) return ZK_OK;
  Scratch flag;
  zk_status st = scratch_alloc(flag, 256, s);
  if (st) return st;
  uint32_t* vflag = static_cast<uint32_t*>(flag.p);
  ZK_HIP(hipMemsetAsync(vflag, 0, 4, s), "hipMemsetAsync");
  for (const InputCheck& k : checks) {
    const uint32_t* w = static_cast<const uint32_t*>(k.p);
    ZK_HIP(k.kind == 2   ? validate_g2(w, k.n, vflag, s)
           : k.kind == 1 ? validate_g1(w, k.n, vflag, s)
                         : validate_fr(w, k.n, vflag, s),
           "input check");
  }
  uint32_t found = 0;
  ZK_HIP(hipMemcpyAsync(&found, vflag, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
  ZK_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (found & VALIDATE_FR) return fail(ZK_EINVAL, std::string(who) + ": an Fr input is not canonical (>= r)");
  if (found & VALIDATE_G1)
    return fail(ZK_EINVAL, std::string(who) + ": a G1 input is not (0, 0) or a canonical point on the curve");
  if (found & VALIDATE_G2)
    return fail(ZK_EINVAL, std::string(who) + ": a G2 input is not zero or a canonical point of order r on the twist");
  return ZK_OK;
}


// ---------------------------------------------------------------- NTT driver
// A transform of 2^L points: one LDS pass up to the tile size, two four-step
// passes through a scratch buffer up to the square of the tile size, else
// three (the second factor split once more; its intermediate lives in the
// output buffer, which every transform of the last pass reads and rewrites
// at the same positions).  Prepared first, then launched pass by pass, so a
// caller can interleave the passes with other work.
struct NttRun {
  NttPass a{}, b{}, c{};
  int passes = 1;
  Scratch tmp;  // intermediate of the two- and three-pass forms
};

// Leading stages a pass with input stride s_in over transforms of 2^m points
// can skip: with valid_n = 2^v s_in, the input indices below valid_n are
// exactly the first 2^v points of every transform (its batch index is below
// s_in), so the other 2^m - 2^v are zero padding.
static uint32_t ntt_zero_log(uint32_t valid_n, uint32_t s_in, uint32_t m) {
  if (valid_n == 0 || valid_n % s_in) return 0;
  const uint32_t V = valid_n / s_in;
  if (V & (V - 1)) return 0;
  const uint32_t v = 31 - __builtin_clz(V);
  return v < m ? m - v : 0;
}

zk_status ntt_prepare(DeviceCtx* c, const uint32_t* in, uint32_t* out, uint32_t L, bool inverse, const f29* pre_lo,
                      const f29* pre_hi, uint32_t valid_n, hipStream_t s, NttRun& r, bool overlapped = false) {
  const uint32_t T = ntt_tile_log();
  const Schedule sched = device_schedule();
  r.a.unit_log = r.b.unit_log = r.c.unit_log = sched.ntt_unit_log;
  const f29* lo = inverse ? c->tw[2] : c->tw[0];
  const f29* hi = inverse ? c->tw[3] : c->tw[1];
  const f29* scale = inverse ? c->ninv + L : nullptr;
  const f29* ladder = inverse ? c->ladder[1] : c->ladder[0];
  if (L <= T) {
    NttPass& p = r.a;
    p.in = in;
    p.out = out;
    p.m = L;
    p.G = 1;
    p.nbatch = 1;
    p.s_in = 1;
    p.s_out = 1;
    p.b_out = 1u << L;
    p.valid_n = valid_n;
    p.tw_lo = lo;
    p.tw_hi = hi;
    p.ladder = ladder;
    p.pre_lo = pre_lo;
    p.pre_hi = pre_hi;
    p.post_scale = scale;
    p.zero_log = ntt_zero_log(valid_n, 1, L);
    r.passes = 1;
    return ZK_OK;
  }
  const bool three = L > 2 * T;
  // pass A transforms have 2^mA points; above 2^(2T) the three factors are
  // near-equal (mA >= mB1 >= mB2), so pass A's workgroups hold several
  // transforms and its strided reads move more than one element at a time
  const uint32_t mA = three ? three_pass_mA(L) : L / 2, mB = L - mA;
  const uint32_t N1 = 1u << mB, N2 = 1u << mA;
  // the schedule's preferred tile (2^10, 2^11 or 2^12 points: four, two or
  // one workgroups per CU) where both passes' transforms fit it, else the
  // smallest that holds them; a transform that runs beside other kernels
  // (overlapped) has its own preference: a 4096-point tile's 144 KB of LDS
  // leaves a compute unit no room for the other kernels' workgroups
  const uint32_t pref = overlapped ? sched.ntt_overlap_tile_log : sched.ntt_tile_log;
  // above 2^(2T), pass B's factor splits into P1 * P2 transforms of 2^p1 and
  // 2^p2 points (p2 = ceil(mB / 2)); every pass's transforms must fit the tile
  const uint32_t need = three ? std::max(mA, (mB + 1) / 2) : mB;
  const uint32_t tile = 1u << std::max(need, std::min(pref, T));
  zk_status st = scratch_alloc(r.tmp, (size_t)32 << L, s);
  if (st) return st;
  uint32_t* Y = static_cast<uint32_t*>(r.tmp.p);
  NttPass& a = r.a;
  a.in = in;
  a.out = Y;
  a.m = mA;
  a.nbatch = N1;
  a.G = std::min(tile / N2, N1);
  a.s_in = N1;
  a.s_out = 1;
  a.b_out = N2;
  a.valid_n = valid_n;
  a.tw_lo = lo;
  a.tw_hi = hi;
  a.ladder = ladder;
  a.post_tw_L = L;
  a.pre_lo = pre_lo;
  a.pre_hi = pre_hi;
  a.zero_log = ntt_zero_log(valid_n, N1, mA);
  // an inverse transform's 2^-L rides on pass A's four-step twiddles (a lo
  // table scaled by it), so no pass multiplies by it on its own
  if (inverse) {
    a.tw_lo = c->tw_inv_n + ((size_t)(L - T - 1) << 14);
    a.tw_scaled = 1;
  }
  // tables built for pass A of the two-pass form (mA = L / 2)
  a.tw_full = (!three && L <= FULL_TW_MAX_LOG) ? c->tw_full[inverse ? 1 : 0][L] : nullptr;
  NttPass& b = r.b;
  b.in = Y;
  b.out = out;
  b.m = mB;
  b.nbatch = N2;
  b.G = std::min(tile / N1, N2);
  b.s_in = N2;
  b.s_out = N2;
  b.b_out = 1;
  b.valid_n = 1u << L;
  b.tw_lo = lo;
  b.tw_hi = hi;
  b.ladder = ladder;
  r.passes = 2;
  if (!three) return ZK_OK;
  // pass B of N1 = P1 * P2 points, i1 = j1 + P1 j2: B1 runs the P2-point
  // transforms over j2 (batch k2 + N2 j1), B2 the P1-point ones over j1
  // (batch k2 + N2 k1'); see the pass equations at the top of ntt.hip
  const uint32_t p2 = three_pass_p2(L), p1 = mB - p2;
  const uint32_t P1 = 1u << p1, P2 = 1u << p2;
  b.out = out;
  b.m = p2;
  b.nbatch = N2 * P1;
  b.G = std::min(tile / P2, b.nbatch);
  b.s_in = N2 * P1;
  b.s_out = N2;
  b.b_out = 1;
  b.b_hi_log = mA;
  b.b_out_hi = N2 * P2;
  b.post_tw_L = mB;
  b.tw_shift = mA;
  b.post_scale = nullptr;
  b.tw_full = L <= NTT_MAX_LOG ? c->tw_b1[inverse ? 1 : 0][L] : nullptr;
  NttPass& c3 = r.c;
  c3.in = out;
  c3.out = out;
  c3.m = p1;
  c3.nbatch = N2 * P2;
  c3.G = std::min(tile / P1, c3.nbatch);
  c3.s_in = N2 * P2;
  c3.s_out = N2 * P2;
  c3.b_out = 1;
  c3.valid_n = 1u << L;
  c3.tw_lo = lo;
  c3.tw_hi = hi;
  c3.ladder = ladder;
  r.passes = 3;
  return ZK_OK;
}

zk_status ntt_first(NttRun& r, hipStream_t s) {
  ZK_HIP(ntt_launch_pass(r.a, s), "ntt pass");
  return ZK_OK;
}

zk_status ntt_second(NttRun& r, hipStream_t s) {
  if (r.passes >= 2) ZK_HIP(ntt_launch_pass(r.b, s), "ntt pass B");
  if (r.passes >= 3) ZK_HIP(ntt_launch_pass(r.c, s), "ntt pass B2");
  return ZK_OK;
}

zk_status run_ntt(DeviceCtx* c, const uint32_t* in, uint32_t* out, uint32_t L, bool inverse, const f29* pre_lo,
                  const f29* pre_hi, uint32_t valid_n, hipStream_t s) {
  NttRun r;
  zk_status st = ntt_prepare(c, in, out, L, inverse, pre_lo, pre_hi, valid_n, s, r);
  if (!st) st = ntt_first(r, s);
  if (!st) st = ntt_second(r, s);
  return st;
}

// ---------------------------------------------------------------- MSM driver
zk_status run_msm(const MsmPlan& plan, const uint64_t* offsets, const uint32_t* mont_points, const uint32_t* scalars,
                  uint32_t* out, hipStream_t s, hipEvent_t after_accumulate = nullptr,
                  hipEvent_t before_accumulate = nullptr) {
  Scratch ws;
  zk_status st = scratch_alloc(ws, msm_workspace_bytes(plan), s);
  if (st) return st;
  const MsmBuffers b = msm_carve(plan, ws.p);
  ZK_HIP(msm_run(plan, offsets, mont_points, scalars, b, out, s, after_accumulate, before_accumulate), "msm");
  return ZK_OK;
}

// Companion stream of a caller stream (one each, default priority), for work
// the library overlaps with the caller's; and a pool of sync-only events.
std::mutex g_side_mu;
std::map<std::pair<int, hipStream_t>, hipStream_t> g_side;
std::vector<hipEvent_t> g_sync_events;

zk_status side_stream(hipStream_t caller, hipStream_t* out) {
  int dev = 0;
  ZK_HIP(hipGetDevice(&dev), "hipGetDevice");
  std::lock_guard<std::mutex> lk(g_side_mu);
  auto it = g_side.find({dev, caller});
  if (it != g_side.end()) {
    *out = it->second;
    return ZK_OK;
  }
  hipStream_t s2 = nullptr;
  ZK_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking), "hipStreamCreateWithFlags");
  g_side[{dev, caller}] = s2;
  *out = s2;
  return ZK_OK;
}

struct SyncEvents {
  hipEvent_t e[2] = {nullptr, nullptr};
  ~SyncEvents() {
    std::lock_guard<std::mutex> lk(g_side_mu);
    for (hipEvent_t x : e)
      if (x) g_sync_events.push_back(x);
  }
};

zk_status sync_events(SyncEvents& ev) {
  for (hipEvent_t& x : ev.e) {
    {
      std::lock_guard<std::mutex> lk(g_side_mu);
      if (!g_sync_events.empty()) {
        x = g_sync_events.back();
        g_sync_events.pop_back();
        continue;
      }
    }
    ZK_HIP(hipEventCreateWithFlags(&x, hipEventDisableTiming), "hipEventCreateWithFlags");
  }
  return ZK_OK;
}

constexpr uint32_t SRS_C = 16;                 // window bits of the main table
constexpr uint32_t SRS_C_SMALL = 12;           // window bits of the small-MSM table
constexpr uint32_t SRS_SMALL_MAX = 1u << 16;   // points covered by the small table
constexpr uint32_t SRS_C_LARGE = 20;           // window bits of the large-MSM table
constexpr uint64_t SRS_LARGE_MIN = 1ull << 21; // MSMs from this size use the large table
// Default table policy, as the autotuner measured it on MI355X: the 16-bit
// table beats the 8-bit one at every size from 2^10 (its reduction tail is no
// longer the bottleneck), so the 8-bit table serves no size unless a policy
// asks for it; the 20-bit table wins from 2^21.
constexpr uint64_t SRS_SMALL_POLICY = 0;
// Commitments of at most this many points run on the small-multiples table
// (msm_tiny.hip) by default.
constexpr uint64_t SRS_TINY_POLICY = TINY_MAX;

}  // namespace

struct zk_srs {
  int device;
  uint64_t n;
  uint32_t c;
  uint32_t W;
  uint32_t* tab;        // W * n Montgomery affine points, row w = 2^(c w) P_i; row 0 = the points
  uint64_t n_small;     // min(n, SRS_SMALL_MAX)
  uint32_t c_small;
  uint32_t W_small;
  uint32_t* tab_small;  // W_small * n_small points for small MSMs
  uint32_t c_large;
  uint32_t W_large;
  uint32_t* tab_large;  // W_large * n points for large MSMs (n >= SRS_LARGE_MIN only)
  uint64_t small_max;   // table policy: n < small_max -> small table,
  uint64_t large_min;   //               n >= large_min -> large table (if built), else main
  uint32_t n_tiny;      // min(n, TINY_MAX)
  uint32_t* tab_tiny;   // m 16^w P_i, m = 1..8, w < 64, i < n_tiny (msm_tiny.hip)
  uint64_t tiny_max;    // policy: 0 < n <= tiny_max -> the small-multiples run
};

struct zk_srs_g2 {
  int device;
  uint64_t n;
  uint32_t* tab;  // G2_W * n Montgomery affine points, row w = 2^(8 w) P_i
};

extern "C" {

const char* zk_last_error(void) { return g_err.c_str(); }

zk_status zk_release_cached_memory(void) {
  int dev = 0;
  ZK_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ZK_EUNSUPPORTED, "device index out of range");
  drop_cached(dev);
  return ZK_OK;
}

zk_status zk_set_scratch_budget(uint64_t bytes) {
  int dev = 0;
  ZK_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev < 0 || dev >= 64) return fail(ZK_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lk(g_cache_mu);
  g_budget[dev] = bytes;
  return ZK_OK;
}

uint64_t zk_scratch_held(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return 0;
  }
  std::lock_guard<std::mutex> lk(g_cache_mu);
  return g_held[dev];
}

zk_status zk_set_schedule(const zk_schedule* sch) {
  const int dev = schedule_device();
  if (dev < 0) return fail(ZK_EDEVICE, "zk_set_schedule: no device");
  Schedule v;
  if (sch) {
    auto pow2 = [](uint32_t x) { return x && !(x & (x - 1)); };
    if (sch->acc_max_slice) {
      if (sch->acc_max_slice < 16 || sch->acc_max_slice > 4096)
        return fail(ZK_EINVAL, "zk_set_schedule: acc_max_slice must be 16..4096");
      v.acc_max_slice = sch->acc_max_slice;
    }
    if (sch->acc_blocks_per_cu) {
      if (sch->acc_blocks_per_cu > 4) return fail(ZK_EINVAL, "zk_set_schedule: acc_blocks_per_cu must be 1..4");
      v.acc_blocks_per_cu = sch->acc_blocks_per_cu;
    }
    if (sch->reduce_chunk) {
      if (!pow2(sch->reduce_chunk) || sch->reduce_chunk > 64)
        return fail(ZK_EINVAL, "zk_set_schedule: reduce_chunk must be a power of two <= 64");
      v.reduce_chunk = sch->reduce_chunk;
    }
    if (sch->sort_chunk) {
      if (!pow2(sch->sort_chunk) || sch->sort_chunk < 256 || sch->sort_chunk > 16384)
        return fail(ZK_EINVAL, "zk_set_schedule: sort_chunk must be a power of two in 256..16384");
      v.sort_chunk = sch->sort_chunk;
    }
    if (sch->sort_bin_entries) {
      if (!pow2(sch->sort_bin_entries) || sch->sort_bin_entries < (1u << 10) || sch->sort_bin_entries > (1u << 20))
        return fail(ZK_EINVAL, "zk_set_schedule: sort_bin_entries must be a power of two in 2^10..2^20");
      v.sort_bin_entries = sch->sort_bin_entries;
    }
    if (sch->ntt_tile_log) {
      if (sch->ntt_tile_log < 10 || sch->ntt_tile_log > 12)
        return fail(ZK_EINVAL, "zk_set_schedule: ntt_tile_log must be 10, 11 or 12");
      v.ntt_tile_log = sch->ntt_tile_log;
    }
    if (sch->ntt_overlap_tile_log) {
      if (sch->ntt_overlap_tile_log < 10 || sch->ntt_overlap_tile_log > 12)
        return fail(ZK_EINVAL, "zk_set_schedule: ntt_overlap_tile_log must be 10, 11 or 12");
      v.ntt_overlap_tile_log = sch->ntt_overlap_tile_log;
    }
    if (sch->ntt_unit_log) {
      if (sch->ntt_unit_log != 2 && sch->ntt_unit_log != 3)
        return fail(ZK_EINVAL, "zk_set_schedule: ntt_unit_log must be 2 or 3");
      v.ntt_unit_log = sch->ntt_unit_log;
    }
  }
  schedule_slots()[dev] = v;
  return ZK_OK;
}

zk_status zk_get_schedule(zk_schedule* sch) {
  if (!sch) return fail(ZK_EINVAL, "zk_get_schedule: NULL argument");
  const Schedule v = device_schedule();
  sch->acc_max_slice = v.acc_max_slice;
  sch->acc_blocks_per_cu = v.acc_blocks_per_cu;
  sch->reduce_chunk = v.reduce_chunk;
  sch->sort_chunk = v.sort_chunk;
  sch->sort_bin_entries = v.sort_bin_entries;
  sch->ntt_tile_log = v.ntt_tile_log;
  sch->ntt_unit_log = v.ntt_unit_log;
  sch->ntt_overlap_tile_log = v.ntt_overlap_tile_log;
  return ZK_OK;
}

zk_status zk_set_validate(int on) {
  g_validate.store(on != 0);
  return ZK_OK;
}

zk_status zk_profile_enable(int on) {
  prof_set_enabled(on != 0);
  return ZK_OK;
}

zk_status zk_profile_only(const char* region) {
  prof_set_filter(region);
  return ZK_OK;
}

zk_status zk_profile_read(const char* region, double* total_ms, uint64_t* launches, int reset) {
  if (!region || !total_ms || !launches) return fail(ZK_EINVAL, "zk_profile_read: NULL argument");
  unsigned long long n = 0;
  if (prof_read(region, total_ms, &n, reset != 0) != 0) return fail(ZK_EDEVICE, "zk_profile_read: event error");
  *launches = n;
  return ZK_OK;
}

zk_status zk_ntt(const zk_fr* in, zk_fr* out, uint32_t log_n, void* stream) {
  if (!in || !out) return fail(ZK_EINVAL, "zk_ntt: NULL buffer");
  if (log_n > ZK_MAX_LOG_NTT) return fail(ZK_EUNSUPPORTED, "zk_ntt: log_n > ZK_MAX_LOG_NTT");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if ((st = check_inputs(c, (hipStream_t)stream, {{in, 1ull << log_n, false}}, "zk_ntt"))) return st;
  return run_ntt(c, reinterpret_cast<const uint32_t*>(in), reinterpret_cast<uint32_t*>(out), log_n, false,
                 nullptr, nullptr, 1u << log_n, (hipStream_t)stream);
}

zk_status zk_intt(const zk_fr* in, zk_fr* out, uint32_t log_n, void* stream) {
  if (!in || !out) return fail(ZK_EINVAL, "zk_intt: NULL buffer");
  if (log_n > ZK_MAX_LOG_NTT) return fail(ZK_EUNSUPPORTED, "zk_intt: log_n > ZK_MAX_LOG_NTT");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if ((st = check_inputs(c, (hipStream_t)stream, {{in, 1ull << log_n, false}}, "zk_intt"))) return st;
  return run_ntt(c, reinterpret_cast<const uint32_t*>(in), reinterpret_cast<uint32_t*>(out), log_n, true,
                 nullptr, nullptr, 1u << log_n, (hipStream_t)stream);
}

zk_status zk_coset_ntt(const zk_fr* coeffs, uint32_t log_n, uint32_t log_blowup, const zk_fr* shift_host,
                       zk_fr* out, void* stream) {
  if (!coeffs || !out) return fail(ZK_EINVAL, "zk_coset_ntt: NULL buffer");
  if (log_n + log_blowup > ZK_MAX_LOG_NTT || log_n > ZK_MAX_LOG_NTT || log_blowup > ZK_MAX_LOG_NTT)
    return fail(ZK_EUNSUPPORTED, "zk_coset_ntt: log_n + log_blowup > ZK_MAX_LOG_NTT");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{coeffs, 1ull << log_n, false}}, "zk_coset_ntt"))) return st;
  const f29* lo = c->coset5[0];
  const f29* hi = c->coset5[1];
  Scratch tab;
  if (shift_host) {
    // canonical check, then tables of shift^e in scratch
    uint32_t w[8];
    std::memcpy(w, shift_host->v, 32);
    unsigned br = 0;
    for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], FrP::M32[i], br, &br);
    if (!br) return fail(ZK_EINVAL, "zk_coset_ntt: shift not canonical (>= r)");
    const size_t tsz = sizeof(f29) << 14;
    st = scratch_alloc(tab, 2 * tsz, s);
    if (st) return st;
    char* base = static_cast<char*>(tab.p);
    Words8 sw;
    std::memcpy(sw.w, w, 32);
    ZK_HIP(ntt_make_pow_tables(sw, reinterpret_cast<f29*>(base), reinterpret_cast<f29*>(base + tsz), s),
           "shift tables");
    lo = reinterpret_cast<const f29*>(base);
    hi = reinterpret_cast<const f29*>(base + tsz);
  }
  return run_ntt(c, reinterpret_cast<const uint32_t*>(coeffs), reinterpret_cast<uint32_t*>(out),
                 log_n + log_blowup, false, lo, hi, 1u << log_n, s);
}

zk_status zk_msm(const zk_g1* bases, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream) {
  if (!out || (n && (!bases || !scalars))) return fail(ZK_EINVAL, "zk_msm: NULL buffer");
  if (n >= (1ull << 31) / 16) return fail(ZK_EUNSUPPORTED, "zk_msm: n too large");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{bases, n, true}, {scalars, n, false}}, "zk_msm"))) return st;
  const MsmPlan plan = msm_plan_generic((uint32_t)n, msm_default_c((uint32_t)n));
  Scratch pts;
  st = scratch_alloc(pts, (size_t)n * 64, s);
  if (st) return st;
  uint32_t* mont = static_cast<uint32_t*>(pts.p);
  ZK_HIP(msm_points_to_mont(reinterpret_cast<const uint32_t*>(bases), mont, n, s), "to_mont");
  return run_msm(plan, nullptr, mont, reinterpret_cast<const uint32_t*>(scalars), reinterpret_cast<uint32_t*>(out),
                 s);
}

zk_status zk_srs_setup(const zk_fr* tau_host, uint64_t n, zk_g1* out, void* stream) {
  if (!tau_host || (n && !out)) return fail(ZK_EINVAL, "zk_srs_setup: NULL argument");
  uint32_t w[8];
  std::memcpy(w, tau_host->v, 32);
  unsigned br = 0;
  for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], FrP::M32[i], br, &br);
  if (!br) return fail(ZK_EINVAL, "zk_srs_setup: tau not canonical (>= r)");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  Tau8 t;
  std::memcpy(t.w, w, 32);
  ZK_HIP(srs_from_tau(t, reinterpret_cast<uint32_t*>(out), n, c->gtab, (hipStream_t)stream), "srs setup");
  return ZK_OK;
}

zk_status zk_srs_lagrange_setup(const zk_fr* tau_host, uint32_t log_n, zk_g1* out, void* stream) {
  if (!tau_host || !out) return fail(ZK_EINVAL, "zk_srs_lagrange_setup: NULL argument");
  if (log_n > ZK_MAX_LOG_NTT) return fail(ZK_EUNSUPPORTED, "zk_srs_lagrange_setup: log_n > ZK_MAX_LOG_NTT");
  uint32_t w[8];
  std::memcpy(w, tau_host->v, 32);
  unsigned br = 0;
  for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], FrP::M32[i], br, &br);
  if (!br) return fail(ZK_EINVAL, "zk_srs_lagrange_setup: tau not canonical (>= r)");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  // c = (tau^n - 1) / n; tau^n = 1 exactly when tau lies in H
  const f29 one = f29_from(FrP::ONE);
  f29 tn = reduce_full<FrP>(to_mont<FrP>(unpack(w)));
  for (uint32_t i = 0; i < log_n; i++) tn = reduce_full<FrP>(mont_mul<FrP>(tn, tn));
  const f29 num = reduce_full<FrP>(sub_k(tn, one, FrP::K2));
  const bool in_h = f29_is_zero_limbs(num);
  uint32_t nw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  nw[log_n >> 5] = 1u << (log_n & 31);
  const f29 ninv = mont_inv<FrP>(reduce_full<FrP>(to_mont<FrP>(unpack(nw))));
  const f29 cm = in_h ? f29_zero() : reduce_full<FrP>(mont_mul<FrP>(num, ninv));
  Tau8 t;
  std::memcpy(t.w, w, 32);
  ZK_HIP(srs_lagrange_from_tau(t, log_n, cm, in_h, c->tw[0], c->tw[1], reinterpret_cast<uint32_t*>(out), c->gtab,
                               (hipStream_t)stream),
         "lagrange setup");
  return ZK_OK;
}

zk_status zk_srs_create(const zk_g1* points, uint64_t n, zk_srs** srs, void* stream) {
  if (!srs || (n && !points)) return fail(ZK_EINVAL, "zk_srs_create: NULL argument");
  if (n >= (1ull << 31) / 16) return fail(ZK_EUNSUPPORTED, "zk_srs_create: n too large");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if ((st = check_inputs(c, (hipStream_t)stream, {{points, n, true}}, "zk_srs_create"))) return st;
  zk_srs* h = new zk_srs();
  ZK_HIP(hipGetDevice(&h->device), "hipGetDevice");
  h->n = n;
  h->c = SRS_C;
  h->W = (254 + SRS_C - 1) / SRS_C;
  h->tab = nullptr;
  h->n_small = std::min<uint64_t>(n, SRS_SMALL_MAX);
  h->c_small = SRS_C_SMALL;
  h->W_small = (254 + SRS_C_SMALL - 1) / SRS_C_SMALL;
  h->tab_small = nullptr;
  h->c_large = SRS_C_LARGE;
  h->W_large = (254 + SRS_C_LARGE - 1) / SRS_C_LARGE;
  h->tab_large = nullptr;
  h->small_max = SRS_SMALL_POLICY;
  h->large_min = SRS_LARGE_MIN;
  h->n_tiny = (uint32_t)std::min<uint64_t>(n, TINY_MAX);
  h->tab_tiny = nullptr;
  h->tiny_max = SRS_TINY_POLICY;
  if (n) {
    const uint32_t* pts = reinterpret_cast<const uint32_t*>(points);
    hipError_t e = hipMalloc(&h->tab, (size_t)h->W * n * 64);
    if (e == hipSuccess) e = hipMalloc(&h->tab_small, (size_t)h->W_small * h->n_small * 64);
    if (e == hipSuccess && n >= SRS_LARGE_MIN) e = hipMalloc(&h->tab_large, (size_t)h->W_large * n * 64);
    if (e == hipSuccess) e = hipMalloc(&h->tab_tiny, (size_t)msm_tiny_table_points(h->n_tiny) * 64);
    if (e == hipSuccess) e = msm_build_table(pts, h->tab, n, h->c, h->W, (hipStream_t)stream);
    if (e == hipSuccess) e = msm_build_tiny_table(h->tab, h->c, h->W, n, h->n_tiny, h->tab_tiny, (hipStream_t)stream);
    if (e == hipSuccess)
      e = msm_build_table(pts, h->tab_small, h->n_small, h->c_small, h->W_small, (hipStream_t)stream);
    if (e == hipSuccess && h->tab_large)
      e = msm_build_table(pts, h->tab_large, n, h->c_large, h->W_large, (hipStream_t)stream);
    if (e != hipSuccess) {
      if (h->tab) (void)hipFree(h->tab);
      if (h->tab_small) (void)hipFree(h->tab_small);
      if (h->tab_large) (void)hipFree(h->tab_large);
      if (h->tab_tiny) (void)hipFree(h->tab_tiny);
      delete h;
      return hip_fail(e, "zk_srs_create: table build");
    }
  }
  *srs = h;
  return ZK_OK;
}

zk_status zk_srs_destroy(zk_srs* srs) {
  if (!srs) return ZK_OK;
  if (srs->tab) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srs->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(srs->tab);
    if (srs->tab_small) (void)hipFree(srs->tab_small);
    if (srs->tab_large) (void)hipFree(srs->tab_large);
    if (srs->tab_tiny) (void)hipFree(srs->tab_tiny);
    (void)hipSetDevice(prev);
  }
  delete srs;
  return ZK_OK;
}

uint64_t zk_srs_size(const zk_srs* srs) { return srs ? srs->n : 0; }

// One commitment picks a pre-shifted table by size, by the SRS's policy:
// 12-bit windows below small_max points (2048 buckets: a short reduction,
// for 22 windows instead of 16), 20-bit windows from large_min (13 windows:
// fewer additions, for 16x the buckets), 16-bit windows between.  Every window of
// the MSM shares one bucket set.
enum class SrsTable { small, main, large };

static SrsTable srs_table_for(const zk_srs* srs, uint64_t n) {
  const uint64_t small_max = srs ? srs->small_max : SRS_SMALL_POLICY;
  const uint64_t large_min = srs ? srs->large_min : SRS_LARGE_MIN;
  if (n < small_max) return SrsTable::small;
  if (n >= large_min && (!srs || srs->tab_large)) return SrsTable::large;
  return SrsTable::main;
}

static MsmPlan srs_plan(const zk_srs* srs, uint64_t n, const uint64_t off[2]) {
  const uint32_t stride = srs ? (uint32_t)srs->n : (uint32_t)n;
  switch (srs_table_for(srs, n)) {
    case SrsTable::small:
      return msm_plan_table(off, 1, SRS_C_SMALL, srs ? (uint32_t)srs->n_small : (uint32_t)n);
    case SrsTable::large:
      return msm_plan_table(off, 1, SRS_C_LARGE, stride);
    default:
      return msm_plan_table(off, 1, SRS_C, stride);
  }
}

// Does an n-point commitment run on the small-multiples table?
static bool srs_uses_tiny(const zk_srs* srs, uint64_t n) {
  return srs && srs->tab_tiny && n > 0 && n <= srs->tiny_max && n <= srs->n_tiny;
}

static zk_status msm_srs_one(const zk_srs* srs, const uint32_t* scalars, uint64_t n, uint32_t* out16,
                             hipStream_t s, hipEvent_t after_accumulate = nullptr,
                             hipEvent_t before_accumulate = nullptr) {
  if (srs_uses_tiny(srs, n)) {
    Scratch ws;
    zk_status st = scratch_alloc(ws, msm_tiny_workspace_bytes((uint32_t)n), s);
    if (st) return st;
    if (before_accumulate) ZK_HIP(hipStreamWaitEvent(s, before_accumulate, 0), "hipStreamWaitEvent");
    ZK_HIP(msm_tiny_run(srs->tab_tiny, srs->n_tiny, scalars, (uint32_t)n, ws.p, out16, s, after_accumulate),
           "msm (small multiples)");
    return ZK_OK;
  }
  const uint64_t off[2] = {0, n};
  const MsmPlan plan = srs_plan(srs, n, off);
  const SrsTable t = srs_table_for(srs, n);
  const uint32_t* tab = t == SrsTable::small ? srs->tab_small : t == SrsTable::large ? srs->tab_large : srs->tab;
  return run_msm(plan, off, tab, scalars, out16, s, after_accumulate, before_accumulate);
}

zk_status zk_srs_set_table_policy(zk_srs* srs, uint64_t small_max, uint64_t large_min) {
  if (!srs) return fail(ZK_EINVAL, "zk_srs_set_table_policy: NULL srs");
  if (small_max > SRS_SMALL_MAX) return fail(ZK_EINVAL, "zk_srs_set_table_policy: small_max above 2^16");
  srs->small_max = small_max;
  srs->large_min = large_min;
  return ZK_OK;
}

zk_status zk_srs_set_tiny_max(zk_srs* srs, uint64_t tiny_max) {
  if (!srs) return fail(ZK_EINVAL, "zk_srs_set_tiny_max: NULL srs");
  if (tiny_max > TINY_MAX) return fail(ZK_EINVAL, "zk_srs_set_tiny_max: tiny_max above 4096");
  srs->tiny_max = tiny_max;
  return ZK_OK;
}

uint32_t zk_srs_window_bits(const zk_srs* srs, uint64_t n) {
  if (!srs || n > srs->n) return 0;
  if (srs_uses_tiny(srs, n)) return 4;
  switch (srs_table_for(srs, n)) {
    case SrsTable::small: return SRS_C_SMALL;
    case SrsTable::large: return SRS_C_LARGE;
    default: return SRS_C;
  }
}

uint64_t zk_msm_srs_workspace_bytes(const zk_srs* srs, uint64_t n) {
  if (n >= (1ull << 31) / 16) return 0;
  if (srs_uses_tiny(srs, n)) return msm_tiny_workspace_bytes((uint32_t)n);
  const uint64_t off[2] = {0, n};
  return msm_workspace_bytes(srs_plan(srs, n, off));
}

uint64_t zk_ntt_workspace_bytes(uint32_t log_n) {
  if (log_n > ZK_MAX_LOG_NTT) return 0;
  return log_n <= ntt_tile_log() ? 0 : ((uint64_t)32 << log_n);
}

zk_status zk_commit_job(const zk_srs* srs, const zk_fr* evals, uint32_t log_n, uint32_t log_blowup,
                        const zk_fr* shift_host, zk_fr* coeffs, zk_g1* commitment, zk_fr* coset, void* stream) {
  if (!srs || !evals || !coeffs || !commitment || !coset) return fail(ZK_EINVAL, "zk_commit_job: NULL argument");
  if (log_n > ZK_MAX_LOG_NTT || log_blowup > ZK_MAX_LOG_NTT || log_n + log_blowup > ZK_MAX_LOG_NTT)
    return fail(ZK_EUNSUPPORTED, "zk_commit_job: log_n + log_blowup > ZK_MAX_LOG_NTT");
  const uint64_t n = 1ull << log_n;
  if (n > srs->n) return fail(ZK_EINVAL, "zk_commit_job: 2^log_n exceeds the SRS size");
  uint32_t sw[8];
  if (shift_host) {
    std::memcpy(sw, shift_host->v, 32);
    unsigned br = 0;
    for (int i = 0; i < 8; i++) (void)__builtin_subc(sw[i], FrP::M32[i], br, &br);
    if (!br) return fail(ZK_EINVAL, "zk_commit_job: shift not canonical (>= r)");
  }
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{evals, n, false}}, "zk_commit_job"))) return st;
  hipStream_t side = nullptr;
  if ((st = side_stream(s, &side))) return st;
  SyncEvents ev;
  if ((st = sync_events(ev))) return st;
  uint32_t* cf = reinterpret_cast<uint32_t*>(coeffs);
  // coefficients on the caller's stream
  if ((st = run_ntt(c, reinterpret_cast<const uint32_t*>(evals), cf, log_n, true, nullptr, nullptr, (uint32_t)n, s)))
    return st;
  // the commitment; the coset transform starts on the companion stream once
  // the accumulation kernel is enqueued, so it fills the compute units the
  // latency-bound reduction leaves idle (measured: running its first pass
  // beside the sort instead slowed the sort more than it hid)
  if ((st = msm_srs_one(srs, cf, n, reinterpret_cast<uint32_t*>(commitment), s, ev.e[0]))) return st;
  ZK_HIP(hipStreamWaitEvent(side, ev.e[0], 0), "hipStreamWaitEvent");
  const f29* lo = c->coset5[0];
  const f29* hi = c->coset5[1];
  Scratch tab;
  if (shift_host) {
    const size_t tsz = sizeof(f29) << 14;
    if ((st = scratch_alloc(tab, 2 * tsz, side))) return st;
    char* base = static_cast<char*>(tab.p);
    Words8 w8;
    std::memcpy(w8.w, sw, 32);
    ZK_HIP(ntt_make_pow_tables(w8, reinterpret_cast<f29*>(base), reinterpret_cast<f29*>(base + tsz), side),
           "shift tables");
    lo = reinterpret_cast<const f29*>(base);
    hi = reinterpret_cast<const f29*>(base + tsz);
  }
  NttRun r;
  if ((st = ntt_prepare(c, cf, reinterpret_cast<uint32_t*>(coset), log_n + log_blowup, false, lo, hi, (uint32_t)n,
                        side, r, true)))
    return st;
  if ((st = ntt_first(r, side))) return st;
  if ((st = ntt_second(r, side))) return st;
  ZK_HIP(hipEventRecord(ev.e[1], side), "hipEventRecord");
  ZK_HIP(hipStreamWaitEvent(s, ev.e[1], 0), "hipStreamWaitEvent");
  return ZK_OK;
}

zk_status zk_msm_srs_ex(const zk_srs* srs, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream,
                        void* accumulate_done_event) {
  if (!srs || !out || (n && !scalars)) return fail(ZK_EINVAL, "zk_msm_srs_ex: NULL argument");
  if (n > srs->n) return fail(ZK_EINVAL, "zk_msm_srs_ex: n exceeds the SRS size");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if ((st = check_inputs(c, (hipStream_t)stream, {{scalars, n, false}}, "zk_msm_srs_ex"))) return st;
  return msm_srs_one(srs, reinterpret_cast<const uint32_t*>(scalars), n, reinterpret_cast<uint32_t*>(out),
                     (hipStream_t)stream, (hipEvent_t)accumulate_done_event);
}

zk_status zk_msm_srs(const zk_srs* srs, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream) {
  if (!srs || !out || (n && !scalars)) return fail(ZK_EINVAL, "zk_msm_srs: NULL argument");
  if (n > srs->n) return fail(ZK_EINVAL, "zk_msm_srs: n exceeds the SRS size");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if ((st = check_inputs(c, (hipStream_t)stream, {{scalars, n, false}}, "zk_msm_srs"))) return st;
  return msm_srs_one(srs, reinterpret_cast<const uint32_t*>(scalars), n, reinterpret_cast<uint32_t*>(out),
                     (hipStream_t)stream);
}

zk_status zk_msm_srs_noalloc(const zk_srs* srs, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream) {
  if (!srs || !out || (n && !scalars)) return fail(ZK_EINVAL, "zk_msm_srs_noalloc: NULL argument");
  if (n > srs->n) return fail(ZK_EINVAL, "zk_msm_srs_noalloc: n exceeds the SRS size");
  int dev = 0;
  ZK_HIP(hipGetDevice(&dev), "hipGetDevice");
  if (dev != srs->device) return fail(ZK_EINVAL, "zk_msm_srs_noalloc: the SRS belongs to another device");
  // the SRS's creation set up this device's context (and its scratch
  // address); nothing here allocates
  uint8_t* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (dev >= 0 && dev < 64 && g_ctx[dev].ready) base = g_ctx[dev].noalloc;
  }
  if (!base) return fail(ZK_EINVAL, "zk_msm_srs_noalloc: device context not set up");
  const bool tiny = srs_uses_tiny(srs, n);
  const uint64_t off[2] = {0, n};
  const MsmPlan plan = srs_plan(srs, n, off);
  const size_t need = (tiny ? msm_tiny_workspace_bytes((uint32_t)n) : msm_workspace_bytes(plan)) + 256;
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(ZK_EUNSUPPORTED, "zk_msm_srs_noalloc: " + std::to_string(n) + " points need " +
                                     std::to_string(need) + " bytes of scratch, above the fixed " +
                                     std::to_string(NOALLOC_SCRATCH_BYTES) + " (use zk_msm_srs)");
  const hipStream_t s = (hipStream_t)stream;
  if (g_validate.load(std::memory_order_relaxed)) {
    // the first 256 bytes hold this call's finding word
    uint32_t* vflag = reinterpret_cast<uint32_t*>(base);
    hipLaunchKernelGGL(noalloc_zero_kernel, dim3(1), dim3(64), 0, s, vflag);
    ZK_HIP(hipGetLastError(), "input check");
    ZK_HIP(validate_fr(reinterpret_cast<const uint32_t*>(scalars), n, vflag, s), "input check");
    uint32_t found = 0;
    ZK_HIP(hipMemcpyAsync(&found, vflag, 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync");
    ZK_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
    if (found) return fail(ZK_EINVAL, "zk_msm_srs_noalloc: an Fr input is not canonical (>= r)");
  }
  if (tiny) {
    ZK_HIP(msm_tiny_run(srs->tab_tiny, srs->n_tiny, reinterpret_cast<const uint32_t*>(scalars), (uint32_t)n,
                        base + 256, reinterpret_cast<uint32_t*>(out), s),
           "msm (small multiples)");
    return ZK_OK;
  }
  const SrsTable t = srs_table_for(srs, n);
  const uint32_t* tab = t == SrsTable::small ? srs->tab_small : t == SrsTable::large ? srs->tab_large : srs->tab;
  const MsmBuffers b = msm_carve(plan, base + 256);
  ZK_HIP(msm_run(plan, off, tab, reinterpret_cast<const uint32_t*>(scalars), b, reinterpret_cast<uint32_t*>(out), s),
         "msm");
  return ZK_OK;
}

zk_status zk_msm_batch(const zk_srs* srs, const zk_fr* scalars, const uint64_t* offsets_host, uint32_t batch,
                       zk_g1* out, void* stream) {
  if (!srs || !offsets_host || (batch && (!out || !scalars))) return fail(ZK_EINVAL, "zk_msm_batch: NULL argument");
  if (offsets_host[0] != 0) return fail(ZK_EINVAL, "zk_msm_batch: offsets_host[0] must be 0");
  for (uint32_t b = 0; b < batch; b++) {
    if (offsets_host[b + 1] < offsets_host[b]) return fail(ZK_EINVAL, "zk_msm_batch: offsets decrease");
    if (offsets_host[b + 1] - offsets_host[b] > srs->n) return fail(ZK_EINVAL, "zk_msm_batch: MSM larger than SRS");
  }
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if (batch == 0) return ZK_OK;
  if (offsets_host[batch] >= (1ull << 31) / 16) return fail(ZK_EUNSUPPORTED, "zk_msm_batch: too many scalars");
  if ((st = check_inputs(c, (hipStream_t)stream, {{scalars, offsets_host[batch], false}}, "zk_msm_batch")))
    return st;
  // one Pippenger run over every MSM: digits of all scalars sorted into
  // per-MSM buckets, one accumulation, one reduction, one output per MSM
  const MsmPlan plan = msm_plan_table(offsets_host, batch, srs->c, (uint32_t)srs->n);
  return run_msm(plan, offsets_host, srs->tab, reinterpret_cast<const uint32_t*>(scalars),
                 reinterpret_cast<uint32_t*>(out), (hipStream_t)stream);
}

zk_status zk_kzg_open_batch(const zk_srs* srs, const zk_fr* polys, uint32_t m, uint64_t n, const zk_fr* x_host,
                            const zk_fr* gamma_host, zk_fr* ys, zk_fr* quotient, zk_g1* proof, void* stream) {
  if (!srs || !x_host || !ys || !proof || m == 0 || (n && !polys) || (m > 1 && !gamma_host))
    return fail(ZK_EINVAL, "zk_kzg_open_batch: bad argument");
  const uint64_t qn = n ? n - 1 : 0;
  if (qn > srs->n) return fail(ZK_EINVAL, "zk_kzg_open_batch: n - 1 exceeds the SRS size");
  if (n >= (1ull << 31) / 16) return fail(ZK_EUNSUPPORTED, "zk_kzg_open_batch: n too large");
  if ((uint64_t)m * n >= (1ull << 40)) return fail(ZK_EUNSUPPORTED, "zk_kzg_open_batch: m * n too large");
  uint32_t xw[8], gw[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  std::memcpy(xw, x_host->v, 32);
  if (m > 1) std::memcpy(gw, gamma_host->v, 32);
  for (const uint32_t* w : {xw, gw}) {
    unsigned br = 0;
    for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], FrP::M32[i], br, &br);
    if (!br) return fail(ZK_EINVAL, "zk_kzg_open_batch: x or gamma not canonical (>= r)");
  }
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{polys, (uint64_t)m * n, false}}, "zk_kzg_open_batch"))) return st;
  const size_t sb = open_scratch_bytes(m, n);
  const size_t qb = quotient ? 0 : (size_t)qn * 32;
  Scratch ws;
  if ((st = scratch_alloc(ws, sb + qb, s))) return st;
  uint32_t* q = quotient ? reinterpret_cast<uint32_t*>(quotient)
                         : reinterpret_cast<uint32_t*>(static_cast<char*>(ws.p) + sb);
  ZK_HIP(open_quotient(reinterpret_cast<const uint32_t*>(polys), m, n, xw, gw, reinterpret_cast<uint32_t*>(ys), q,
                       ws.p, s),
         "kzg open");
  return msm_srs_one(srs, q, qn, reinterpret_cast<uint32_t*>(proof), s);
}

zk_status zk_kzg_open(const zk_srs* srs, const zk_fr* coeffs, uint64_t n, const zk_fr* x_host, zk_fr* y,
                      zk_fr* quotient, zk_g1* proof, void* stream) {
  return zk_kzg_open_batch(srs, coeffs, 1, n, x_host, nullptr, y, quotient, proof, stream);
}

// Shift s of the coset s H_(B n) (host canonical words, default 5) and the
// inverses of the B values s^n omega_B^k - 1 that X^n - 1 takes there:
// times 2^522 (times_r2) for a Montgomery product with a value divided by
// 2^261, else times 2^261 (the Montgomery form of the inverse).
static zk_status coset_vanishing(const zk_fr* shift_host, uint32_t log_n, uint32_t log_blowup, bool times_r2,
                                 const char* who, uint32_t sw[8], f29& sm, QuotZinv& zi) {
  const uint32_t five[8] = {5, 0, 0, 0, 0, 0, 0, 0};
  std::memcpy(sw, shift_host ? shift_host->v : five, 32);
  unsigned br = 0;
  for (int i = 0; i < 8; i++) (void)__builtin_subc(sw[i], FrP::M32[i], br, &br);
  if (!br) return fail(ZK_EINVAL, std::string(who) + ": shift not canonical (>= r)");
  const f29 one = f29_from(FrP::ONE);
  sm = reduce_full<FrP>(to_mont<FrP>(unpack(sw)));
  if (f29_is_zero_limbs(sm)) return fail(ZK_EINVAL, std::string(who) + ": shift is zero");
  f29 sn = sm;  // s^n by log_n squarings
  for (uint32_t i = 0; i < log_n; i++) sn = reduce_full<FrP>(mont_mul<FrP>(sn, sn));
  f29 wb = reduce_full<FrP>(to_mont<FrP>(unpack(FR_OMEGA_2_28)));  // omega_B = omega_(2^28)^(2^(28 - log_b))
  for (uint32_t i = 0; i < 28 - log_blowup; i++) wb = reduce_full<FrP>(mont_mul<FrP>(wb, wb));
  f29 pk = sn;
  for (uint32_t k = 0; k < (1u << log_blowup); k++) {
    const f29 z = reduce_full<FrP>(sub_k(pk, one, FrP::K2));
    if (f29_is_zero_limbs(z))
      return fail(ZK_EINVAL, std::string(who) + ": X^n - 1 vanishes on the coset (bad shift)");
    const f29 zinv = reduce_full<FrP>(mont_inv<FrP>(z));
    zi.zinv_r2[k] = times_r2 ? reduce_full<FrP>(mont_mul<FrP>(zinv, f29_from(FrP::R2))) : zinv;
    pk = reduce_full<FrP>(mont_mul<FrP>(pk, wb));
  }
  for (uint32_t k = 1u << log_blowup; k < (1u << QUOT_MAX_LOG_BLOWUP); k++) zi.zinv_r2[k] = f29_zero();
  return ZK_OK;
}

zk_status zk_quotient_mul(const zk_srs* srs, const zk_fr* a, const zk_fr* b, const zk_fr* c_evals, uint32_t log_n,
                          uint32_t log_blowup, const zk_fr* shift_host, zk_fr* t_coeffs, zk_g1* t_commit,
                          void* stream) {
  if (!srs || !a || !b || !c_evals || !t_coeffs || !t_commit) return fail(ZK_EINVAL, "zk_quotient_mul: NULL argument");
  if (log_blowup < 1 || log_blowup > QUOT_MAX_LOG_BLOWUP)
    return fail(ZK_EINVAL, "zk_quotient_mul: log_blowup must be 1..4");
  if (log_n > ZK_MAX_LOG_NTT || log_n + log_blowup > ZK_MAX_LOG_NTT)
    return fail(ZK_EUNSUPPORTED, "zk_quotient_mul: log_n + log_blowup > ZK_MAX_LOG_NTT");
  const uint64_t n = 1ull << log_n;
  if (n > srs->n) return fail(ZK_EINVAL, "zk_quotient_mul: 2^log_n exceeds the SRS size");
  uint32_t sw[8];
  f29 sm;
  QuotZinv zi;
  zk_status st0 = coset_vanishing(shift_host, log_n, log_blowup, true, "zk_quotient_mul", sw, sm, zi);
  if (st0) return st0;
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{a, n, false}, {b, n, false}, {c_evals, n, false}}, "zk_quotient_mul"))) return st;
  const uint32_t L = log_n + log_blowup;
  const uint64_t big = 1ull << L;
  const size_t tsz = sizeof(f29) << 14;
  Scratch ws;
  if ((st = scratch_alloc(ws, (size_t)32 * (n + 3 * big) + (shift_host ? 4 * tsz : 0), s))) return st;
  uint32_t* coef = static_cast<uint32_t*>(ws.p);
  uint32_t* E[3] = {coef + 8 * n, coef + 8 * (n + big), coef + 8 * (n + 2 * big)};
  const f29 *lo = c->coset5[0], *hi = c->coset5[1], *ilo = c->coset5inv[0], *ihi = c->coset5inv[1];
  if (shift_host) {
    f29* t = reinterpret_cast<f29*>(coef + 8 * (n + 3 * big));
    Words8 fw, iw;
    std::memcpy(fw.w, sw, 32);
    host_words(from_mont<FrP>(mont_inv<FrP>(sm)), iw.w);
    ZK_HIP(ntt_make_pow_tables(fw, t, t + (1u << 14), s), "shift tables");
    ZK_HIP(ntt_make_pow_tables(iw, t + (2u << 14), t + (3u << 14), s), "shift tables");
    lo = t;
    hi = t + (1u << 14);
    ilo = t + (2u << 14);
    ihi = t + (3u << 14);
  }
  // f, h, g on the coset: coefficients, then the coset transform of each
  const zk_fr* in[3] = {a, b, c_evals};
  for (int k = 0; k < 3; k++) {
    if ((st = run_ntt(c, reinterpret_cast<const uint32_t*>(in[k]), coef, log_n, true, nullptr, nullptr, (uint32_t)n,
                      s)))
      return st;
    if ((st = run_ntt(c, coef, E[k], L, false, lo, hi, (uint32_t)n, s))) return st;
  }
  // t on the coset, then its coefficients: inverse transform, times s^-i
  ZK_HIP(quot_mul_pointwise(E[0], E[1], E[2], big, log_blowup, zi, s), "quotient pointwise");
  if ((st = run_ntt(c, E[0], E[0], L, true, nullptr, nullptr, (uint32_t)big, s))) return st;
  ZK_HIP(quot_scale_powers(E[0], n, ilo, ihi, reinterpret_cast<uint32_t*>(t_coeffs), s), "quotient scale");
  return msm_srs_one(srs, reinterpret_cast<const uint32_t*>(t_coeffs), n, reinterpret_cast<uint32_t*>(t_commit), s);
}

zk_status zk_quotient_polyiop(const zk_srs* srs, const zk_fr* evals, uint32_t N, uint32_t log_n,
                              const zk_constraint_term* terms_host, uint32_t nterms, uint32_t log_blowup,
                              const zk_fr* shift_host, zk_fr* q_coeffs, zk_g1* q_commit, void* stream) {
  if (!srs || !evals || !terms_host || !q_coeffs || !q_commit)
    return fail(ZK_EINVAL, "zk_quotient_polyiop: NULL argument");
  if (N < 1 || N > ZK_POLYIOP_MAX_WITNESS) return fail(ZK_EINVAL, "zk_quotient_polyiop: N must be 1..8");
  if (nterms < 1 || nterms > ZK_POLYIOP_MAX_TERMS) return fail(ZK_EINVAL, "zk_quotient_polyiop: nterms must be 1..16");
  if (log_blowup < 1 || log_blowup > QUOT_MAX_LOG_BLOWUP)
    return fail(ZK_EINVAL, "zk_quotient_polyiop: log_blowup must be 1..4");
  if (log_n > ZK_MAX_LOG_NTT || log_n + log_blowup > ZK_MAX_LOG_NTT)
    return fail(ZK_EUNSUPPORTED, "zk_quotient_polyiop: log_n + log_blowup > ZK_MAX_LOG_NTT");
  static_assert(ZK_POLYIOP_MAX_WITNESS == POLYIOP_MAX_N && ZK_POLYIOP_MAX_TERMS == POLYIOP_MAX_TERMS &&
                    ZK_POLYIOP_MAX_DEGREE == POLYIOP_MAX_DEG,
                "Poly-IOP limits of the header and the kernel agree");
  // the terms: coefficient c * 2^(261 d) in Montgomery limbs (a chain of
  // d - 1 products of plain operands and one with it gives the plain term)
  PolyIopTerms T{};
  T.nterms = nterms;
  T.N = N;
  uint32_t d = 0;
  for (uint32_t t = 0; t < nterms; t++) {
    const zk_constraint_term& in = terms_host[t];
    if (in.nfactors > ZK_POLYIOP_MAX_DEGREE)
      return fail(ZK_EINVAL, "zk_quotient_polyiop: a term has more than 4 factors");
    uint32_t cw[8];
    std::memcpy(cw, in.coeff.v, 32);
    unsigned br = 0;
    for (int i = 0; i < 8; i++) (void)__builtin_subc(cw[i], FrP::M32[i], br, &br);
    if (!br) return fail(ZK_EINVAL, "zk_quotient_polyiop: a coefficient is not canonical (>= r)");
    uint32_t packed = 0;
    for (uint32_t i = 0; i < in.nfactors; i++) {
      if (in.factor[i] >= 2 * N) return fail(ZK_EINVAL, "zk_quotient_polyiop: factor index >= 2N");
      packed |= in.factor[i] << (8 * i);
    }
    T.nfac[t] = in.nfactors;
    T.fac[t] = packed;
    f29 c = reduce_full<FrP>(unpack(cw));  // plain c
    for (uint32_t i = 0; i < in.nfactors; i++) c = reduce_full<FrP>(to_mont<FrP>(c));  // c 2^(261 i)
    T.coeff[t] = c;
    const bool is_one = cw[0] == 1 && !(cw[1] | cw[2] | cw[3] | cw[4] | cw[5] | cw[6] | cw[7]);
    T.ident[t] = (in.nfactors == 1 && is_one) ? 1u : 0u;
    d = std::max(d, in.nfactors);
  }
  if ((1u << log_blowup) < d) return fail(ZK_EINVAL, "zk_quotient_polyiop: blowup 2^log_blowup below the degree");
  const uint64_t n = 1ull << log_n;
  const uint64_t qlen = (uint64_t)(d > 1 ? d - 1 : 1) * n;  // deg Q <= d (n - 1) - n
  if (qlen > srs->n) return fail(ZK_EINVAL, "zk_quotient_polyiop: the quotient has more coefficients than the SRS points");
  uint32_t sw[8];
  f29 sm;
  QuotZinv zi;
  zk_status st = coset_vanishing(shift_host, log_n, log_blowup, false, "zk_quotient_polyiop", sw, sm, zi);
  if (st) return st;
  DeviceCtx* c;
  if ((st = ctx_get(&c))) return st;
  const hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{evals, (uint64_t)N * n, false}}, "zk_quotient_polyiop"))) return st;
  const uint32_t L = log_n + log_blowup;
  const uint64_t big = 1ull << L;
  const size_t tsz = sizeof(f29) << 14;
  Scratch ws;
  if ((st = scratch_alloc(ws, (size_t)32 * (n + (N + 1) * big) + (shift_host ? 4 * tsz : 0), s))) return st;
  uint32_t* coef = static_cast<uint32_t*>(ws.p);
  uint32_t* E = coef + 8 * n;                // N coset vectors of big points each
  uint32_t* V = E + 8 * (size_t)N * big;     // R / Z on the coset, then its inverse transform
  const f29 *lo = c->coset5[0], *hi = c->coset5[1], *ilo = c->coset5inv[0], *ihi = c->coset5inv[1];
  if (shift_host) {
    f29* t = reinterpret_cast<f29*>(V + 8 * big);
    Words8 fw, iw;
    std::memcpy(fw.w, sw, 32);
    host_words(from_mont<FrP>(mont_inv<FrP>(sm)), iw.w);
    ZK_HIP(ntt_make_pow_tables(fw, t, t + (1u << 14), s), "shift tables");
    ZK_HIP(ntt_make_pow_tables(iw, t + (2u << 14), t + (3u << 14), s), "shift tables");
    lo = t;
    hi = t + (1u << 14);
    ilo = t + (2u << 14);
    ihi = t + (3u << 14);
  }
  // every witness on the coset: coefficients, then the coset transform
  for (uint32_t k = 0; k < N; k++) {
    if ((st = run_ntt(c, reinterpret_cast<const uint32_t*>(evals) + 8 * (size_t)k * n, coef, log_n, true, nullptr,
                      nullptr, (uint32_t)n, s)))
      return st;
    if ((st = run_ntt(c, coef, E + 8 * (size_t)k * big, L, false, lo, hi, (uint32_t)n, s))) return st;
  }
  // Q on the coset, then its coefficients: inverse transform, times s^-i
  ZK_HIP(quot_polyiop_pointwise(E, big, log_blowup, T, zi, V, s), "quotient pointwise");
  if ((st = run_ntt(c, V, V, L, true, nullptr, nullptr, (uint32_t)big, s))) return st;
  ZK_HIP(quot_scale_powers(V, qlen, ilo, ihi, reinterpret_cast<uint32_t*>(q_coeffs), s), "quotient scale");
  return msm_srs_one(srs, reinterpret_cast<const uint32_t*>(q_coeffs), qlen, reinterpret_cast<uint32_t*>(q_commit),
                     s);
}

zk_status zk_calibrate_mad_rate(uint32_t blocks, uint32_t iters, double* mads_per_s, void* stream) {
  if (!mads_per_s || blocks == 0 || iters == 0) return fail(ZK_EINVAL, "zk_calibrate_mad_rate: bad argument");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  Scratch sink;
  if ((st = scratch_alloc(sink, 256, s))) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ZK_HIP(hipEventCreate(&e0), "hipEventCreate");
  hipError_t e = hipEventCreate(&e1);
  if (e == hipSuccess) e = prof_mad_rate_launch(blocks, iters, static_cast<uint32_t*>(sink.p), s);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) e = prof_mad_rate_launch(blocks, iters, static_cast<uint32_t*>(sink.p), s);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "zk_calibrate_mad_rate");
  *mads_per_s = ms > 0 ? (double)prof_mad_count(blocks, iters) / (ms * 1e-3) : 0.0;
  return ZK_OK;
}

zk_status zk_transcript_challenge(const void* data, uint64_t bytes, zk_fr* challenge, void* stream) {
  if (!challenge || (bytes && !data)) return fail(ZK_EINVAL, "zk_transcript_challenge: NULL argument");
  if (bytes >= (1ull << 40)) return fail(ZK_EUNSUPPORTED, "zk_transcript_challenge: input too long");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  // 2^256 in Montgomery form: twice the Montgomery form of 2^255
  uint32_t w[8] = {0, 0, 0, 0, 0, 0, 0, 0x80000000u};
  const f29 h = reduce_full<FrP>(to_mont<FrP>(unpack(w)));
  const f29 c256 = reduce_full<FrP>(add_n(h, h));
  ZK_HIP(transcript_challenge(static_cast<const uint8_t*>(data), bytes, c256, reinterpret_cast<uint32_t*>(challenge),
                              (hipStream_t)stream),
         "transcript");
  return ZK_OK;
}

zk_status zk_acc_fold(uint32_t k, const zk_g1* C, const zk_g1* C2, uint32_t d, const zk_g1* E, const zk_g1* E2,
                      const zk_g1* Ej, uint64_t len_v, const zk_fr* v, const zk_fr* v2, uint64_t len_e,
                      const zk_fr* e, const zk_fr* e2, const zk_fr* ej, const zk_fr* gamma, zk_g1* C_out,
                      zk_g1* E_out, zk_fr* v_out, zk_fr* e_out, void* stream) {
  if (!gamma || !E || !E2 || !E_out || (d > 1 && !Ej) || (k && (!C || !C2 || !C_out)) ||
      (len_v && (!v || !v2 || !v_out)) || (len_e && (!e || !e2 || !e_out || (d > 1 && !ej))))
    return fail(ZK_EINVAL, "zk_acc_fold: NULL argument");
  if (d < 1 || d > ACC_MAX_D) return fail(ZK_EINVAL, "zk_acc_fold: d must be 1..15");
  if (k >= (1u << 20)) return fail(ZK_EUNSUPPORTED, "zk_acc_fold: k too large");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s,
                         {{C, k, true}, {C2, k, true}, {E, 1, true}, {E2, 1, true}, {Ej, d - 1ull, true},
                          {gamma, 1, false}, {v, len_v, false}, {v2, len_v, false}, {e, len_e, false},
                          {e2, len_e, false}, {ej, (d - 1ull) * len_e, false}},
                         "zk_acc_fold")))
    return st;
  Scratch ws;
  if ((st = scratch_alloc(ws, acc_fold_g1_scratch_bytes(k, d), s))) return st;
  const uint32_t* gw = reinterpret_cast<const uint32_t*>(gamma);
  // the Fr parts (HBM streams) run on the companion stream beside the G1
  // part (a few waves of dependent point operations); the caller's stream
  // waits for both
  hipStream_t side = nullptr;
  if ((st = side_stream(s, &side))) return st;
  SyncEvents ev;
  if ((st = sync_events(ev))) return st;
  ZK_HIP(hipEventRecord(ev.e[0], s), "hipEventRecord");
  ZK_HIP(hipStreamWaitEvent(side, ev.e[0], 0), "hipStreamWaitEvent");
  ZK_HIP(fr_rlc(reinterpret_cast<const uint32_t*>(v2), nullptr, reinterpret_cast<const uint32_t*>(v), 1, len_v, gw,
                reinterpret_cast<uint32_t*>(v_out), side),
         "acc fold fr");
  ZK_HIP(fr_rlc(reinterpret_cast<const uint32_t*>(e2), reinterpret_cast<const uint32_t*>(ej),
                reinterpret_cast<const uint32_t*>(e), d, len_e, gw, reinterpret_cast<uint32_t*>(e_out), side),
         "acc fold errors");
  ZK_HIP(acc_fold_g1(reinterpret_cast<const uint32_t*>(C), reinterpret_cast<const uint32_t*>(C2), k,
                     reinterpret_cast<const uint32_t*>(E), reinterpret_cast<const uint32_t*>(E2),
                     reinterpret_cast<const uint32_t*>(Ej), d, gw, reinterpret_cast<uint32_t*>(C_out),
                     reinterpret_cast<uint32_t*>(E_out), ws.p, s),
         "acc fold g1");
  ZK_HIP(hipEventRecord(ev.e[1], side), "hipEventRecord");
  ZK_HIP(hipStreamWaitEvent(s, ev.e[1], 0), "hipStreamWaitEvent");
  return ZK_OK;
}

zk_status zk_srs_g2_setup(const zk_fr* tau_host, uint64_t n, zk_g2* out, void* stream) {
  if (!tau_host || (n && !out)) return fail(ZK_EINVAL, "zk_srs_g2_setup: NULL argument");
  if (n >= (1ull << 26)) return fail(ZK_EUNSUPPORTED, "zk_srs_g2_setup: n too large");
  uint32_t w[8];
  std::memcpy(w, tau_host->v, 32);
  unsigned br = 0;
  for (int i = 0; i < 8; i++) (void)__builtin_subc(w[i], FrP::M32[i], br, &br);
  if (!br) return fail(ZK_EINVAL, "zk_srs_g2_setup: tau not canonical (>= r)");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  Scratch gt;
  if ((st = scratch_alloc(gt, (size_t)254 * G2_AFF_WORDS * 4, s))) return st;
  ZK_HIP(g2_srs_from_tau(w, reinterpret_cast<uint32_t*>(out), n, static_cast<uint32_t*>(gt.p), s), "g2 srs setup");
  return ZK_OK;
}

zk_status zk_srs_g2_create(const zk_g2* points, uint64_t n, zk_srs_g2** srs, void* stream) {
  if (!srs || (n && !points)) return fail(ZK_EINVAL, "zk_srs_g2_create: NULL argument");
  if (n >= (1ull << 26)) return fail(ZK_EUNSUPPORTED, "zk_srs_g2_create: n too large");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  if ((st = check_inputs(c, (hipStream_t)stream, {{points, n, 2}}, "zk_srs_g2_create"))) return st;
  zk_srs_g2* h = new zk_srs_g2();
  ZK_HIP(hipGetDevice(&h->device), "hipGetDevice");
  h->n = n;
  h->tab = nullptr;
  if (n) {
    hipError_t e = hipMalloc(&h->tab, (size_t)G2_W * n * G2_AFF_WORDS * 4);
    if (e == hipSuccess)
      e = g2_build_table(reinterpret_cast<const uint32_t*>(points), h->tab, n, (hipStream_t)stream);
    if (e != hipSuccess) {
      if (h->tab) (void)hipFree(h->tab);
      delete h;
      return hip_fail(e, "zk_srs_g2_create: table build");
    }
  }
  *srs = h;
  return ZK_OK;
}

zk_status zk_srs_g2_destroy(zk_srs_g2* srs) {
  if (!srs) return ZK_OK;
  if (srs->tab) {
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(srs->device);
    (void)hipDeviceSynchronize();
    (void)hipFree(srs->tab);
    (void)hipSetDevice(prev);
  }
  delete srs;
  return ZK_OK;
}

uint64_t zk_srs_g2_size(const zk_srs_g2* srs) { return srs ? srs->n : 0; }

zk_status zk_msm_g2_srs(const zk_srs_g2* srs, const zk_fr* scalars, uint64_t n, zk_g2* out, void* stream) {
  if (!srs || !out || (n && !scalars)) return fail(ZK_EINVAL, "zk_msm_g2_srs: NULL argument");
  if (n > srs->n) return fail(ZK_EINVAL, "zk_msm_g2_srs: n exceeds the SRS size");
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  const hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{scalars, n, false}}, "zk_msm_g2_srs"))) return st;
  Scratch ws;
  if ((st = scratch_alloc(ws, g2_msm_scratch_bytes(n), s))) return st;
  ZK_HIP(g2_msm(srs->tab, srs->n, reinterpret_cast<const uint32_t*>(scalars), n, reinterpret_cast<uint32_t*>(out),
                ws.p, s),
         "g2 msm");
  return ZK_OK;
}

zk_status zk_fold(const zk_g1* inst, const zk_fr* gammas, uint32_t m, uint32_t k, zk_g1* out, void* stream) {
  if (!inst || !out || m == 0 || (m > 1 && !gammas)) return fail(ZK_EINVAL, "zk_fold: bad argument");
  if ((uint64_t)m * k >= (1ull << 31) / 16) return fail(ZK_EUNSUPPORTED, "zk_fold: too many points");
  if (k == 0) return ZK_OK;
  DeviceCtx* c;
  zk_status st = ctx_get(&c);
  if (st) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = check_inputs(c, s, {{inst, (uint64_t)m * k, true}, {gammas, m - 1ull, false}}, "zk_fold"))) return st;
  // few instances: every term sigma_i C_i on its own quad (the latency of one
  // scalar multiple); many: one Pippenger MSM per component
  const bool per_term = m <= G1_RLC_TERMS_MAX && (uint64_t)m * k <= (1u << 16);
  Scratch ws;
  const size_t sig_bytes = ((size_t)m * 32 + 255) / 256 * 256;
  st = scratch_alloc(ws, per_term ? sig_bytes + g1_rlc_scratch_bytes(m, k) : (size_t)m * (32 + 64 + 64) + 512, s);
  if (st) return st;
  uint32_t* sigma = static_cast<uint32_t*>(ws.p);
  ZK_HIP(fold_sigmas(reinterpret_cast<const uint32_t*>(gammas), m, sigma, s), "fold sigmas");
  if (per_term) {
    ZK_HIP(g1_rlc(reinterpret_cast<const uint32_t*>(inst), sigma, m, k, reinterpret_cast<uint32_t*>(out),
                  static_cast<char*>(ws.p) + sig_bytes, s),
           "fold terms");
    return ZK_OK;
  }
  uint32_t* col = sigma + (size_t)m * 8;
  uint32_t* mont = col + (size_t)m * 16;
  const MsmPlan plan = msm_plan_generic(m, msm_default_c(m));
  for (uint32_t j = 0; j < k; j++) {
    ZK_HIP(gather_component(reinterpret_cast<const uint32_t*>(inst), m, k, j, col, s), "fold gather");
    ZK_HIP(msm_points_to_mont(col, mont, m, s), "fold to_mont");
    st = run_msm(plan, nullptr, mont, sigma, reinterpret_cast<uint32_t*>(out) + (size_t)j * 16, s);
    if (st) return st;
  }
  return ZK_OK;
}

}  // extern "C"
