// Radix-2 NTT / inverse NTT / coset NTT over the BN254 scalar field Fr.
//
// What is computed (the paper's witness encoding: a length-n vector is a
// polynomial's evaluations on H = {omega^i}, element i = f(omega^i)):
//   forward  X[k] = sum_i x[i] omega_N^(i k)           (coefficients -> evaluations)
//   inverse  x[i] = N^-1 sum_k X[k] omega_N^(-i k)     (evaluations -> coefficients)
//   coset    E[j] = f(g omega_(Bn)^j): inputs scaled by g^i, zero-padded to Bn
// with omega_N = 5^((r-1)/N), natural order in and out.
//
// Scheme: a transform of N = N1 * N2 points runs as two passes over HBM (the
// "four-step" factorisation), each pass a batch of LDS-resident radix-2
// transforms of at most 4096 points:
//   pass A: for every i1 < N1, Y[i1][k2] = omega_N^(i1 k2) * NTT_N2(x[i1 + N1 i2])
//   pass B: for every k2 < N2, X[k2 + N2 k1] = NTT_N1(Y[i1][k2])
// Above 2^24 points N1 exceeds a tile and pass B is itself factored,
// N1 = P1 * P2, i1 = j1 + P1 j2, k1 = k1' + P2 k1'' (three passes in all):
//   pass B1: Z[k2 + N2 k1' + N2 P2 j1] = omega_N1^(j1 k1') * NTT_P2(Y[j1 + P1 j2][k2])
//   pass B2: X[k2 + N2 k1' + N2 P2 k1''] = NTT_P1(Z[...j1...])
// B1's batch index k2 + N2 j1 is split (b_hi_log) so that B2 reads every one
// of its transforms at a single stride.
// Inside a tile the points are loaded in bit-reversed order into LDS and run
// through log2(M) decimation-in-time stages.  A workgroup owns G adjacent
// transforms so that each strided global access moves G*32 contiguous bytes.
//
// Arithmetic: data stay plain canonical integers (32-bit words); twiddles are
// Montgomery-form constants in 29-bit limbs, so one Montgomery product
// returns the plain product w*v.  Twiddle tables hold omega_(2^28)^e for
// e < 2^14 ("lo") and e = j*2^14 ("hi"); omega_N^e = lo * hi of the exponent
// e*2^(28-L) split in two halves.  In-tile twiddles come from a "ladder"
// that stores each stage's roots omega_(2^k)^j contiguously, so the lanes of
// a wave read adjacent entries rather than one cache line each.
#include "ntt.h"
#include "prof.h"

namespace zk {

namespace {

constexpr uint32_t TILE_LOG = 12;
constexpr uint32_t TILE = 1u << TILE_LOG;    // elements per workgroup, at most
constexpr uint32_t NTT_THREADS = 512;        // threads per workgroup, at most (one 8-point unit each)

__device__ __forceinline__ void ld8(const uint32_t* p, uint32_t w[8]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
  w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}

__device__ __forceinline__ void st8(uint32_t* p, const uint32_t w[8]) {
  reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

__device__ __forceinline__ f29 ldf29(const f29* t, uint32_t i) { return t[i]; }

// LDS slot of tile point e: one 32-byte pad after every 8 points.  Units of
// the first stages read points 8 (or 64) apart; unpadded, those 256-byte
// strides put the lanes of an access on the same banks.
__device__ __forceinline__ uint32_t* lds_at(uint32_t* lds, uint32_t e) { return lds + (e + (e >> 3)) * 8; }

// omega^(e) of the 2^28-th root for e < 2^28, from the split tables (times
// the constant of a scaled lo table, which then also serves e < 2^14 alone
// but never lets hi stand alone).
__device__ __forceinline__ f29 pow28(const f29* lo, const f29* hi, uint32_t E, bool scaled = false) {
  const uint32_t a = E & 0x3fffu, b = E >> 14;
  if (b == 0) return ldf29(lo, a);
  if (a == 0 && !scaled) return ldf29(hi, b);
  return mont_mul<FrP>(ldf29(lo, a), ldf29(hi, b));
}

// Inside a tile values are kept in [0, 2q) (2q < 2^255), not canonical: a
// twiddle product of such a value is < 2q without a final correction, and a
// sum or difference needs one conditional correction by 2q.  The store makes
// every value canonical.
__device__ __forceinline__ uint32_t q2_word(int i) {
  return (FrP::M32[i] << 1) | (i ? FrP::M32[i - 1] >> 31 : 0u);
}

__device__ __forceinline__ void add_2q(const uint32_t a[8], const uint32_t b[8], uint32_t r[8]) {
  uint32_t sum[8], d[8];
  unsigned c = 0, br = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) sum[i] = __builtin_addc(a[i], b[i], c, &c);
#pragma unroll
  for (int i = 0; i < 8; i++) d[i] = __builtin_subc(sum[i], q2_word(i), br, &br);
#pragma unroll
  for (int i = 0; i < 8; i++) r[i] = br ? sum[i] : d[i];
}

__device__ __forceinline__ void sub_2q(const uint32_t a[8], const uint32_t b[8], uint32_t r[8]) {
  uint32_t d[8];
  unsigned br = 0, c = 0;
#pragma unroll
  for (int i = 0; i < 8; i++) d[i] = __builtin_subc(a[i], b[i], br, &br);
  const uint32_t mask = 0u - br;
#pragma unroll
  for (int i = 0; i < 8; i++) r[i] = __builtin_addc(d[i], q2_word(i) & mask, c, &c);
}

// a * w (w a Montgomery-form twiddle) for a < 2q: < a q / 2^261 + q < 2q.
__device__ __forceinline__ void mul_tw_2q(const uint32_t a[8], const f29& w, uint32_t r[8]) {
  pack(mont_mul<FrP>(unpack(a), w), r);
}

// Twiddles of a unit's R stages: stage s+T uses omega_(2^(s+T))^(j + qlow h)
// for qlow < 2^T, ladder entry 2^(s+T-1) + j + qlow h, kept at index
// 2^T - 1 + qlow.  All 2^R - 1 are loaded before the unit's points, so
// their latency overlaps the LDS reads and the first butterflies instead of
// stalling each product.
template <int R>
struct UnitTw {
  f29 w[(1 << R) - 1];
};

template <int R>
__device__ __forceinline__ void load_unit_tw(UnitTw<R>& tw, uint32_t s, uint32_t j, uint32_t h,
                                             const f29* __restrict__ ladder) {
#pragma unroll
  for (int T = 0; T < R; T++)
#pragma unroll
    for (int ql = 0; ql < (1 << T); ql++) tw.w[(1 << T) - 1 + ql] = ldf29(ladder, (1u << (s + T - 1)) + j + ql * h);
}

// One butterfly of stage s+T on registers x[q], x[q + 2^T] of a unit (q with
// bit T clear); its twiddle is omega_(2^(s+T))^jt, jt = j + (q mod 2^T) h.
// Twiddles that are 1 (j = 0 in the first stage of a tile) are skipped.
template <int Q, int R, int T, int P>
__device__ __forceinline__ void dit_butterflies(uint32_t (&x)[Q][8], uint32_t s, const UnitTw<R>& tw) {
  constexpr uint32_t q = ((P >> T) << (T + 1)) | (P & ((1u << T) - 1));
  constexpr uint32_t r = q + (1u << T);
  constexpr uint32_t qlow = q & ((1u << T) - 1);
  uint32_t tv[8];
  if (s == 1 && qlow == 0) {
#pragma unroll
    for (int w = 0; w < 8; w++) tv[w] = x[r][w];
  } else {
    mul_tw_2q(x[r], tw.w[(1u << T) - 1 + qlow], tv);
  }
  add_2q(x[q], tv, x[r]);
  sub_2q(x[q], tv, tv);
#pragma unroll
  for (int w = 0; w < 8; w++) {
    const uint32_t sum = x[r][w];
    x[r][w] = tv[w];
    x[q][w] = sum;
  }
  if constexpr (P + 1 < Q / 2) dit_butterflies<Q, R, T, P + 1>(x, s, tw);
}

template <int Q, int T, int R>
__device__ __forceinline__ void dit_levels(uint32_t (&x)[Q][8], uint32_t s, const UnitTw<R>& tw) {
  dit_butterflies<Q, R, T, 0>(x, s, tw);
  if constexpr (T + 1 < R) dit_levels<Q, T + 1, R>(x, s, tw);
}

// R consecutive decimation-in-time stages s .. s+R-1 on the LDS tile, each
// thread holding 2^R points in registers.  A unit is the set of points
// base + q*h (q < 2^R, h = 2^(s-1)) that these stages combine only among
// themselves: stage s+T pairs q with q + 2^T.
template <int R>
__device__ __forceinline__ void dit_stages(uint32_t* lds, uint32_t s, uint32_t m, uint32_t TE,
                                           const f29* __restrict__ ladder) {
  constexpr int Q = 1 << R;
  const uint32_t h = 1u << (s - 1);
  const uint32_t units_per_tr = 1u << (m - R);
  for (uint32_t u = threadIdx.x; u < TE / Q; u += blockDim.x) {
    const uint32_t b = u >> (m - R), ul = u & (units_per_tr - 1);
    const uint32_t j = ul & (h - 1), grp = ul >> (s - 1);
    const uint32_t base = (b << m) + (grp << (s + R - 1)) + j;
    UnitTw<R> tw;
    load_unit_tw<R>(tw, s, j, h, ladder);
    uint32_t x[Q][8];
#pragma unroll
    for (int q = 0; q < Q; q++) ld8(lds_at(lds, base + q * h), x[q]);
    dit_levels<Q, 0, R>(x, s, tw);
#pragma unroll
    for (int q = 0; q < Q; q++) st8(lds_at(lds, base + q * h), x[q]);
  }
}

// Workgroups go to the eight XCDs round robin (block b to XCD b mod 8), each
// XCD with its own L2.  Blocks are renumbered so that every XCD runs one
// contiguous range of tiles: neighbouring tiles read the two halves (or
// quarters) of the same 128-byte lines in a strided pass, and then fetch
// each line into one L2 only.  A bijection of [0, nb) for any nb.
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nb) {
  constexpr uint32_t XCDS = 8;
  const uint32_t q = nb / XCDS, r = nb % XCDS, x = b % XCDS;
  return x * q + min(x, r) + b / XCDS;
}

// MAXR = 3: a thread holds 8 points and runs up to three stages per LDS round
// trip (fewer round trips; 206 VGPRs, two waves per SIMD).  MAXR = 2: 4
// points and two stages (more round trips, but at most 128 VGPRs, so the
// workgroups a compute unit's LDS holds fill four waves per SIMD).
template <int MAXR>
__device__ __forceinline__ void ntt_pass_body(const NttPass& a) {
  extern __shared__ uint32_t lds[];
  const uint32_t M = 1u << a.m;
  const uint32_t g0 = xcd_contiguous(blockIdx.x, gridDim.x) * a.G;
  const uint32_t G = min(a.G, a.nbatch - g0);
  const uint32_t TE = M * G;
  const uint32_t tid = threadIdx.x;

  // ---- load (bit-reversed into LDS), coset pre-scale, zero padding.  Only
  // the first 2^(m - z) points of each transform can be nonzero (z =
  // zero_log); in bit-reversed order they sit at slots that are multiples of
  // 2^z, and the first z stages turn each such group [v, 0, ..., 0] into
  // [v, v, ..., v], so v is written to its 2^z slots and those stages are
  // skipped.
  const uint32_t z = a.zero_log;
  const uint32_t TL = TE >> z;
  for (uint32_t e = tid; e < TL; e += blockDim.x) {
    const uint32_t b = e % G, i = e / G;
    const uint32_t gi = (g0 + b) + i * a.s_in;
    uint32_t w[8];
    if (gi < a.valid_n) {
      ld8(a.in + (size_t)gi * 8, w);
      if (a.pre_lo) {
        const f29 s = pow28(a.pre_lo, a.pre_hi, gi);
        mul_plain_by_mont<FrP>(w, s, w);
      }
    } else {
#pragma unroll
      for (int q = 0; q < 8; q++) w[q] = 0;
    }
    const uint32_t slot = b * M + (a.m ? (__brev(i) >> (32 - a.m)) : 0);
    for (uint32_t r = 0; r < (1u << z); r++) st8(lds_at(lds, slot + r), w);
  }
  __syncthreads();

  // ---- decimation-in-time stages, up to MAXR per LDS round trip
  for (uint32_t st = 1 + z; st <= a.m;) {
    const uint32_t left = a.m - st + 1;
    if (left == 1) {
      dit_stages<1>(lds, st, a.m, TE, a.ladder);
      st += 1;
    } else if (MAXR >= 3 && left >= 3) {
      dit_stages<MAXR>(lds, st, a.m, TE, a.ladder);
      st += MAXR;
    } else {
      dit_stages<2>(lds, st, a.m, TE, a.ladder);
      st += 2;
    }
    __syncthreads();
  }

  // ---- store with optional four-step twiddle and final scale
  const bool row_out = (a.s_out == 1);
  for (uint32_t e = tid; e < TE; e += blockDim.x) {
    const uint32_t b = row_out ? e / M : e % G;
    const uint32_t k = row_out ? e % M : e / G;
    uint32_t w[8];
    ld8(lds_at(lds, b * M + k), w);
    const uint32_t bb = g0 + b;
    const size_t ob = a.b_hi_log ? (size_t)(bb & ((1u << a.b_hi_log) - 1)) * a.b_out + (size_t)(bb >> a.b_hi_log) * a.b_out_hi
                                 : (size_t)bb * a.b_out;
    if (a.tw_full) {
      // the twiddle of (b, k) read from its table (adjacent lanes, adjacent
      // words) instead of formed by a product of two split-table entries
      const size_t ti = ((size_t)(bb >> a.tw_shift) << a.m) + k;
      f29 t;
#pragma unroll
      for (int l = 0; l < 9; l++) t.l[l] = a.tw_full[((size_t)l << a.post_tw_L) + ti];
      mul_tw_2q(w, t, w);
    } else if (a.post_tw_L) {
      const uint32_t ex = ((bb >> a.tw_shift) * k) & ((1u << a.post_tw_L) - 1);
      if (ex || a.tw_scaled) mul_tw_2q(w, pow28(a.tw_lo, a.tw_hi, ex << (28 - a.post_tw_L), a.tw_scaled != 0), w);
    }
    if (a.post_scale) mul_tw_2q(w, *a.post_scale, w);
    canon32<FrP>(w);
    st8(a.out + (ob + (size_t)k * a.s_out) * 8, w);
  }
}

__global__ void __launch_bounds__(NTT_THREADS) ntt_pass_kernel(NttPass a) { ntt_pass_body<3>(a); }

__global__ void __launch_bounds__(NTT_THREADS) __attribute__((amdgpu_waves_per_eu(4)))
ntt_pass_kernel_r2(NttPass a) {
  ntt_pass_body<2>(a);
}

// Ladder of in-tile twiddles: ladder[2^(k-1) + j] = omega_(2^k)^j for
// j < 2^(k-1), k = 1 .. TILE_LOG, gathered from a "hi" table
// (hi[e] = omega_(2^28)^(e 2^14), so omega_(2^k)^j = hi[j 2^(14-k)]).
__global__ void ladder_kernel(const f29* __restrict__ hi, f29* __restrict__ ladder) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx == 0 || idx >= TILE) return;
  const uint32_t k = 32 - __clz(idx);  // 2^(k-1) <= idx < 2^k
  const uint32_t j = idx - (1u << (k - 1));
  ladder[idx] = hi[j << (14 - k)];
}

// out[l 2^14 + e] = lo[e] * scales[l], canonical.
__global__ void scale_tables_kernel(const f29* __restrict__ lo, const f29* __restrict__ scales, uint32_t nscales,
                                    f29* __restrict__ out) {
  const uint32_t idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (nscales << 14)) return;
  out[idx] = reduce_full<FrP>(mont_mul<FrP>(lo[idx & 0x3fffu], scales[idx >> 14]));
}

// Entry i = i1 2^mA + k2 of a first pass's post twiddles: omega_(2^L)^(i1 k2),
// limb l at out[l 2^L + i].
__global__ void full_tw_kernel(const f29* __restrict__ lo, const f29* __restrict__ hi, uint32_t scaled, uint32_t L,
                               uint32_t mA, uint32_t* __restrict__ out) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (1u << L)) return;
  const uint32_t ex = ((i >> mA) * (i & ((1u << mA) - 1))) & ((1u << L) - 1);
  const f29 w = pow28(lo, hi, ex << (28 - L), scaled != 0);
#pragma unroll
  for (int l = 0; l < 9; l++) out[((size_t)l << L) + i] = w.l[l];
}

// lo[e] = base^e, hi[e] = base^(e * 2^14) for e < 2^14 (Montgomery form).
__global__ void pow_tables_kernel(Words8 bw, f29* lo, f29* hi) {
  const uint32_t e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (1u << 14)) return;
  const f29 base = reduce_full<FrP>(to_mont<FrP>(unpack(bw.w)));
  uint32_t ex[8] = {e, 0, 0, 0, 0, 0, 0, 0};
  lo[e] = e ? reduce_full<FrP>(mont_pow<FrP>(base, ex)) : f29_from(FrP::ONE);
  ex[0] = e << 14;
  hi[e] = e ? reduce_full<FrP>(mont_pow<FrP>(base, ex)) : f29_from(FrP::ONE);
}

}  // namespace

size_t ntt_pass_lds_bytes() { return (size_t)(TILE + TILE / 8 + 1) * 32; }

hipError_t ntt_launch_pass(const NttPass& p, hipStream_t s) {
  const uint32_t blocks = (p.nbatch + p.G - 1) / p.G;
  // LDS and threads sized to the tile: 2048-point tiles (74 KB) let two
  // workgroups share a CU, so one's loads and stores overlap the other's
  // butterflies (1024-point tiles let four share it)
  const uint32_t te = (1u << p.m) * p.G;
  const bool r2 = p.unit_log == 2;
  uint32_t threads = te / (r2 ? 4 : 8);
  if (threads < 64) threads = 64;
  if (threads > NTT_THREADS) threads = NTT_THREADS;
  if (p.zero_log > p.m) return hipErrorInvalidValue;
  const ProfToken t = prof_begin("ntt.pass", s);
  if (r2)
    hipLaunchKernelGGL(ntt_pass_kernel_r2, dim3(blocks), dim3(threads), (size_t)(te + te / 8 + 1) * 32, s, p);
  else
    hipLaunchKernelGGL(ntt_pass_kernel, dim3(blocks), dim3(threads), (size_t)(te + te / 8 + 1) * 32, s, p);
  prof_end(t, s);
  return hipGetLastError();
}

hipError_t ntt_pass_setup() {
  hipError_t e = hipFuncSetAttribute((const void*)ntt_pass_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)ntt_pass_lds_bytes());
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute((const void*)ntt_pass_kernel_r2, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ntt_pass_lds_bytes());
}

hipError_t ntt_make_pow_tables(Words8 base, f29* lo, f29* hi, hipStream_t s) {
  hipLaunchKernelGGL(pow_tables_kernel, dim3((1u << 14) / 256), dim3(256), 0, s, base, lo, hi);
  return hipGetLastError();
}

uint32_t ntt_tile_log() { return TILE_LOG; }

hipError_t ntt_full_twiddles(const f29* lo, const f29* hi, uint32_t scaled, uint32_t L, uint32_t mA, uint32_t* out,
                             hipStream_t s) {
  if (L == 0 || L > 28 || mA > L) return hipErrorInvalidValue;
  const uint32_t n = 1u << L;
  hipLaunchKernelGGL(full_tw_kernel, dim3((n + 255) / 256), dim3(256), 0, s, lo, hi, scaled, L, mA, out);
  return hipGetLastError();
}

size_t ntt_ladder_entries() { return TILE; }

hipError_t ntt_scale_tables(const f29* lo, const f29* scales, uint32_t nscales, f29* out, hipStream_t s) {
  if (nscales == 0) return hipSuccess;
  hipLaunchKernelGGL(scale_tables_kernel, dim3((nscales << 14) / 256), dim3(256), 0, s, lo, scales, nscales, out);
  return hipGetLastError();
}

hipError_t ntt_make_ladder(const f29* hi, f29* ladder, hipStream_t s) {
  hipLaunchKernelGGL(ladder_kernel, dim3(TILE / 256), dim3(256), 0, s, hi, ladder);
  return hipGetLastError();
}

}  // namespace zk
