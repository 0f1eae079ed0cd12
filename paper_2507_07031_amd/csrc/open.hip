// KZG opening over Fr: the evaluation y = f(x) and the quotient
// q(X) = (f(X) - y) / (X - x) of the Polynomial Commitment opening, and the
// batched form at one point, where the numerator is sum_i gamma^i (f_i - f_i(x)).
//
// Division by the monic X - x is the first-order recurrence
//   Q_j = f_j + x Q_(j+1),  Q_n = 0,   q_(j-1) = Q_j (j >= 1),  y = Q_0,
// i.e. Q_j = sum_(k >= j) f_k x^(k - j), a suffix scan whose combining rule
// multiplies the right-hand part by x to the length of the left-hand part.
// It runs as a tiled scan in three launches:
//   1. tiles   every tile of T = 256 * 8 coefficients is evaluated at x
//              (L_b = sum_(k in tile) f_k x^(k - tile start)), for every
//              polynomial; with several polynomials the combination
//              g = sum_i gamma^i f_i is written alongside;
//   2. carries one workgroup per polynomial turns the tile values into
//              y_i = sum_b L_b x^(T b); one more (the only one for a single
//              polynomial) scans the tile values of g into the carry into
//              every tile, C_(b+1) = Q_((b+1) T), and tabulates the 64 lane
//              powers the apply launch's in-tile scan needs;
//   3. apply   every tile re-evaluates its chunks, combines them with its
//              carry, and runs the recurrence down through its coefficients,
//              writing the quotient.
// Inside a workgroup each thread owns 8 consecutive coefficients; the chunk
// values are combined by a suffix scan across the wave (lane shuffles) and a
// short Horner step across the four waves (LDS).
//
// Arithmetic: coefficients are plain canonical integers; x, gamma and their
// powers are Montgomery-form constants, so a Montgomery product with one
// yields the plain product.  Intermediate values stay below 16 r (sums of
// at most a few reduced products) and are made canonical at every store.
#include <utility>

#include "field.h"
#include "open.h"
#include "prof.h"

namespace zk {

namespace {

constexpr uint32_t OPEN_NT = 256;               // threads per workgroup (4 waves)
constexpr uint32_t OPEN_E = 8;                  // coefficients per thread
constexpr uint32_t OPEN_T = OPEN_NT * OPEN_E;   // coefficients per tile
constexpr uint32_t CARRY_NT = 256;

// f(0), f(1), ..., f(N - 1) with compile-time indices, so that per-thread
// arrays stay in registers (the loop bodies are too large for the unroller).
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

struct OpenArgs {
  f29 x;       // x (Montgomery form)
  f29 gamma;   // gamma (Montgomery form)
  f29 pw[7];   // x^(OPEN_E 2^l): chunk-to-chunk multipliers of the in-tile scan
};

struct CarryArgs {
  f29 X;       // x^OPEN_T: tile-to-tile multiplier
  f29 pw[7];   // X^(G 2^l)
  f29 xe[6];   // x^(OPEN_E 2^l): for the lane powers of the in-tile scan
  uint32_t G;  // tiles per thread
};

__device__ __forceinline__ void ld8(const uint32_t* p, uint32_t w[8]) {
  const uint4 a = reinterpret_cast<const uint4*>(p)[0];
  const uint4 b = reinterpret_cast<const uint4*>(p)[1];
  w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
  w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
}

__device__ __forceinline__ void st_canon(uint32_t* p, const f29& v) {
  uint32_t w[8];
  pack(reduce_full<FrP>(v), w);
  reinterpret_cast<uint4*>(p)[0] = make_uint4(w[0], w[1], w[2], w[3]);
  reinterpret_cast<uint4*>(p)[1] = make_uint4(w[4], w[5], w[6], w[7]);
}

__device__ __forceinline__ f29 shfl_down_f29(const f29& v, uint32_t d) {
  f29 r;
#pragma unroll
  for (int i = 0; i < 9; i++) r.l[i] = (uint32_t)__shfl_down((int)v.l[i], d, 64);
  return r;
}

__device__ __forceinline__ f29 mac(const f29& a, const f29& b, const f29& c) {
  return add_n(a, mont_mul<FrP>(b, c));  // a + b*c (c Montgomery form)
}

struct ScanOut {
  f29 carry;  // Q just after this thread's chunk (CARRY only)
  f29 total;  // Q at the workgroup's first position
};

// Workgroup of 4 waves; thread t holds h, the value of its chunk at the
// scan's multiplier b (chunks `per` positions long, in thread order), and
// pw[l] = b^(per 2^l).  `tail` is the value just after the last chunk.
// Returns the workgroup total (every thread) and, if CARRY, each thread's
// carry: the sum over later chunks and the tail, scaled to its chunk's end.
// lds: 4 elements, free on entry; the caller synchronises before reusing it.
// lane_pow (CARRY): b^(per (63 - lane)) for every lane, or nullptr to form
// it here from pw.
template <bool CARRY>
__device__ __forceinline__ ScanOut block_suffix(const f29& h, const f29 (&pw)[7], const f29& tail, f29* lds,
                                                const f29* lane_pow = nullptr) {
  const uint32_t lane = __lane_id(), wave = threadIdx.x >> 6;
  // inclusive suffix scan across the wave: S_t = sum_(k >= t) h_k b^(per (k - t))
  f29 S = h;
#pragma unroll
  for (int l = 0; l < 6; l++) {
    const uint32_t d = 1u << l;
    f29 o = shfl_down_f29(S, d);
    if (lane + d >= 64) o = f29_zero();
    S = mac(S, o, pw[l]);
  }
  if (lane == 0) lds[wave] = S;
  __syncthreads();
  // values at the wave boundaries, from the tail down
  f29 K = tail, Kw = tail;
#pragma unroll
  for (int w = 3; w >= 0; --w) {
    if ((uint32_t)w == wave) Kw = K;
    K = mac(lds[w], K, pw[6]);
  }
  ScanOut r;
  r.total = K;
  if (CARRY) {
    f29 nxt = shfl_down_f29(S, 1);
    if (lane == 63) nxt = f29_zero();
    f29 p;
    if (lane_pow) {
      p = lane_pow[lane];
    } else {
      // b^(per (63 - lane)) from the bits of 63 - lane
      const f29 one = f29_from(FrP::ONE);
      const uint32_t e = 63u - lane;
      p = one;
#pragma unroll
      for (int l = 0; l < 6; l++) p = mont_mul<FrP>(p, ((e >> l) & 1u) ? pw[l] : one);
    }
    r.carry = mac(nxt, Kw, p);
  } else {
    r.carry = f29_zero();
  }
  return r;
}

__device__ __forceinline__ f29 ld_coeff(const uint32_t* f, uint64_t j, uint64_t n) {
  if (j >= n) return f29_zero();
  uint32_t w[8];
  ld8(f + j * 8, w);
  return unpack(w);
}

// Launch 1.  Grid: one workgroup per tile.  tile_vals[i * nt + b] = L_b of
// polynomial i (canonical); BATCH (m > 1): g, the gamma combination of the
// coefficients, and its tile values sum_i gamma^i L_(i,b) in row m.
template <bool BATCH>
__global__ __launch_bounds__(OPEN_NT) void open_tiles_kernel(const uint32_t* __restrict__ polys, uint32_t m,
                                                             uint64_t n, OpenArgs a, f29* __restrict__ tile_vals,
                                                             uint32_t nt, uint32_t* __restrict__ g) {
  __shared__ f29 lds[2][4];
  const uint64_t s = (uint64_t)blockIdx.x * OPEN_T + (uint64_t)threadIdx.x * OPEN_E;
  f29 acc[OPEN_E];
  f29 lg = f29_zero();
  for (int32_t i = (int32_t)m - 1; i >= 0; --i) {
    const uint32_t* f = polys + (uint64_t)i * n * 8;
    f29 v[OPEN_E];
#pragma unroll
    for (uint32_t k = 0; k < OPEN_E; k++) v[k] = ld_coeff(f, s + k, n);
    f29 h = v[OPEN_E - 1];
    static_for<OPEN_E - 1>([&](auto c) { h = mac(v[OPEN_E - 2 - c], h, a.x); });
    const ScanOut r = block_suffix<false>(h, a.pw, f29_zero(), lds[i & 1]);
    if (threadIdx.x == 0) {
      const f29 li = reduce_full<FrP>(r.total);
      tile_vals[(uint64_t)i * nt + blockIdx.x] = li;
      if (BATCH) lg = (uint32_t)i == m - 1 ? li : mac(li, lg, a.gamma);
    }
    if (BATCH) {
      const bool first = (uint32_t)i == m - 1;
      static_for<OPEN_E>([&](auto k) { acc[k] = first ? v[k] : mac(v[k], acc[k], a.gamma); });
    }
  }
  if (BATCH) {
#pragma unroll
    for (uint32_t k = 0; k < OPEN_E; k++)
      if (s + k < n) st_canon(g + (s + k) * 8, acc[k]);
    if (threadIdx.x == 0) tile_vals[(uint64_t)m * nt + blockIdx.x] = reduce_full<FrP>(lg);
  }
}

// Tile value b of row `row` of tile_vals (zero past the last tile).
__device__ __forceinline__ f29 tile_value(const f29* tile_vals, uint32_t nt, uint32_t row, uint32_t b) {
  if (b >= nt) return f29_zero();
  return tile_vals[(uint64_t)row * nt + b];
}

// Launch 2.  Grid: m workgroups (y of each polynomial) plus, for m > 1, one
// for the carries of g (row m); with m == 1 workgroup 0 does both.  Thread t
// owns tiles [t G, t G + G).  The carry workgroup also writes lane_pow[t] =
// x^(OPEN_E (63 - t)), t < 64, for the apply launch's in-tile scan.
__global__ __launch_bounds__(CARRY_NT) void open_carry_kernel(const f29* __restrict__ tile_vals, uint32_t m,
                                                              uint32_t nt, CarryArgs a, f29* __restrict__ carry_in,
                                                              f29* __restrict__ lane_pow,
                                                              uint32_t* __restrict__ ys) {
  __shared__ f29 lds[4];
  const uint32_t poly = blockIdx.x;
  const uint32_t src = (m == 1) ? 0u : poly;  // poly == m: the combination
  const bool carries = (m == 1) || poly == m;
  const uint32_t b0 = threadIdx.x * a.G;
  f29 h = f29_zero();
  for (int32_t k = (int32_t)a.G - 1; k >= 0; --k) h = mac(tile_value(tile_vals, nt, src, b0 + k), h, a.X);
  ScanOut r;
  if (carries)
    r = block_suffix<true>(h, a.pw, f29_zero(), lds);
  else
    r = block_suffix<false>(h, a.pw, f29_zero(), lds);
  if (poly < m && threadIdx.x == 0) st_canon(ys + (uint64_t)poly * 8, r.total);
  if (carries) {
    f29 Q = r.carry;
    for (int32_t k = (int32_t)a.G - 1; k >= 0; --k) {
      const uint32_t b = b0 + k;
      if (b < nt) {
        carry_in[b] = reduce_full<FrP>(Q);
        Q = mac(tile_value(tile_vals, nt, src, b), Q, a.X);
      }
    }
    if (threadIdx.x < 64) {
      const f29 one = f29_from(FrP::ONE);
      const uint32_t e = 63u - threadIdx.x;
      f29 p = one;
      for (int l = 0; l < 6; l++) p = mont_mul<FrP>(p, ((e >> l) & 1u) ? a.xe[l] : one);
      lane_pow[threadIdx.x] = reduce_full<FrP>(p);
    }
  }
}

// Launch 3.  Grid: one workgroup per tile.  q[j - 1] = Q_j for 1 <= j < n.
__global__ __launch_bounds__(OPEN_NT) void open_apply_kernel(const uint32_t* __restrict__ f, uint64_t n, OpenArgs a,
                                                             const f29* __restrict__ carry_in,
                                                             const f29* __restrict__ lane_pow,
                                                             uint32_t* __restrict__ q) {
  __shared__ f29 lds[4];
  const uint64_t s = (uint64_t)blockIdx.x * OPEN_T + (uint64_t)threadIdx.x * OPEN_E;
  f29 v[OPEN_E];
#pragma unroll
  for (uint32_t k = 0; k < OPEN_E; k++) v[k] = ld_coeff(f, s + k, n);
  f29 h = v[OPEN_E - 1];
  static_for<OPEN_E - 1>([&](auto c) { h = mac(v[OPEN_E - 2 - c], h, a.x); });
  const ScanOut r = block_suffix<true>(h, a.pw, carry_in[blockIdx.x], lds, lane_pow);
  f29 Q = r.carry;
  static_for<OPEN_E>([&](auto c) {
    constexpr int k = OPEN_E - 1 - decltype(c)::value;
    Q = mac(v[k], Q, a.x);
    const uint64_t j = s + (uint64_t)k;
    if (j >= 1 && j < n) st_canon(q + (j - 1) * 8, Q);
  });
}

// Host: Montgomery form of a canonical value, and powers.
f29 host_mont(const uint32_t w[8]) { return reduce_full<FrP>(to_mont<FrP>(unpack(w))); }

f29 host_sq(const f29& a) { return reduce_full<FrP>(mont_mul<FrP>(a, a)); }

f29 host_pow(const f29& a, uint64_t e) {
  f29 r = f29_from(FrP::ONE), b = a;
  while (e) {
    if (e & 1) r = reduce_full<FrP>(mont_mul<FrP>(r, b));
    b = host_sq(b);
    e >>= 1;
  }
  return r;
}

uint32_t tiles_of(uint64_t n) { return (uint32_t)((n + OPEN_T - 1) / OPEN_T); }

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

size_t open_scratch_bytes(uint32_t m, uint64_t n) {
  const uint64_t nt = tiles_of(n);
  const uint64_t rows = m + (m > 1 ? 1 : 0);
  size_t b = align256(sizeof(f29) * (size_t)rows * nt) + align256(sizeof(f29) * (nt + 1)) + align256(sizeof(f29) * 64);
  if (m > 1) b += align256((size_t)n * 32);
  return b;
}

hipError_t open_quotient(const uint32_t* polys, uint32_t m, uint64_t n, const uint32_t x[8],
                         const uint32_t gamma[8], uint32_t* ys, uint32_t* q, void* scratch, hipStream_t s) {
  const uint32_t nt = tiles_of(n);
  char* p = static_cast<char*>(scratch);
  const uint64_t rows = m + (m > 1 ? 1 : 0);
  f29* tile_vals = reinterpret_cast<f29*>(p);
  p += align256(sizeof(f29) * (size_t)rows * nt);
  f29* carry_in = reinterpret_cast<f29*>(p);
  p += align256(sizeof(f29) * (nt + 1));
  f29* lane_pow = reinterpret_cast<f29*>(p);
  p += align256(sizeof(f29) * 64);
  uint32_t* g = m > 1 ? reinterpret_cast<uint32_t*>(p) : nullptr;

  OpenArgs a;
  a.x = host_mont(x);
  a.gamma = m > 1 ? host_mont(gamma) : f29_from(FrP::ONE);
  a.pw[0] = host_pow(a.x, OPEN_E);
  for (int l = 1; l < 7; l++) a.pw[l] = host_sq(a.pw[l - 1]);
  CarryArgs c;
  c.X = host_pow(a.x, OPEN_T);
  for (int l = 0; l < 6; l++) c.xe[l] = a.pw[l];
  c.G = nt ? (nt + CARRY_NT - 1) / CARRY_NT : 1;
  c.pw[0] = host_pow(c.X, c.G);
  for (int l = 1; l < 7; l++) c.pw[l] = host_sq(c.pw[l - 1]);

  const ProfToken tok = prof_begin("open.scan", s);
  if (nt) {
    if (m > 1)
      hipLaunchKernelGGL(open_tiles_kernel<true>, dim3(nt), dim3(OPEN_NT), 0, s, polys, m, n, a, tile_vals, nt, g);
    else
      hipLaunchKernelGGL(open_tiles_kernel<false>, dim3(nt), dim3(OPEN_NT), 0, s, polys, m, n, a, tile_vals, nt, g);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(open_carry_kernel, dim3(m + (m > 1 ? 1 : 0)), dim3(CARRY_NT), 0, s, tile_vals, m, nt, c,
                     carry_in, lane_pow, ys);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (nt && n > 1) {
    hipLaunchKernelGGL(open_apply_kernel, dim3(nt), dim3(OPEN_NT), 0, s, m > 1 ? g : polys, n, a, carry_in,
                       lane_pow, q);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  prof_end(tok, s);
  return hipSuccess;
}

}  // namespace zk
