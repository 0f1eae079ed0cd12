/* zk.h -- C ABI of the MI355X (gfx950) KZG commit / fold hot path.
 *
 * What the library computes, after the ZKTorch paper ("Compiling ML Inference
 * to Zero-Knowledge Proofs via Parallel Proof Accumulation"):
 *
 *  - KZG commitment (Preliminaries, Polynomial Commitment): com = [f(tau)]_1,
 *    which for coefficients f_i and the SRS [tau^i]_1 is the multi-scalar
 *    multiplication sum_i f_i [tau^i]_1 over G1 of BN254 (the curve fixed by
 *    the Experimental Setup).  zk_msm, zk_msm_srs, zk_msm_batch.
 *  - KZG setup (same section): the SRS [tau^0]_1, [tau^1]_1, ... for a known
 *    trapdoor.  zk_srs_setup (test and benchmark use; deployments load a
 *    ceremony's points and call zk_srs_create).
 *  - Witness encoding (Foldable basic blocks): a length-n vector is the
 *    evaluations of its polynomial on H = {omega^i}, element i = f(omega^i).
 *    zk_intt turns evaluations into coefficients, zk_ntt the reverse, and
 *    zk_coset_ntt evaluates on a coset of a larger domain, as the quotients by
 *    X^n - 1 of the Mul block and the Poly-IOP require.
 *  - Accumulation (Parallel Accumulation, prover step 5): the random linear
 *    combination gamma * v + v' of the G1 commitments of two instances, run
 *    as a tree over m instances.  zk_fold.
 *
 * Conventions
 *  - zk_fr: an element of the BN254 scalar field Fr, 8 little-endian 32-bit
 *    words, canonical (value < r).
 *  - zk_g1: an affine G1 point, x then y, each 8 little-endian words,
 *    canonical (< p).  The point at infinity is (0, 0) (not on the curve).
 *  - Roots of unity: omega_N = 5^((r-1)/N); natural order in and out.
 *  - Every array argument is a DEVICE pointer owned by the caller, unless its
 *    name ends in _host.  The library keeps no pointer to caller memory after
 *    the enqueued work completes.
 *  - stream: a hipStream_t (NULL: the null stream).  Calls enqueue work and
 *    return; results are ready when the stream reaches that point.
 *  - Scratch memory comes from a library cache of device blocks: a block
 *    freed by a call is reused by later calls (on another stream only after
 *    that stream waits on the block's last use); hipMalloc runs only when no
 *    cached block fits.  zk_release_cached_memory() returns the cache.
 *  - The first call on a device builds that device's constant tables (NTT
 *    twiddles, including per-size four-step twiddle tables, about 0.65 GB,
 *    and the SRS generator table), held until the process ends; they are
 *    outside the scratch cache and its budget.
 *  - Return: ZK_OK, or a negative code with a message in zk_last_error().
 *    Argument errors are detected before anything is enqueued.  A failed
 *    launch or allocation returns ZK_EDEVICE / ZK_ENOMEM; nothing aborts.
 */
#ifndef ZK_H
#define ZK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct zk_fr {
  uint32_t v[8];
} zk_fr;

typedef struct zk_g1 {
  uint32_t x[8];
  uint32_t y[8];
} zk_g1;

/* An affine G2 point: x = x0 + x1 u, y = y0 + y1 u in Fq2 = Fq[u]/(u^2 + 1),
 * each component 8 little-endian words, canonical (< p).  The point at
 * infinity is all zeros. */
typedef struct zk_g2 {
  uint32_t x0[8];
  uint32_t x1[8];
  uint32_t y0[8];
  uint32_t y1[8];
} zk_g2;

typedef int zk_status;
#define ZK_OK 0
#define ZK_EINVAL (-1)      /* bad argument (NULL, size out of range, ...)   */
#define ZK_ENOMEM (-2)      /* device allocation failed                      */
#define ZK_EDEVICE (-3)     /* HIP runtime / kernel launch error             */
#define ZK_EBUDGET (-4)     /* scratch would exceed zk_set_scratch_budget    */
#define ZK_EUNSUPPORTED (-5) /* valid request outside the library's limits  */

/* Largest transform: log_n (+ log_blowup) <= ZK_MAX_LOG_NTT. */
#define ZK_MAX_LOG_NTT 28

/* Prepared SRS: the points in the kernels' Montgomery form plus, for every
 * Pippenger window w, the points multiplied by 2^(c w).  Opaque. */
typedef struct zk_srs zk_srs;

/* Message for the last failed call on this thread ("" if none). */
const char* zk_last_error(void);

/* Forward transform of 2^log_n coefficients:
 *   out[k] = sum_i in[i] omega^(i k),  omega = omega_(2^log_n).
 * in == out is allowed.  log_n <= ZK_MAX_LOG_NTT. */
zk_status zk_ntt(const zk_fr* in, zk_fr* out, uint32_t log_n, void* stream);

/* Inverse transform (evaluations on H -> coefficients):
 *   out[i] = n^-1 sum_k in[k] omega^(-i k).  in == out is allowed. */
zk_status zk_intt(const zk_fr* in, zk_fr* out, uint32_t log_n, void* stream);

/* Coset evaluation of the polynomial with 2^log_n coefficients `coeffs` on
 * g * H_(N), N = 2^(log_n + log_blowup):
 *   out[j] = f(g omega_N^j), j < N;  out has N elements.
 * shift_host: g as a host zk_fr, or NULL for g = 5 (outside every H_N).
 * coeffs must not overlap out.  log_n + log_blowup <= ZK_MAX_LOG_NTT. */
zk_status zk_coset_ntt(const zk_fr* coeffs, uint32_t log_n, uint32_t log_blowup, const zk_fr* shift_host,
                       zk_fr* out, void* stream);

/* Multi-scalar multiplication with arbitrary bases:
 *   *out = sum_{i<n} scalars[i] * bases[i]   (scalars as integers < r).
 * bases may contain (0, 0).  n = 0 gives (0, 0).  out: one zk_g1. */
zk_status zk_msm(const zk_g1* bases, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream);

/* KZG setup for a known trapdoor: out[i] = [tau^i]_1 = tau^i G, i < n,
 * G = (1, 2).  tau_host: host zk_fr. */
zk_status zk_srs_setup(const zk_fr* tau_host, uint64_t n, zk_g1* out, void* stream);

/* KZG setup in the Lagrange basis of H = {omega^j : j < n}, n = 2^log_n, for
 * a known trapdoor (Polynomial Commitment: srs; the vector encoding of
 * Foldable basic blocks): out[j] = [l_j(tau)]_1, where l_j is the polynomial
 * of degree < n with l_j(omega^i) = 1 if i = j and 0 otherwise.  A vector v
 * of evaluations on H then commits as sum_j v_j out[j] = [f(tau)]_1 for the
 * interpolant f of v: zk_msm_srs over an SRS prepared from these points
 * commits evaluations directly, without the inverse NTT, and small entries
 * (quantized activations) stay small scalars.  A prefix of m < n points is
 * not a Lagrange basis of a smaller domain: commit vectors of length n
 * (shorter vectors are read as zero-padded to n).  out: n zk_g1.  Test and
 * benchmark use; deployments load a ceremony's Lagrange-form points and call
 * zk_srs_create. */
zk_status zk_srs_lagrange_setup(const zk_fr* tau_host, uint32_t log_n, zk_g1* out, void* stream);

/* Prepare an SRS (any n affine points, e.g. from zk_srs_setup or a
 * ceremony) for commitments.  Allocates 16 * 64 * n bytes (the points times
 * 2^(16 w), w < 16), 22 * 64 * min(n, 2^16) bytes (times 2^(12 w), for
 * small commitments), 32768 * min(n, 4096) bytes (the small multiples of
 * zk_srs_set_tiny_max) and, for n >= 2^21, 13 * 64 * n bytes (times 2^(20 w))
 * of device memory owned by the handle; the work is enqueued on `stream`.
 * The handle is bound to the current device. */
zk_status zk_srs_create(const zk_g1* points, uint64_t n, zk_srs** srs, void* stream);

/* Release a prepared SRS (synchronises the device first). */
zk_status zk_srs_destroy(zk_srs* srs);

/* Number of points of a prepared SRS (0 for NULL). */
uint64_t zk_srs_size(const zk_srs* srs);

/* Table policy of a prepared SRS (which pre-shifted table, hence which
 * window size, serves an n-point commitment): n < small_max uses the 12-bit
 * windows of the first 2^16 points, n >= large_min the 20-bit windows (only
 * when that table was built, i.e. zk_srs_size >= 2^21), anything else the
 * 16-bit windows.  Defaults: 0 and 2^21, the autotuner's measurement on
 * MI355X (paper_2507_07031_amd/autotune.py times each table per size on the
 * running device and sets measured thresholds).  The result of a
 * commitment does not depend on the policy.  small_max <= 2^16, else
 * ZK_EINVAL.  Set it while no call on this SRS is being enqueued. */
zk_status zk_srs_set_table_policy(zk_srs* srs, uint64_t small_max, uint64_t large_min);

/* Small commitments (§2.1, the KZG commitment [f(tau)]_1 = sum_i f_i
 * [tau^i]_1, for few coefficients): an n-point commitment with
 * 0 < n <= tiny_max runs on the handle's table of small multiples
 * m 16^w [tau^i]_1 (m = 1..8, w < 64, i < min(zk_srs_size, 4096): 32 KB per
 * point, built by zk_srs_create), one table point per nonzero signed 4-bit
 * digit summed by trees, instead of a bucket (Pippenger) run; the result
 * is the same.  Default 4096; 0 turns the path off.  tiny_max <= 4096, else
 * ZK_EINVAL.  Set it while no call on this SRS is being enqueued. */
zk_status zk_srs_set_tiny_max(zk_srs* srs, uint64_t tiny_max);

/* Window bits the policy picks for an n-point commitment (4 on the
 * small-multiples table, else 12, 16 or 20), or 0 for NULL /
 * n > zk_srs_size. */
uint32_t zk_srs_window_bits(const zk_srs* srs, uint64_t n);

/* Launch schedule of the MSM and transform kernels on the current device:
 * the knobs paper_2507_07031_amd/autotune.py tunes besides the table policy.
 * No result depends on them, only times.  In zk_set_schedule a field of 0
 * keeps the built-in value (and a NULL schedule restores every default);
 * zk_get_schedule returns the values in effect.  Set while no call on the
 * device is being enqueued.
 *  acc_max_slice      most sorted (bucket, point) entries one accumulating
 *                     thread takes per round of workgroups, 16..4096 (256)
 *  acc_blocks_per_cu  accumulation workgroups per compute unit and round, 1..4 (2)
 *  reduce_chunk       buckets per chunk of the running-sum bucket reduction,
 *                     a power of two <= 64 (built-in: 4, 8 or 16 by bucket count)
 *  sort_chunk         scalars per coarse-sort workgroup, a power of two in
 *                     256..16384 (1024)
 *  sort_bin_entries   entries per coarse bin the two-level bucket sort aims
 *                     at, a power of two in 2^10..2^20 (2^15)
 *  ntt_tile_log       preferred transform tile, 10, 11 or 12 (2^10, 2^11 or
 *                     2^12 points, used where both passes' transforms fit
 *                     it, else the smallest tile that holds them) (11)
 *  ntt_unit_log       transform stages per LDS round trip: 3 (each thread
 *                     holds 8 points) or 2 (4 points, more threads) (3)
 *  ntt_overlap_tile_log  tile of a transform the library runs beside other
 *                     kernels (zk_commit_job's coset transform beside the
 *                     MSM's reduction), 10, 11 or 12 (11)
 * ZK_EINVAL for a value out of range (nothing is changed then). */
typedef struct zk_schedule {
  uint32_t acc_max_slice;
  uint32_t acc_blocks_per_cu;
  uint32_t reduce_chunk;
  uint32_t sort_chunk;
  uint32_t sort_bin_entries;
  uint32_t ntt_tile_log;
  uint32_t ntt_unit_log;
  uint32_t ntt_overlap_tile_log;
} zk_schedule;
zk_status zk_set_schedule(const zk_schedule* schedule_host);
zk_status zk_get_schedule(zk_schedule* schedule_host);

/* KZG commitment to coefficients: *out = sum_{i<n} scalars[i] [tau^i]_1 over
 * the first n points of the prepared SRS (n <= zk_srs_size(srs)). */
zk_status zk_msm_srs(const zk_srs* srs, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream);

/* One commit job on a witness vector (Polynomial Commitment preliminaries;
 * the vector is its polynomial's evaluations on H, Sec. 4.4.1):
 *   coeffs     = iNTT(evals)                       (2^log_n elements)
 *   commitment = sum_i coeffs_i [tau^i]_1          (2^log_n <= zk_srs_size)
 *   coset      = f(g omega_(2^(log_n+log_blowup))^j), j < 2^(log_n+log_blowup),
 * as zk_intt, zk_msm_srs and zk_coset_ntt would give (shift_host NULL: g = 5).
 * The library overlaps the parts on a companion stream of `stream`: the
 * coset transform runs there beside the MSM's latency-bound reduction (it
 * starts once the bucket accumulation is enqueued).  All results are ordered
 * on `stream` when the call's work there completes.  evals and coeffs may alias; the other
 * buffers must not overlap. */
zk_status zk_commit_job(const zk_srs* srs, const zk_fr* evals, uint32_t log_n, uint32_t log_blowup,
                        const zk_fr* shift_host, zk_fr* coeffs, zk_g1* commitment, zk_fr* coset, void* stream);

/* zk_msm_srs for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and result as zk_msm_srs (the commitment sum_{i<n} scalars[i]
 * [tau^i]_1 over the first n prepared points, n = 0 gives (0, 0)).  Its
 * scratch is a fixed 128 MiB device array in the library, one copy per GPU,
 * held until the process ends; the call makes no allocation, no memset and
 * no host synchronisation (unless zk_set_validate is on), so a sequence of
 * such calls can be captured into a HIP graph (profiling off; the first call
 * in the process should run before capture starts).
 *  - Limit: the MSM's scratch must fit the array: up to 2^18 points under the
 *    default table policy.  A larger n returns ZK_EUNSUPPORTED, with the
 *    needed and available bytes in zk_last_error; use zk_msm_srs then.
 *  - Every call on one GPU shares that GPU's array: calls that overlap in
 *    time (on different streams, or from different threads) race and give
 *    wrong results.  Calls ordered on one stream are safe.  Each call clears
 *    what it needs; nothing carries over between calls.
 *  - The current device must be the SRS's device (ZK_EINVAL otherwise). */
zk_status zk_msm_srs_noalloc(const zk_srs* srs, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream);

/* zk_msm_srs that also records `accumulate_done_event` (a hipEvent_t, may be
 * NULL) on `stream` as soon as its bucket-accumulation kernel is enqueued.
 * What follows on the stream is a latency-bound reduction that leaves most
 * compute units idle: independent work (e.g. the same polynomial's coset
 * evaluation) made to wait on this event on another stream overlaps it. */
zk_status zk_msm_srs_ex(const zk_srs* srs, const zk_fr* scalars, uint64_t n, zk_g1* out, void* stream,
                        void* accumulate_done_event);

/* Device scratch (bytes) that zk_msm_srs takes from the stream-ordered pool
 * for an n-point commitment (srs NULL: a 16-bit-window SRS of n points), and
 * that zk_ntt / zk_intt / zk_coset_ntt take for a 2^log_n-point transform.
 * Host-only queries, for admission control by memory budget; 0 if the size
 * is out of range. */
uint64_t zk_msm_srs_workspace_bytes(const zk_srs* srs, uint64_t n);
uint64_t zk_ntt_workspace_bytes(uint32_t log_n);

/* `batch` commitments over prefixes of one prepared SRS:
 *   out[b] = sum_{i < n_b} scalars[offsets_host[b] + i] [tau^i]_1,
 *   n_b = offsets_host[b+1] - offsets_host[b] <= zk_srs_size(srs).
 * offsets_host: host array of batch + 1 non-decreasing entries, the first 0. */
zk_status zk_msm_batch(const zk_srs* srs, const zk_fr* scalars, const uint64_t* offsets_host, uint32_t batch,
                       zk_g1* out, void* stream);

/* KZG opening (Preliminaries, Polynomial Commitment: open): for the
 * polynomial f with n coefficients `coeffs` (lowest degree first) and the
 * point x,
 *   *y     = f(x),
 *   q(X)   = (f(X) - y) / (X - x)            (n - 1 coefficients),
 *   *proof = [q(tau)]_1 = sum_i q_i [tau^i]_1 over the prepared SRS,
 * so that the verifier's pairing check e(proof, [tau - x]_2) =
 * e(com - [y]_1, [1]_2) holds for com = [f(tau)]_1.
 *   x_host:   host zk_fr (canonical; any value, also one in a domain H).
 *   y:        one device zk_fr.          proof: one device zk_g1.
 *   quotient: device array of n - 1 zk_fr that receives q, or NULL (the
 *             quotient then lives in library scratch only).
 * Requires n - 1 <= zk_srs_size(srs).  n = 0 (the zero polynomial) gives
 * y = 0 and proof = (0, 0); n = 1 gives y = coeffs[0] and proof = (0, 0).
 * No buffer may overlap another. */
zk_status zk_kzg_open(const zk_srs* srs, const zk_fr* coeffs, uint64_t n, const zk_fr* x_host, zk_fr* y,
                      zk_fr* quotient, zk_g1* proof, void* stream);

/* Batched KZG opening at one point (same passage: the prover sends every
 * f_i(x), then one proof for the verifier's challenge gamma):
 *   ys[i]  = f_i(x),  i < m,
 *   h(X)   = sum_i gamma^i (f_i(X) - ys[i]) / (X - x)   (n - 1 coefficients),
 *   *proof = [h(tau)]_1.
 * polys: m polynomials of n coefficients each, polys[i * n + j] (pad a
 * shorter polynomial with zero high coefficients).  gamma_host: host zk_fr,
 * ignored (may be NULL) when m = 1.  ys: m device zk_fr.  quotient: as for
 * zk_kzg_open (receives h).  The verifier's check is
 * e(proof, [tau - x]_2) = e(sum_i gamma^i (com_i - [ys[i]]_1), [1]_2). */
zk_status zk_kzg_open_batch(const zk_srs* srs, const zk_fr* polys, uint32_t m, uint64_t n, const zk_fr* x_host,
                            const zk_fr* gamma_host, zk_fr* ys, zk_fr* quotient, zk_g1* proof, void* stream);

/* Quotient of the Mul basic block (Foldable basic blocks, Mul): for witness
 * vectors a, b, c on H (n = 2^log_n elements each, c_i = a_i b_i) with
 * interpolants f, h, g (element i = value at omega^i),
 *   t(X) = (f(X) h(X) - g(X)) / (X^n - 1)          (degree <= n - 2),
 *   t_coeffs[i] = t_i, i < n (t_coeffs[n - 1] = 0),
 *   *t_commit   = [t(tau)]_1 over the first n SRS points.
 * Computed on the coset s H_(B n), B = 2^log_blowup (1 <= log_blowup <= 4;
 * B = 2 is enough for this degree): the coset evaluations of f, h, g, the
 * pointwise (f h - g) / (X^n - 1) (B distinct divisor values), the inverse
 * coset transform, then the commitment.  shift_host: s as a host zk_fr, or
 * NULL for s = 5; a shift whose coset meets a root of X^n - 1 is rejected.
 * If c is not the entrywise product of a and b there is no such quotient:
 * the result is then the interpolant of (f h - g) / (X^n - 1) on the coset.
 * Requires n <= zk_srs_size(srs) and log_n + log_blowup <= ZK_MAX_LOG_NTT.
 * Scratch: 32 (n + 3 B n) bytes from the library cache. */
zk_status zk_quotient_mul(const zk_srs* srs, const zk_fr* a, const zk_fr* b, const zk_fr* c, uint32_t log_n,
                          uint32_t log_blowup, const zk_fr* shift_host, zk_fr* t_coeffs, zk_g1* t_commit,
                          void* stream);

/* One term c * x_a * x_b * ... of a Poly-IOP constraint R (Basic blocks based
 * on a Poly-IOP): factor index a < N names the witness polynomial f_a(x),
 * N <= a < 2N names f_(a-N)(omega x); nfactors = 0 is the constant c. */
#define ZK_POLYIOP_MAX_WITNESS 8
#define ZK_POLYIOP_MAX_TERMS 16
#define ZK_POLYIOP_MAX_DEGREE 4
typedef struct zk_constraint_term {
  zk_fr coeff;                             /* canonical                      */
  uint32_t nfactors;                       /* 0 .. ZK_POLYIOP_MAX_DEGREE     */
  uint32_t factor[ZK_POLYIOP_MAX_DEGREE];  /* each < 2N; unused slots ignored */
} zk_constraint_term;

/* Quotient of a Poly-IOP constraint (Basic blocks based on a Poly-IOP,
 * protocol step 1): for N witness vectors on H, evals[k * n + i] =
 * f_k(omega^i) (n = 2^log_n, 1 <= N <= ZK_POLYIOP_MAX_WITNESS), and R the
 * sum of the nterms terms (1 .. ZK_POLYIOP_MAX_TERMS) of degree d (the
 * largest nfactors),
 *   Q(X)        = R(f_0(X), .., f_(N-1)(X), f_0(omega X), .., f_(N-1)(omega X)) / (X^n - 1),
 *   q_coeffs[i] = Q_i, i < max(d - 1, 1) n    (deg Q <= d (n - 1) - n),
 *   *q_commit   = [Q(tau)]_1 over the first max(d - 1, 1) n SRS points.
 * The paper's instances: BooleanCheck (N = 1, R = x_0 - x_0^2), Sub Check
 * (N = 2, R = x_1 + x_0 - x_2), i-thIsZero (N = 2, R = x_0 x_1).
 * Computed on the coset s H_(B n), B = 2^log_blowup (1 <= log_blowup <= 4,
 * B >= d): the coset evaluations of every f_k, the pointwise R / (X^n - 1)
 * (f_k(omega x) at coset point j is point j + B of the same coset vector;
 * X^n - 1 takes B distinct values there), the inverse coset transform and
 * the commitment.  shift_host: s as a host zk_fr, or NULL for s = 5; a
 * shift whose coset meets a root of X^n - 1 is rejected.  If the witnesses
 * do not satisfy R on H there is no such Q: the result is then the
 * interpolant of R / (X^n - 1) on the coset, cut to the length above.  The
 * paper's blinding f + (X^n - 1) b is not applied (the caller's witnesses
 * carry it).  terms_host: host array.  ZK_EINVAL for counts, indices or a
 * blowup out of range, or an SRS shorter than the quotient.  Scratch:
 * 32 (n + (N + 1) B n) bytes from the library cache. */
zk_status zk_quotient_polyiop(const zk_srs* srs, const zk_fr* evals, uint32_t N, uint32_t log_n,
                              const zk_constraint_term* terms_host, uint32_t nterms, uint32_t log_blowup,
                              const zk_fr* shift_host, zk_fr* q_coeffs, zk_g1* q_commit, void* stream);

/* Fiat-Shamir challenge from a transcript (the random oracles rho_acc and
 * rho_NARK of Parallel Accumulation, which the paper leaves unspecified):
 *   *challenge = (SHA-256(0x00 || data) || SHA-256(0x01 || data)) mod r,
 * the two 32-byte digests read as one 512-bit little-endian integer (SHA-256
 * as FIPS 180-4 defines it).  data: `bytes` bytes of device memory (e.g.
 * the instances' commitments, E terms and Fr parts, as stored); challenge:
 * one device zk_fr, usable directly as zk_acc_fold's gamma.  One workgroup;
 * meant for transcripts of kilobytes. */
zk_status zk_transcript_challenge(const void* data, uint64_t bytes, zk_fr* challenge, void* stream);

/* One step of the accumulation prover (Parallel Accumulation, prover steps
 * 5-6) on the device parts of two accumulators: acc = (C, E, v, e), weighted
 * by gamma, and acc' = (C2, E2, v2, e2), with the correction terms E_j and
 * the error vectors e_j of the relation of degree d (1 <= d <= 15):
 *   C_out[i] = gamma C[i] + C2[i],                         i < k
 *   *E_out   = E2 + sum_(j=1)^(d-1) gamma^j Ej[j-1] + gamma^d E
 *   v_out[i] = gamma v[i] + v2[i],                         i < len_v
 *              (the Fr parts mu, pi, r_i, m_i, concatenated by the caller)
 *   e_out[i] = e2[i] + sum_(j=1)^(d-1) gamma^j ej[(j-1) len_e + i] + gamma^d e[i]
 * G1 arguments are zk_g1 arrays ((0, 0) = infinity), Fr arguments zk_fr
 * arrays, gamma one device zk_fr (e.g. from zk_transcript_challenge).  Ej
 * and ej may be NULL when d = 1; Fr parts of length 0 may be NULL.  The
 * new mu'' = gamma mu + mu' is the first element of v_out when mu leads v.
 * Outputs must not overlap inputs. */
zk_status zk_acc_fold(uint32_t k, const zk_g1* C, const zk_g1* C2, uint32_t d, const zk_g1* E, const zk_g1* E2,
                      const zk_g1* Ej, uint64_t len_v, const zk_fr* v, const zk_fr* v2, uint64_t len_e,
                      const zk_fr* e, const zk_fr* e2, const zk_fr* ej, const zk_fr* gamma, zk_g1* C_out,
                      zk_g1* E_out, zk_fr* v_out, zk_fr* e_out, void* stream);

/* Commitments in G2 (Preliminaries: [x]_2 = x H; MulScalar's s', Mul's h',
 * MatMul's B' and D' are G2 commitments): G2 is the order-r subgroup of the
 * BN254 twist y^2 = x^3 + 3/(9 + u) over Fq2, H its usual generator
 * (x = 0x1800deef...c2 + 0x198e9393...ed u as in Ethereum's precompiles).
 *
 * zk_srs_g2_setup: out[i] = [tau^i]_2 = tau^i H, i < n, for a known trapdoor
 * (test and benchmark use).  zk_srs_g2_create prepares n G2 points (with
 * zk_set_validate on: checked canonical, on the twist and of order r) with
 * 32 * 128 * n bytes of pre-shifted table owned by the handle;
 * zk_msm_g2_srs: *out = sum_{i<n} scalars[i] P_i over the first n prepared
 * points (n <= zk_srs_g2_size), n = 0 gives infinity.  n < 2^26. */
typedef struct zk_srs_g2 zk_srs_g2;
zk_status zk_srs_g2_setup(const zk_fr* tau_host, uint64_t n, zk_g2* out, void* stream);
zk_status zk_srs_g2_create(const zk_g2* points, uint64_t n, zk_srs_g2** srs, void* stream);
zk_status zk_srs_g2_destroy(zk_srs_g2* srs);
uint64_t zk_srs_g2_size(const zk_srs_g2* srs);
zk_status zk_msm_g2_srs(const zk_srs_g2* srs, const zk_fr* scalars, uint64_t n, zk_g2* out, void* stream);

/* Fold m instances of k G1 commitments each (inst[i*k + j]) into one:
 * the tree of pairwise folds gamma * left + right (adjacent pairs per level,
 * an odd last instance carried up, challenges consumed level by level, left
 * to right: gammas[0..m-2]).  m = 2 is exactly out[j] = gamma*inst[j] +
 * inst[k + j].  out: k points.  m >= 1. */
zk_status zk_fold(const zk_g1* inst, const zk_fr* gammas, uint32_t m, uint32_t k, zk_g1* out, void* stream);

/* Input validation (off by default).  When on, every call checks on the
 * device, before any other work, that its Fr inputs are canonical (< r) and
 * its G1 inputs are (0, 0) or canonical affine points on y^2 = x^3 + 3, and
 * returns ZK_EINVAL (message in zk_last_error) if one is not; G2 inputs
 * must be all zeros or canonical points of order r on the twist.  The check
 * waits for the call's stream, so validated calls are synchronous. */
zk_status zk_set_validate(int on);

/* Wait for and free every cached scratch block of the current device. */
zk_status zk_release_cached_memory(void);

/* HBM budget for the library's scratch on the current device (for callers
 * that admit work by memory, such as a serving loop; 0, the default, is no
 * cap).  The budget covers every scratch block the library holds there,
 * cached ones included.  When a call needs a new block that would take the
 * total over the budget, the library first frees the device's cached blocks
 * (waiting for their last use); if the block still does not fit, the call
 * returns ZK_EBUDGET.  A call's scratch is taken before its kernels are
 * enqueued, so a call failing this way has enqueued no work of its own
 * except, for calls that allocate in stages, stages that precede the
 * failing allocation (its outputs are then unspecified).  Caller buffers
 * are not counted.  Lowering the budget frees nothing by itself. */
zk_status zk_set_scratch_budget(uint64_t bytes);

/* Scratch bytes the library holds on the current device, cached blocks
 * included (0 if there is no device). */
uint64_t zk_scratch_held(void);

/* Calibration of the integer-multiply roof: runs `blocks` workgroups of 256
 * threads, each thread 8 independent chains of iters * 16 dependent
 * v_mad_u64_u32 products (the only multiply of the Montgomery products), on
 * the current device and stream, and returns the sustained rate in products
 * per second (timed with events; synchronises the stream). */
zk_status zk_calibrate_mad_rate(uint32_t blocks, uint32_t iters, double* mads_per_s, void* stream);

/* Observability: when enabled, the library brackets named kernel regions
 * with HIP events recorded on the stream the kernels run on.  Regions:
 *   "msm.sort"        decompose + histogram + scan + counting-sort scatter
 *   "msm.accumulate"  the bucket-accumulation kernel (mixed additions)
 *   "msm.reduce"      record levels + bucket reduction + window combine
 *   "ntt.pass"        one LDS-tiled NTT pass (1 or 2 per transform)
 * zk_profile_read waits for the recorded regions named `region` and returns
 * the sum of their durations and their count; reset != 0 forgets them. */
zk_status zk_profile_enable(int on);
zk_status zk_profile_read(const char* region, double* total_ms, uint64_t* launches, int reset);
/* Record only the regions called `region` (NULL: every region).  Each
 * recorded region adds two timestamp events to its stream; timing one
 * region keeps that cost out of the others. */
zk_status zk_profile_only(const char* region);

#ifdef __cplusplus
}
#endif

#endif /* ZK_H */
