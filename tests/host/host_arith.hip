// Host (CPU) build of the kernels' field and curve code, for CPU tests.
//
// Compiles the same __host__ __device__ functions the HIP kernels use into a
// plain x86 shared library, so the limb arithmetic, the lazy-reduction bounds
// and the point formulas can be checked against Python integers without a
// GPU.  Every entry point takes canonical little-endian 32-bit words.
#include <stdint.h>

#include "../../paper_2507_07031_amd/csrc/curve.h"
#include "../../paper_2507_07031_amd/csrc/g2.h"
#include "../../paper_2507_07031_amd/csrc/glv.h"

using namespace zk;

namespace {

template <class F>
f29 load_mont(const uint32_t w[8]) {
  return reduce_full<F>(to_mont<F>(unpack(w)));
}

template <class F>
void store_plain(const f29& a, uint32_t w[8]) {
  pack(from_mont<F>(a), w);
}

}  // namespace

extern "C" {

void host_fq_mul(const uint32_t* a, const uint32_t* b, uint32_t* out) {
  store_plain<FqP>(mont_mul<FqP>(load_mont<FqP>(a), load_mont<FqP>(b)), out);
}

void host_fq_sqr(const uint32_t* a, uint32_t* out) {
  store_plain<FqP>(mont_sqr<FqP>(load_mont<FqP>(a)), out);
}

void host_fq_inv(const uint32_t* a, uint32_t* out) {
  store_plain<FqP>(mont_inv<FqP>(load_mont<FqP>(a)), out);
}

// The batched binary GCD alone (no Fermat backup): returns 1 if it finished.
int host_fq_inv_bgcd(const uint32_t* a, uint32_t* out) { return inv_bgcd32<FqP>(a, out) ? 1 : 0; }
int host_fr_inv_bgcd(const uint32_t* a, uint32_t* out) { return inv_bgcd32<FrP>(a, out) ? 1 : 0; }

void host_fr_mul(const uint32_t* a, const uint32_t* b, uint32_t* out) {
  store_plain<FrP>(mont_mul<FrP>(load_mont<FrP>(a), load_mont<FrP>(b)), out);
}

// Raw limb access: products of arbitrary (already Montgomery) limb vectors.
void host_fq_mont_mul_raw(const uint32_t* a9, const uint32_t* b9, uint32_t* out9) {
  f29 a, b;
  for (int i = 0; i < 9; i++) {
    a.l[i] = a9[i];
    b.l[i] = b9[i];
  }
  f29 r = mont_mul<FqP>(a, b);
  for (int i = 0; i < 9; i++) out9[i] = r.l[i];
}

int host_fq_is_zero_mod(const uint32_t* a9) {
  f29 a;
  for (int i = 0; i < 9; i++) a.l[i] = a9[i];
  return is_zero_mod<FqP>(a) ? 1 : 0;
}

void host_fq_reduce_full(const uint32_t* a9, uint32_t* out9) {
  f29 a;
  for (int i = 0; i < 9; i++) a.l[i] = a9[i];
  f29 r = reduce_full<FqP>(a);
  for (int i = 0; i < 9; i++) out9[i] = r.l[i];
}

// sum of affine points (16 words each) by repeated mixed addition.
void host_g1_sum_madd(const uint32_t* pts, uint64_t n, uint32_t* out) {
  xyzz acc = xyzz_inf();
  for (uint64_t i = 0; i < n; i++) {
    aff p;
    if (aff_from_plain_words(pts + 16 * i, p)) acc = madd(acc, p);
  }
  to_affine_words(acc, out);
}

// sum of affine points by full XYZZ additions (pairwise tree).
void host_g1_sum_add(const uint32_t* pts, uint64_t n, uint32_t* out) {
  xyzz acc = xyzz_inf();
  for (uint64_t i = 0; i < n; i++) {
    aff p;
    if (aff_from_plain_words(pts + 16 * i, p)) acc = add(acc, from_aff(p));
  }
  to_affine_words(acc, out);
}

void host_g1_dbl(const uint32_t* pt, uint32_t* out) {
  aff p;
  xyzz a = aff_from_plain_words(pt, p) ? from_aff(p) : xyzz_inf();
  to_affine_words(dbl(a), out);
}

void host_g1_mul_small(const uint32_t* pt, uint32_t k, uint32_t* out) {
  aff p;
  xyzz a = aff_from_plain_words(pt, p) ? from_aff(p) : xyzz_inf();
  to_affine_words(mul_small(a, k), out);
}

void host_g1_neg(const uint32_t* pt, uint32_t* out) {
  aff p;
  if (!aff_from_plain_words(pt, p)) {
    for (int i = 0; i < 16; i++) out[i] = 0;
    return;
  }
  to_affine_words(from_aff(aff_neg(p)), out);
}

// XYZZ given as raw 29-bit limbs (36 words, Montgomery coordinates):
// lets tests push representations to the edge of the bounded box.
static xyzz load_xyzz_raw(const uint32_t* w) {
  xyzz a;
  for (int i = 0; i < 9; i++) {
    a.X.l[i] = w[i];
    a.Y.l[i] = w[9 + i];
    a.ZZ.l[i] = w[18 + i];
    a.ZZZ.l[i] = w[27 + i];
  }
  return a;
}

static void store_xyzz_raw(const xyzz& a, uint32_t* w) {
  for (int i = 0; i < 9; i++) {
    w[i] = a.X.l[i];
    w[9 + i] = a.Y.l[i];
    w[18 + i] = a.ZZ.l[i];
    w[27 + i] = a.ZZZ.l[i];
  }
}

void host_xyzz_add_raw(const uint32_t* a, const uint32_t* b, uint32_t* out) {
  store_xyzz_raw(add(load_xyzz_raw(a), load_xyzz_raw(b)), out);
}

void host_xyzz_madd_raw(const uint32_t* a, const uint32_t* pt, uint32_t* out) {
  aff p;
  aff_from_plain_words(pt, p);
  store_xyzz_raw(madd(load_xyzz_raw(a), p), out);
}

void host_xyzz_madd_signed_raw(const uint32_t* a, const uint32_t* pt, int neg, uint32_t* out) {
  aff p;
  aff_from_plain_words(pt, p);
  store_xyzz_raw(madd_signed(load_xyzz_raw(a), p, neg != 0), out);
}

// sum of +-points (signs[i] != 0: subtract) by the signed mixed addition.
void host_g1_sum_madd_signed(const uint32_t* pts, const int* signs, uint64_t n, uint32_t* out) {
  xyzz acc = xyzz_inf();
  for (uint64_t i = 0; i < n; i++) {
    aff p;
    if (aff_from_plain_words(pts + 16 * i, p)) acc = madd_signed(acc, p, signs[i] != 0);
  }
  to_affine_words(acc, out);
}

void host_xyzz_dbl_raw(const uint32_t* a, uint32_t* out) {
  store_xyzz_raw(dbl(load_xyzz_raw(a)), out);
}

void host_xyzz_to_affine(const uint32_t* a, uint32_t* out) {
  to_affine_words(load_xyzz_raw(a), out);
}

}  // extern "C"

// ---- G2 (Fq2 and twist points) ----------------------------------------------

static fp2 load_fp2_raw(const uint32_t* w) {
  fp2 a;
  for (int i = 0; i < 9; i++) {
    a.c0.l[i] = w[i];
    a.c1.l[i] = w[9 + i];
  }
  return a;
}

static void store_fp2_raw(const fp2& a, uint32_t* w) {
  for (int i = 0; i < 9; i++) {
    w[i] = a.c0.l[i];
    w[9 + i] = a.c1.l[i];
  }
}

extern "C" {

// op: 0 add, 1 sub, 2 mul, 3 sqr, 4 inv (Montgomery components as raw
// 29-bit limbs, 18 words per element).
void host_fq2_op_raw(int op, const uint32_t* a, const uint32_t* b, uint32_t* out) {
  const fp2 x = load_fp2_raw(a), y = load_fp2_raw(b);
  fp2 r;
  switch (op) {
    case 0: r = fp2_add(x, y); break;
    case 1: r = fp2_sub(x, y); break;
    case 2: r = fp2_mul(x, y); break;
    case 3: r = fp2_sqr(x); break;
    default: r = fp2_inv(x); break;
  }
  store_fp2_raw(r, out);
}

// a b - c d by fp2_mul_sub (same raw layout).
void host_fq2_mul_sub_raw(const uint32_t* a, const uint32_t* b, const uint32_t* c, const uint32_t* d,
                          uint32_t* out) {
  store_fp2_raw(fp2_mul_sub(load_fp2_raw(a), load_fp2_raw(b), load_fp2_raw(c), load_fp2_raw(d)), out);
}

// sum of affine G2 points (32 words each, (0,0,0,0) = infinity).
void host_g2_sum_madd(const uint32_t* pts, uint64_t n, uint32_t* out) {
  g2xyzz acc = g2_inf();
  for (uint64_t i = 0; i < n; i++) {
    g2aff p;
    if (g2_from_words(pts + 32 * i, p)) acc = g2_madd(acc, p);
  }
  g2_to_words(acc, out);
}

void host_g2_sum_add(const uint32_t* pts, uint64_t n, uint32_t* out) {
  g2xyzz acc = g2_inf();
  for (uint64_t i = 0; i < n; i++) {
    g2aff p;
    if (g2_from_words(pts + 32 * i, p)) acc = g2_add(acc, g2_from_aff(p));
  }
  g2_to_words(acc, out);
}

void host_g2_dbl(const uint32_t* pt, uint32_t* out) {
  g2aff p;
  const g2xyzz a = g2_from_words(pt, p) ? g2_from_aff(p) : g2_inf();
  g2_to_words(g2_dbl(a), out);
}

void host_g2_neg(const uint32_t* pt, uint32_t* out) {
  g2aff p;
  if (!g2_from_words(pt, p)) {
    for (int i = 0; i < 32; i++) out[i] = 0;
    return;
  }
  g2_to_words(g2_from_aff(g2_aff_neg(p)), out);
}

int host_g2_valid(const uint32_t* pt) { return g2_words_valid(pt) ? 1 : 0; }

// k (8 words, < r) -> out: k1 (4 words), k2 (4 words), sign of k1, sign of k2.
void host_glv_split(const uint32_t* k, uint32_t* out) {
  uint32_t kk[8], k1[4], k2[4];
  for (int i = 0; i < 8; i++) kk[i] = k[i];
  bool n1 = false, n2 = false;
  glv_split(kk, k1, n1, k2, n2);
  for (int i = 0; i < 4; i++) {
    out[i] = k1[i];
    out[4 + i] = k2[i];
  }
  out[8] = n1 ? 1u : 0u;
  out[9] = n2 ? 1u : 0u;
}

// The endomorphism as the kernels apply it: X of an XYZZ point times beta
// (Montgomery product), then affine.  It maps 2P, whose ZZ is not 1, so
// out = phi(2P).
void host_glv_phi(const uint32_t* pt, uint32_t* out) {
  aff a;
  if (!aff_from_plain_words(pt, a)) {
    for (int i = 0; i < 16; i++) out[i] = 0;
    return;
  }
  xyzz p = dbl(from_aff(a));  // a point with ZZ != 1
  p.X = mont_mul<Fq>(p.X, load_mont<Fq>(GlvConst::BETA));
  to_affine_words(p, out);
}

}  // extern "C"
