"""Seeded input generators (numpy PCG64) for the commit / fold workloads.

Layout conventions used everywhere in this repository:

* A field element (Fr scalar or evaluation) is 8 little-endian uint32 limbs,
  value canonical (< modulus).  An array of them is ``uint32[n, 8]``.
* Seeds: the trapdoor tau uses ``TAU_SEED``; workload k (1-based, see
  ``CONFIG_SEEDS``) uses seed k.  Independent sub-streams of one seed are
  selected with an integer ``tag`` through ``numpy.random.SeedSequence``.

Nothing here multiplies field elements or touches curve points: the only
modulus-dependent steps are the rejection test ``x < r`` that makes uniform
draws canonical, and writing a small negative integer -m as the limbs of r - m
(a change of limb 0 only, because m < 2^16 is far below r's low limb).
"""
from __future__ import annotations

import numpy as np

# The BN254 scalar-field prime r (the group order of G1), as fixed by the
# experimental setup (BN254 over a 254-bit prime field).
FR_MODULUS = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001

TAU_SEED = 1001
CONFIG_SEEDS = {
    "tiny": 1,        # MSM 2^10 + NTT/iNTT 2^12
    "commit": 2,      # iNTT 2^20 -> MSM 2^20 -> 4x coset NTT
    "quantized": 3,   # MSM 2^22 with int16-activation scalars
    "batched": 4,     # 256 uneven MSMs + fold of 64 commitments
    "serving": 5,     # Poisson stream of commit jobs
}

_R_U64 = [(FR_MODULUS >> (64 * i)) & 0xFFFFFFFFFFFFFFFF for i in range(4)]
_TOP_MASK = (1 << 62) - 1  # keep the low 254 bits of a 256-bit draw


def rng_for(seed: int, tag: int = 0) -> np.random.Generator:
    """Independent PCG64 stream for (seed, tag)."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(tag)])))


def _below_r(w: np.ndarray) -> np.ndarray:
    """Row-wise test (little-endian uint64 x4 rows) of value < r."""
    lt = np.zeros(w.shape[0], dtype=bool)
    eq = np.ones(w.shape[0], dtype=bool)
    for i in (3, 2, 1, 0):
        ri = np.uint64(_R_U64[i])
        lt |= eq & (w[:, i] < ri)
        eq &= w[:, i] == ri
    return lt


def uniform_fr(seed: int, n: int, tag: int = 0) -> np.ndarray:
    """n elements uniform in [0, r): 32 random bytes -> little-endian integer,
    keep the low 254 bits, reject if >= r (acceptance about 0.757)."""
    n = int(n)
    out = np.empty((n, 4), dtype=np.uint64)
    if n == 0:
        return out.view(np.uint32).reshape(0, 8)
    rng = rng_for(seed, tag)
    filled = 0
    while filled < n:
        m = int((n - filled) * 1.34) + 64
        w = np.frombuffer(rng.bytes(32 * m), dtype="<u8").reshape(m, 4).copy()
        w[:, 3] &= np.uint64(_TOP_MASK)
        ok = w[_below_r(w)]
        take = min(n - filled, ok.shape[0])
        out[filled:filled + take] = ok[:take]
        filled += take
    return np.ascontiguousarray(out).view(np.uint32).reshape(n, 8)


def quantized_fr(seed: int, n: int, bits: int = 16, sigma: float = 32.0,
                 zero_frac: float = 0.3, tag: int = 0) -> np.ndarray:
    """Fixed-point activations embedded in Fr: x = rint(N(0, sigma^2)), clipped to
    the signed ``bits``-bit range, a Bernoulli(zero_frac) mask set to 0, then
    x < 0 written as r - |x|."""
    if bits not in (8, 16):
        raise ValueError("bits must be 8 or 16")
    rng = rng_for(seed, tag)
    x = np.rint(rng.normal(0.0, sigma, size=int(n)))
    lo, hi = -(1 << (bits - 1)), (1 << (bits - 1)) - 1
    x = np.clip(x, lo, hi).astype(np.int64)
    x[rng.random(int(n)) < zero_frac] = 0
    out = np.zeros((int(n), 8), dtype=np.uint32)
    pos = x >= 0
    out[pos, 0] = x[pos].astype(np.uint32)
    neg = ~pos
    r_limbs = np.array([(FR_MODULUS >> (32 * i)) & 0xFFFFFFFF for i in range(8)], dtype=np.uint64)
    out[neg, :] = r_limbs.astype(np.uint32)
    out[neg, 0] = (r_limbs[0] - (-x[neg]).astype(np.uint64)).astype(np.uint32)
    return out


def quantized_values(seed: int, n: int, bits: int = 16, sigma: float = 32.0,
                     zero_frac: float = 0.3, tag: int = 0) -> np.ndarray:
    """The signed integers behind ``quantized_fr`` (same draws), int64[n]."""
    rng = rng_for(seed, tag)
    x = np.rint(rng.normal(0.0, sigma, size=int(n)))
    lo, hi = -(1 << (bits - 1)), (1 << (bits - 1)) - 1
    x = np.clip(x, lo, hi).astype(np.int64)
    x[rng.random(int(n)) < zero_frac] = 0
    return x


def log_uniform_sizes(seed: int, count: int, lo_exp: float, hi_exp: float, tag: int = 0) -> np.ndarray:
    """count sizes n = rint(2^U), U ~ Uniform[lo_exp, hi_exp] (continuous)."""
    rng = rng_for(seed, tag)
    u = rng.uniform(lo_exp, hi_exp, size=int(count))
    return np.rint(np.exp2(u)).astype(np.int64)


def poisson_arrivals(seed: int, count: int, rate_per_s: float, tag: int = 0) -> np.ndarray:
    """Arrival times (s) of a Poisson process: cumulative exponential gaps."""
    rng = rng_for(seed, tag)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=int(count)))


def tau_scalar(seed: int = TAU_SEED) -> np.ndarray:
    """The SRS trapdoor: one uniform nonzero Fr element, uint32[8]."""
    tag = 0
    while True:
        t = uniform_fr(seed, 1, tag=tag)[0]
        if t.any():
            return t
        tag += 1


def commit_job_eval_sizes(n: np.ndarray) -> np.ndarray:
    """Domain size of a commit job: the next power of two >= n (n >= 1)."""
    n = np.asarray(n, dtype=np.int64)
    return np.left_shift(1, np.ceil(np.log2(np.maximum(n, 1))).astype(np.int64))


def ints_to_limbs(values) -> np.ndarray:
    """Python ints (each < 2^256) -> uint32[len, 8] little-endian limbs."""
    vals = list(values)
    buf = b"".join(int(v).to_bytes(32, "little") for v in vals)
    return np.frombuffer(buf, dtype="<u4").reshape(len(vals), 8).copy()


def limbs_to_ints(arr: np.ndarray) -> list:
    """uint32[..., 8] little-endian limbs -> flat list of Python ints."""
    a = np.ascontiguousarray(np.asarray(arr, dtype=np.uint32)).reshape(-1, 8)
    raw = a.astype("<u4").tobytes()
    return [int.from_bytes(raw[32 * i:32 * i + 32], "little") for i in range(a.shape[0])]
