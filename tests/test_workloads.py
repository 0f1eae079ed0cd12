"""The seeded input generators produce the distributions the workloads name."""
import numpy as np

from workloads import generators as gen

R = gen.FR_MODULUS


def test_uniform_fr_canonical_and_deterministic():
    a = gen.uniform_fr(2, 5000)
    b = gen.uniform_fr(2, 5000)
    assert a.shape == (5000, 8) and a.dtype == np.uint32
    assert np.array_equal(a, b)
    vals = gen.limbs_to_ints(a)
    assert all(0 <= v < R for v in vals)
    # top bits are used: about half of the draws are above r / 2
    frac_hi = sum(v > R // 2 for v in vals) / len(vals)
    assert 0.45 < frac_hi < 0.55
    assert not np.array_equal(a, gen.uniform_fr(3, 5000))
    assert gen.uniform_fr(1, 0).shape == (0, 8)


def test_limb_roundtrip():
    vals = [0, 1, R - 1, (1 << 255) + 12345, 2 ** 32 - 1]
    assert gen.limbs_to_ints(gen.ints_to_limbs(vals)) == vals


def test_quantized_distribution():
    n = 1 << 16
    q = gen.quantized_fr(3, n)
    x = gen.quantized_values(3, n)
    vals = gen.limbs_to_ints(q)
    assert vals == [int(v) % R for v in x]
    zeros = float(np.mean(x == 0))
    neg = float(np.mean(x < 0))
    assert 0.28 < zeros < 0.34
    assert 0.30 < neg < 0.38
    assert np.abs(x).max() < 300
    q8 = gen.quantized_values(3, n, bits=8)
    assert q8.min() >= -128 and q8.max() <= 127


def test_sizes_and_arrivals():
    s = gen.log_uniform_sizes(4, 256, 8, 18)
    assert s.min() >= 256 and s.max() <= 1 << 18
    assert 2e4 < s.mean() < 6e4
    t = gen.poisson_arrivals(5, 2000, 200.0)
    gaps = np.diff(t)
    assert np.all(gaps >= 0)
    assert 0.004 < gaps.mean() < 0.006
    n = np.array([1, 2, 3, 1024, 1025, 1 << 22])
    assert list(gen.commit_job_eval_sizes(n)) == [1, 2, 4, 1024, 2048, 1 << 22]


def test_tau_nonzero():
    t = gen.tau_scalar()
    v = gen.limbs_to_ints(t[None, :])[0]
    assert 0 < v < R
