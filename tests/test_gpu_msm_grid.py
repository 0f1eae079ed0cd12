"""GPU parity of the MSM's accumulation launch at its edges, bit-exact against
the oracle's closed form [sum_i s_i tau^i]_1.

The accumulation grid is planned from the n * W digit bound, and each thread's
slice comes from the sorted total, which zero digits make smaller.  The cases:
  * a total of zero (all scalars zero) and of one window (one nonzero scalar);
  * a few hundred nonzero scalars among 2^20 (most threads get no entries);
  * 2^20 - 1 points, a grid one thread short of a power of two;
  * scalars that are 1 (one digit each, a single bucket holding every entry);
  * quantized activations (int16 and int8), small and at 2^20.
"""
import numpy as np
import pytest

from oracle import field, msm as omsm
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import ints_to_limbs, limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R
N = 1 << 20


@pytest.fixture(scope="module")
def zk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_07031_amd import zk as m
    return m


@pytest.fixture(scope="module")
def tau():
    t = gen.tau_scalar()
    return t, limbs_to_ints(t[None, :])[0]


@pytest.fixture(scope="module")
def srs(zk, tau):
    import torch
    log("srs setup 2^20")
    h = zk.SRS(zk.srs_setup(tau[0], N))
    torch.cuda.synchronize()
    yield h
    h.close()


def _commit(zk, h, s):
    import torch
    out = zk.msm_srs(h, zk.to_device(s))
    torch.cuda.synchronize()
    return points_from_host(zk.to_host(out))[0]


def test_all_zero_scalars(zk, srs):
    log("msm grid: all-zero scalars 2^16")
    assert _commit(zk, srs, np.zeros((1 << 16, 8), np.uint32)) is None


def test_one_nonzero_scalar(zk, tau, srs):
    s = np.zeros((N, 8), np.uint32)
    i = 777_777
    v = fr_from_host(gen.uniform_fr(6001, 1))[0]
    s[i] = ints_to_limbs([v])[0]
    log("msm grid: one nonzero among 2^20")
    assert _commit(zk, srs, s) == omsm.srs_msm_closed_form(tau[1], [0] * i + [v])


def test_sparse_scalars(zk, tau, srs):
    rng = gen.rng_for(6002)
    idx = np.sort(rng.choice(N, 300, replace=False))
    vals = gen.uniform_fr(6003, 300)
    s = np.zeros((N, 8), np.uint32)
    s[idx] = vals
    log("msm grid: 300 nonzero among 2^20")
    assert _commit(zk, srs, s) == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))


def test_one_short_of_power_of_two(zk, tau, srs):
    s = gen.uniform_fr(6004, N - 1)
    log("msm grid: 2^20 - 1 uniform")
    assert _commit(zk, srs, s) == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))


def test_single_bucket(zk, tau, srs):
    # every scalar is 1: one digit each, all in one bucket of one window
    n = 1 << 18
    s = np.zeros((n, 8), np.uint32)
    s[:, 0] = 1
    log("msm grid: 2^18 scalars equal to 1")
    assert _commit(zk, srs, s) == omsm.srs_msm_closed_form(tau[1], [1] * n)


@pytest.mark.parametrize("n,bits", [(1 << 10, 16), ((1 << 14) + 3, 16), ((1 << 16) + 5, 8), (1 << 20, 8)])
def test_quantized_small(zk, tau, srs, n, bits):
    # int16 and int8 activations: one live window after the negation trick
    s = gen.quantized_fr(6005 + n, n, bits=bits)
    log("msm grid: quantized int%d n=%d" % (bits, n))
    assert _commit(zk, srs, s) == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))
