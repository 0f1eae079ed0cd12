"""GPU parity of small commitments on the small-multiples table.

Commitments of up to 4096 points sum one table point m 16^w [tau^i]_1 per
nonzero signed 4-bit digit (§2.1 commitment, no bucket run).  Every result is
compared with the oracle's closed form sum_i s_i [tau^i]_1 = (sum_i s_i tau^i) G
and with the bucket (Pippenger) run of the same commitment (the path turned
off), over sizes around the workgroup (4 scalars x 64 windows) and tree
(256 partials) boundaries, scalars whose digits hit every sign, magnitude 8
and the carries between windows, an SRS shorter than the table, the
no-allocation entry point and the commit job.
"""
import numpy as np
import pytest

from oracle import field, msm as omsm
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R


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
def srs13(zk, tau):
    import torch
    log("tiny: srs setup 2^13")
    pts = zk.srs_setup(tau[0], 1 << 13)
    h = zk.SRS(pts)
    torch.cuda.synchronize()
    yield pts, h
    h.close()


def _commit(zk, h, s_host, tiny):
    import torch
    zk.srs_set_tiny_max(h, 4096 if tiny else 0)
    out = zk.msm_srs(h, zk.to_device(s_host))
    torch.cuda.synchronize()
    zk.srs_set_tiny_max(h, 4096)
    return points_from_host(zk.to_host(out))[0]


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4096])
def test_tiny_sizes_closed_form(zk, tau, srs13, n):
    _, h = srs13
    s = gen.uniform_fr(5100 + n, n)
    log("tiny msm n", n)
    assert zk.srs_window_bits(h, n) == 4
    expect = omsm.srs_msm_closed_form(tau[1], fr_from_host(s))
    assert _commit(zk, h, s, tiny=True) == expect
    assert _commit(zk, h, s, tiny=False) == expect


def test_tiny_policy_bounds(zk, srs13):
    _, h = srs13
    assert zk.srs_window_bits(h, 4097) == 16
    zk.srs_set_tiny_max(h, 100)
    assert zk.srs_window_bits(h, 100) == 4 and zk.srs_window_bits(h, 101) == 16
    zk.srs_set_tiny_max(h, 4096)
    with pytest.raises(zk.ZkError):
        zk.srs_set_tiny_max(h, 4097)


def _digit_scalars():
    """Canonical scalars whose signed 4-bit digits take every value and carry."""
    half = (R - 1) // 2
    vals = [0, 1, 2, 7, 8, 9, 15, 16, 0x88, 0xF8, 0x8F,
            R - 1, R - 2, R - 8, R - 9, half, half + 1, half - 1,
            (1 << 252), (1 << 252) - 1, (1 << 253) - 1 if (1 << 253) - 1 < R else R - 3,
            int("8" * 63, 16), int("7" * 63, 16), int("f" * 62, 16), int("9" * 63, 16),
            sum(8 << (4 * w) for w in range(0, 63, 2)), sum(15 << (4 * w) for w in range(1, 63, 2))]
    return [v % R for v in vals]


def test_tiny_digit_edges(zk, tau, srs13):
    _, h = srs13
    vals = _digit_scalars()
    n = len(vals)
    s = gen.ints_to_limbs(vals)
    log("tiny digit edges", n)
    expect = omsm.srs_msm_closed_form(tau[1], vals)
    assert _commit(zk, h, s, tiny=True) == expect
    # each value alone, at a position that is not the first
    for k, v in enumerate(vals):
        one = [0] * 3
        one[2] = v
        got = _commit(zk, h, gen.ints_to_limbs(one), tiny=True)
        assert got == omsm.srs_msm_closed_form(tau[1], one), (k, hex(v))


def test_tiny_short_srs(zk, tau):
    import torch
    pts = zk.srs_setup(tau[0], 100)
    h = zk.SRS(pts)
    try:
        for n in (1, 99, 100):
            s = gen.uniform_fr(5300 + n, n)
            log("tiny short srs n", n)
            assert zk.srs_window_bits(h, n) == 4
            out = zk.msm_srs(h, zk.to_device(s))
            torch.cuda.synchronize()
            got = points_from_host(zk.to_host(out))[0]
            assert got == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))
    finally:
        h.close()


def test_tiny_noalloc_and_commit_job(zk, tau, srs13):
    import torch
    _, h = srs13
    n = 777
    s = gen.uniform_fr(5400, n)
    log("tiny noalloc", n)
    out = torch.empty((1, 16), dtype=torch.int32, device="cuda")
    zk.msm_srs_noalloc(h, zk.to_device(s), out)
    torch.cuda.synchronize()
    assert points_from_host(zk.to_host(out))[0] == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))
    # commit job of 2^9 evaluations: its commitment equals the MSM of the
    # coefficients the job returns (small-multiples path) and the bucket run
    ev = zk.to_device(gen.uniform_fr(5401, 1 << 9))
    log("tiny commit job 2^9")
    coeffs, com, _ = zk.commit_job(h, ev, log_blowup=2)
    torch.cuda.synchronize()
    c_host = zk.to_host(coeffs)
    expect = omsm.srs_msm_closed_form(tau[1], fr_from_host(c_host))
    assert points_from_host(zk.to_host(com))[0] == expect
    assert _commit(zk, h, c_host, tiny=False) == expect
