"""GPU parity of the G2 SRS setup and MSM (zk_srs_g2_setup, zk_msm_g2_srs)
against the oracle, bit-exact: SRS points, tiny MSMs against the oracle's
naive sum (edge scalars 0, 1, r - 1, 128 and 2^253 multiples whose digits
carry), MSMs whose bucket and bit sums meet equal or opposite points, and
MSMs of several sizes and scalar distributions against the closed form
[sum_i s_i tau^i]_2, including points at infinity.
"""
import numpy as np
import pytest

from oracle import field, g2 as og2
from tests.gpu_helpers import fr_from_host, log
from workloads import generators as gen
from workloads import ints_to_limbs, limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R
SRS_N = 1 << 16


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
    log("g2 srs setup 2^16")
    pts = zk.srs_g2_setup(tau[0], SRS_N)
    h = zk.SRSG2(pts)
    torch.cuda.synchronize()
    yield pts, h
    h.close()


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def _g2_from_host(arr):
    v = limbs_to_ints(np.asarray(arr, dtype=np.uint32).reshape(-1, 8))
    return [og2.decode(tuple(v[4 * i:4 * i + 4])) for i in range(len(v) // 4)]


def _g2_to_host(pts):
    vals = []
    for p in pts:
        vals += list(og2.encode(p))
    return ints_to_limbs(vals).reshape(len(pts), 32)


def test_g2_srs_points(zk, tau, srs):
    pts, _ = srs
    h = _host(zk, pts)
    idx = [0, 1, 2, 1000, SRS_N - 1]
    got = _g2_from_host(h[idx])
    assert got[0] == og2.H
    for j, p in zip(idx, got):
        assert p == og2.gen_mul(pow(tau[1], j, R)), j


def test_g2_msm_edge_scalars(zk, srs):
    # arbitrary bases (not an SRS), including infinity, against the naive sum
    ks = limbs_to_ints(gen.uniform_fr(9700, 8, tag=1))
    bases = [og2.gen_mul(k) for k in ks]
    bases[3] = None
    bases[5] = bases[4]
    scal = [0, 1, R - 1, 128, 127, 129, 2 ** 253 + 2 ** 8 * 128, (R - 1) // 2]
    log("g2 msm edge scalars")
    h = zk.SRSG2(zk.to_device(_g2_to_host(bases)))
    out = zk.msm_g2_srs(h, zk.to_device(ints_to_limbs(scal).reshape(-1, 8)))
    assert _g2_from_host(_host(zk, out))[0] == og2.naive_msm(bases, scal)
    # single terms
    for i in (1, 2, 6):
        e = [0] * 8
        e[i] = scal[i]
        out = zk.msm_g2_srs(h, zk.to_device(ints_to_limbs(e).reshape(-1, 8)))
        assert _g2_from_host(_host(zk, out))[0] == og2.mul(scal[i], bases[i])
    h.close()


def test_g2_msm_equal_and_opposite_sums(zk):
    # sums that meet equal or opposite points in the bucket, bit-slice and
    # final trees: the doubling and cancellation paths of their additions
    P = og2.gen_mul(limbs_to_ints(gen.uniform_fr(9710, 1, tag=1))[0])
    cases = [
        ("every bucket holds P", [P] * 128, list(range(1, 129)), og2.mul(128 * 129 // 2, P)),
        ("two equal partials in a bucket", [P] * 64, [1] * 64, og2.mul(64, P)),
        ("two opposite partials in a bucket", [P] * 32 + [og2.neg(og2.mul(32, P))], [1] * 33, None),
    ]
    for name, bases, scal, want in cases:
        log("g2 msm: " + name)
        h = zk.SRSG2(zk.to_device(_g2_to_host(bases)))
        out = zk.msm_g2_srs(h, zk.to_device(ints_to_limbs(scal).reshape(-1, 8)))
        assert _g2_from_host(_host(zk, out))[0] == want, name
        h.close()


@pytest.mark.parametrize("n,kind", [(0, "uniform"), (1, "uniform"), (5, "uniform"), (300, "uniform"),
                                    (4097, "quantized"), (20000, "uniform"), (SRS_N, "uniform"),
                                    (SRS_N, "quantized")])
def test_g2_msm_closed_form(zk, tau, srs, n, kind):
    _, h = srs
    s = (gen.uniform_fr(9800 + n, max(n, 1)) if kind == "uniform"
         else gen.quantized_fr(9800 + n, max(n, 1)))[:n]
    log("g2 msm n=%d %s" % (n, kind))
    out = zk.msm_g2_srs(h, zk.to_device(s if n else np.zeros((1, 8), np.uint32)), n=n)
    want = og2.srs_msm_closed_form(tau[1], fr_from_host(s) if n else [])
    assert _g2_from_host(_host(zk, out))[0] == want


def test_g2_msm_rejects_oversize(zk, srs):
    _, h = srs
    s = gen.uniform_fr(9900, SRS_N + 1)
    with pytest.raises(zk.ZkError) as ei:
        zk.msm_g2_srs(h, zk.to_device(s))
    assert ei.value.code == zk.ZK_EINVAL


def test_g2_validation_mode(zk):
    from tests.test_host_arith import _fq2_sqrt
    good = [og2.gen_mul(k) for k in (3, 5, 7)] + [None]
    q = good[0]
    off_curve = (q[0], og2.f2_add(q[1], (1, 0)))
    outside = None
    for t in range(1, 60):
        x = (t, 1)
        y = _fq2_sqrt(og2.f2_add(og2.f2_mul(og2.f2_mul(x, x), x), og2.B2))
        if y is not None and og2.mul(R, (x, y)) is not None:
            outside = (x, y)
            break
    assert outside is not None and og2.on_curve(outside)
    zk.set_validate(True)
    try:
        log("g2 validation: valid points")
        h = zk.SRSG2(zk.to_device(_g2_to_host(good)))
        h.close()
        for bad in (off_curve, outside):
            log("g2 validation: rejected point")
            with pytest.raises(zk.ZkError) as ei:
                zk.SRSG2(zk.to_device(_g2_to_host(good + [bad])))
            assert ei.value.code == zk.ZK_EINVAL
    finally:
        zk.set_validate(False)
