"""GPU parity of the Mul-block quotient (zk_quotient_mul) against the oracle:
every coefficient of t = (f h - g) / (X^n - 1) bit-exact, and the
commitment against the closed form [t(tau)]_1, over one- and two-pass
transform sizes and blowups 2, 4 and 16; at the full 2^20 size, the
quotient identity at a random point and at tau with f, h, g evaluated
barycentrically from the witness vectors.
"""
import numpy as np
import pytest

from oracle import field, kzg, quotient as oq
from oracle.ntt import barycentric_eval, horner
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import ints_to_limbs, limbs_to_ints

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
def srs(zk, tau):
    import torch
    log("srs setup 2^20")
    h = zk.SRS(zk.srs_setup(tau[0], 1 << 20))
    torch.cuda.synchronize()
    yield h
    h.close()


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def _witness(seed, n):
    a = gen.uniform_fr(seed, n, tag=1)
    b = gen.uniform_fr(seed, n, tag=2)
    av, bv = fr_from_host(a), fr_from_host(b)
    cv = [field.fr_mul(x, y) for x, y in zip(av, bv)]
    return a, b, ints_to_limbs(cv).reshape(n, 8), av, bv, cv


@pytest.mark.parametrize("logn,logb", [(0, 1), (1, 1), (2, 2), (3, 1), (5, 4), (8, 2), (10, 1), (12, 2),
                                       (13, 1), (14, 2), (16, 1)])
def test_quotient_exact(zk, tau, srs, logn, logb):
    n = 1 << logn
    a, b, c, av, bv, cv = _witness(8000 + logn, n)
    log("quotient mul n=2^%d blowup=2^%d" % (logn, logb))
    t, com = zk.quotient_mul(srs, zk.to_device(a), zk.to_device(b), zk.to_device(c), log_blowup=logb)
    th = fr_from_host(_host(zk, t))
    want, rem, _ = oq.mul_quotient(av, bv, cv)
    assert rem == [0] * n
    assert th == want
    assert points_from_host(_host(zk, com))[0] == kzg.proof_closed_form(tau[1], want)


def test_quotient_custom_and_rejected_shifts(zk, tau, srs):
    n = 1 << 9
    a, b, c, av, bv, cv = _witness(8100, n)
    da, db, dc = zk.to_device(a), zk.to_device(b), zk.to_device(c)
    want, _, _ = oq.mul_quotient(av, bv, cv)
    for s in (7, 3 * R // 5):
        log("quotient custom shift", s % 1000)
        t, com = zk.quotient_mul(srs, da, db, dc, log_blowup=2, shift=ints_to_limbs([s])[0])
        assert fr_from_host(_host(zk, t)) == want
    # s = 1: X^n - 1 vanishes at the coset's first point
    with pytest.raises(zk.ZkError) as ei:
        zk.quotient_mul(srs, da, db, dc, log_blowup=1, shift=ints_to_limbs([1])[0])
    assert ei.value.code == zk.ZK_EINVAL
    with pytest.raises(zk.ZkError):
        zk.quotient_mul(srs, da, db, dc, log_blowup=5)


def test_quotient_full_size_identity(zk, tau, srs):
    n = 1 << 20
    a, b, c, av, bv, cv = _witness(8200, n)
    log("quotient mul n=2^20 blowup=4")
    t, com = zk.quotient_mul(srs, zk.to_device(a), zk.to_device(b), zk.to_device(c), log_blowup=2)
    th = fr_from_host(_host(zk, t))
    assert th[n - 1] == 0
    z = limbs_to_ints(gen.uniform_fr(8201, 1, tag=3))[0]
    for pt in (z, tau[1]):
        fz, hz, gz = (barycentric_eval(v, pt) for v in (av, bv, cv))
        assert horner(th, pt) * oq.vanishing_at(pt, n) % R == (fz * hz - gz) % R
    assert points_from_host(_host(zk, com))[0] == kzg.proof_closed_form(tau[1], th)
