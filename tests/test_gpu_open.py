"""GPU parity of the KZG opening (zk_kzg_open, zk_kzg_open_batch) against the
oracle, bit-exact: evaluations, every quotient coefficient, and the proof
against the closed form [q(tau)]_1 with the test trapdoor.  Sizes cover one
tile (2048 coefficients), several tiles with ragged tails, more than 256
tiles (several tiles per carry thread) and the full 2^20 workload; points
include 0, 1 and a root of unity; batches include gamma = 0.
"""
import numpy as np
import pytest

from oracle import field, g1, kzg, msm as omsm, ntt as ontt
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import ints_to_limbs, limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R
SRS_LOG = 20


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
    log("srs setup 2^%d" % SRS_LOG)
    pts = zk.srs_setup(tau[0], 1 << SRS_LOG)
    h = zk.SRS(pts)
    torch.cuda.synchronize()
    yield h
    h.close()


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def _fr_words(v):
    return ints_to_limbs([v % R])[0]


def _point(kind, seed):
    if kind == "zero":
        return 0
    if kind == "one":
        return 1
    if kind == "root":
        return ontt.root_of_unity(1 << 20) ** 3 % R
    return limbs_to_ints(gen.uniform_fr(seed, 1, tag=7))[0]


def _check_single(zk, tau, srs, n, xkind, seed):
    a = gen.uniform_fr(seed, max(n, 1))[:n]
    x = _point(xkind, seed)
    log("kzg open n=%d x=%s seed=%d" % (n, xkind, seed))
    dev = zk.to_device(a.reshape(-1, 8) if n else np.zeros((1, 8), np.uint32))
    y, q, pi = zk.kzg_open(srs, dev, _fr_words(x), n=n, want_quotient=True)
    yh = fr_from_host(_host(zk, y))[0]
    qh = fr_from_host(_host(zk, q)) if n > 1 else []
    pih = points_from_host(_host(zk, pi))[0]
    want_y, want_q = kzg.open_at(fr_from_host(a) if n else [], x)
    assert yh == want_y
    assert len(qh) == len(want_q)
    if qh != want_q:
        bad = [i for i in range(len(qh)) if qh[i] != want_q[i]]
        raise AssertionError("quotient differs at %d indices, first %s" % (len(bad), bad[:8]))
    assert pih == kzg.proof_closed_form(tau[1], want_q)


@pytest.mark.parametrize("n,xkind", [
    (0, "rand"), (1, "rand"), (2, "rand"), (3, "zero"), (9, "one"), (100, "rand"),
    (2047, "rand"), (2048, "root"), (2049, "rand"), (4101, "one"), (6145, "zero"),
    (70001, "rand"), (600000, "rand"),
])
def test_kzg_open_exact(zk, tau, srs, n, xkind):
    _check_single(zk, tau, srs, n, xkind, 5000 + n)


def test_kzg_open_full_size(zk, tau, srs):
    # the 2^20-coefficient workload; also the verifier identity with the
    # device commitment: com - y G = (tau - x) pi
    n = 1 << 20
    _check_single(zk, tau, srs, n, "rand", 77)
    a = gen.uniform_fr(77, n)
    x = _point("rand", 77)
    dev = zk.to_device(a)
    y, _, pi = zk.kzg_open(srs, dev, _fr_words(x))
    com = zk.msm_srs(srs, dev)
    yh = fr_from_host(_host(zk, y))[0]
    assert kzg.verify_with_trapdoor(tau[1], points_from_host(_host(zk, com))[0], x, yh,
                                    points_from_host(_host(zk, pi))[0])


def test_kzg_open_largest_for_srs(zk, tau, srs):
    # n - 1 = SRS size is the largest opening; one more is rejected
    n = (1 << SRS_LOG) + 1
    a = gen.uniform_fr(91, n)
    x = _point("rand", 91)
    log("kzg open n = srs + 1")
    y, q, pi = zk.kzg_open(srs, zk.to_device(a), _fr_words(x), want_quotient=True)
    av = fr_from_host(a)
    want_y, want_q = kzg.open_at(av, x)
    assert fr_from_host(_host(zk, y))[0] == want_y
    assert fr_from_host(_host(zk, q)) == want_q
    assert points_from_host(_host(zk, pi))[0] == kzg.proof_closed_form(tau[1], want_q)
    b = gen.uniform_fr(92, n + 1)
    with pytest.raises(zk.ZkError) as ei:
        zk.kzg_open(srs, zk.to_device(b), _fr_words(x))
    assert ei.value.code == zk.ZK_EINVAL


def test_kzg_open_without_quotient_buffer(zk, tau, srs):
    n = 30001
    a = gen.uniform_fr(93, n)
    x = _point("rand", 93)
    dev = zk.to_device(a)
    _, q, pi1 = zk.kzg_open(srs, dev, _fr_words(x), want_quotient=True)
    y2, none, pi2 = zk.kzg_open(srs, dev, _fr_words(x))
    assert none is None
    assert np.array_equal(_host(zk, pi1), _host(zk, pi2))
    _, want_q = kzg.open_at(fr_from_host(a), x)
    assert points_from_host(_host(zk, pi2))[0] == kzg.proof_closed_form(tau[1], want_q)


def test_kzg_open_rejects_bad_point(zk, srs):
    a = gen.uniform_fr(94, 16)
    bad = np.array([0xFFFFFFFF] * 8, dtype=np.uint32)
    with pytest.raises(zk.ZkError) as ei:
        zk.kzg_open(srs, zk.to_device(a), bad)
    assert ei.value.code == zk.ZK_EINVAL


@pytest.mark.parametrize("m,n,gkind", [
    (1, 5000, "rand"), (2, 2049, "rand"), (3, 777, "zero"), (5, 20000, "rand"), (8, 1 << 16, "rand"),
    (4, 600001, "one"),
])
def test_kzg_open_batch_exact(zk, tau, srs, m, n, gkind):
    import torch
    polys = np.stack([gen.uniform_fr(6000 + 31 * i + n, n) for i in range(m)])
    x = _point("rand", 6000 + n)
    gamma = {"zero": 0, "one": 1}.get(gkind) if gkind != "rand" else limbs_to_ints(gen.uniform_fr(6001 + n, 1, tag=9))[0]
    log("kzg batch open m=%d n=%d gamma=%s" % (m, n, gkind))
    dev = zk.to_device(polys.reshape(m * n, 8)).reshape(m, n, 8)
    ys, h, pi = zk.kzg_open_batch(srs, dev, _fr_words(x), _fr_words(gamma), want_quotient=True)
    torch.cuda.synchronize()
    pv = [fr_from_host(polys[i]) for i in range(m)]
    want_ys, want_h = kzg.batch_open_at(pv, x, gamma)
    assert fr_from_host(_host(zk, ys)) == want_ys
    assert fr_from_host(_host(zk, h)) == want_h
    assert points_from_host(_host(zk, pi))[0] == kzg.proof_closed_form(tau[1], want_h)


def test_kzg_open_batch_verifier_identity(zk, tau, srs):
    # sum_i gamma^i (com_i - y_i G) = (tau - x) pi with device commitments
    m, n = 3, 3001
    polys = np.stack([gen.uniform_fr(7100 + i, n) for i in range(m)])
    x = _point("rand", 7100)
    gamma = limbs_to_ints(gen.uniform_fr(7101, 1, tag=9))[0]
    dev = zk.to_device(polys.reshape(m * n, 8))
    ys, _, pi = zk.kzg_open_batch(srs, dev.reshape(m, n, 8), _fr_words(x), _fr_words(gamma))
    coms = [points_from_host(_host(zk, zk.msm_srs(srs, dev[i * n:(i + 1) * n])))[0] for i in range(m)]
    assert kzg.batch_verify_with_trapdoor(tau[1], coms, x, fr_from_host(_host(zk, ys)), gamma,
                                          points_from_host(_host(zk, pi))[0])
