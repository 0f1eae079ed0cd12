"""GPU parity of the Poly-IOP quotient (zk_quotient_polyiop) against the
oracle: every coefficient of Q = R(f(x), f(omega x)) / (X^n - 1) bit-exact,
and the commitment [Q(tau)]_1 against its closed form, for the paper's
BooleanCheck, Sub Check and i-thIsZero constraints, a degree-2 running
product z(omega x) = z(x) f(x) (the omega-shifted operand is the coset
vector rotated by B points), a cubic with a constant term and general
coefficients on a 4x coset, and a caller's shift; at the full 2^20 size,
BooleanCheck and the running product element by element.  Requests the
library cannot serve (blowup below the degree, bad factor indices, too many
witnesses or terms, an SRS too short for the quotient) are refused.
"""
import numpy as np
import pytest

from oracle import field, kzg, polyiop as op
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import ints_to_limbs, limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R

RUNNING_PRODUCT = [(1, [2]), (R - 1, [0, 1])]        # z(omega x) - z(x) f(x)


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


def _boolean(seed, n):
    bits = gen.rng_for(seed, 1).integers(0, 2, size=n)
    return [int(b) for b in bits]


def _sub_check(seed, n):
    g = fr_from_host(gen.uniform_fr(seed, n, tag=2))
    return [g, [(g[(i + 1) % n] - g[i]) % R for i in range(n)]]


def _ith_is_zero(seed, n):
    i0 = int(gen.rng_for(seed, 3).integers(0, n))
    d = fr_from_host(gen.uniform_fr(seed, n, tag=4))
    d[i0] = 0
    return [[1 if j == i0 else 0 for j in range(n)], d]


def _running_product(seed, n):
    f = fr_from_host(gen.uniform_fr(seed, n, tag=5))
    f = [v or 1 for v in f]
    prod = 1
    for v in f[:-1]:
        prod = prod * v % R
    f[-1] = pow(prod, -1, R)
    z = [fr_from_host(gen.uniform_fr(seed, 1, tag=6))[0] or 1]
    for i in range(n - 1):
        z.append(z[-1] * f[i] % R)
    return [z, f]


def _cubic(seed, n):
    # R = 3 f1^3 - 3 f1 + 5 f2(omega x) - 5 f2(x) - 5 f1(x) - 5 k: f1 takes
    # values in {0, 1, -1} (so f1^3 = f1 on H) and f2 is the running sum
    # f2_(i+1) = f2_i + f1_i + k, cyclic because k = -(sum f1) / n
    f1 = [(int(v) - 1) % R for v in gen.rng_for(seed, 9).integers(0, 3, size=n)]
    k = (-sum(f1) * pow(n, -1, R)) % R
    f2 = [fr_from_host(gen.uniform_fr(seed, 1, tag=10))[0]]
    for i in range(n - 1):
        f2.append((f2[-1] + f1[i] + k) % R)
    terms = [(3, [0, 0, 0]), (R - 3, [0]), (5, [3]), (R - 5, [1]), (R - 5, [0]), ((-5 * k) % R, [])]
    return [f1, f2], terms


def _run(zk, srs, vecs, terms, logb, shift=None):
    n = len(vecs[0])
    ev = zk.to_device(ints_to_limbs([v for vec in vecs for v in vec]).reshape(len(vecs), n, 8))
    return zk.quotient_polyiop(srs, ev, terms, log_blowup=logb, shift=shift)


def _check(zk, tau, srs, vecs, terms, logb, shift=None, label=""):
    q_dev, com = _run(zk, srs, vecs, terms, logb, shift)
    want, rem, _ = op.polyiop_quotient(vecs, terms)
    assert not any(rem), "witness does not satisfy R (%s)" % label
    got = fr_from_host(_host(zk, q_dev))
    assert len(got) == len(want), label
    if got != want:
        bad = [i for i, (a, b) in enumerate(zip(got, want)) if a != b]
        raise AssertionError("%s: %d of %d coefficients differ, first at %d" % (label, len(bad), len(got), bad[0]))
    assert points_from_host(_host(zk, com))[0] == kzg.proof_closed_form(tau[1], want), label


@pytest.mark.parametrize("logn,logb", [(0, 1), (1, 1), (2, 2), (3, 1), (8, 4), (12, 1), (13, 2), (16, 1)])
def test_boolean_check_exact(zk, tau, srs, logn, logb):
    n = 1 << logn
    log("polyiop boolean check n=2^%d blowup=2^%d" % (logn, logb))
    _check(zk, tau, srs, [_boolean(8500 + logn, n)], op.BOOLEAN_CHECK, logb, label="boolean")


@pytest.mark.parametrize("logn", [1, 2, 5, 12, 14])
def test_shifted_constraints_exact(zk, tau, srs, logn):
    n = 1 << logn
    log("polyiop shifted constraints n=2^%d" % logn)
    _check(zk, tau, srs, _sub_check(8600 + logn, n), op.SUB_CHECK, 1, label="sub check")
    _check(zk, tau, srs, _ith_is_zero(8700 + logn, n), op.ITH_IS_ZERO, 1, label="i-th is zero")
    _check(zk, tau, srs, _running_product(8800 + logn, n), RUNNING_PRODUCT, 1, label="running product")
    _check(zk, tau, srs, _running_product(8900 + logn, n), RUNNING_PRODUCT, 3, label="running product 8x")


def test_cubic_with_constant_and_custom_shift(zk, tau, srs):
    # a degree-3 constraint on a 4x coset (and an 8x one), with general
    # coefficients, a constant term and an omega-shifted operand, under the
    # default shift and a caller's
    n = 1 << 10
    vecs, terms = _cubic(9000, n)
    for shift, logb in ((None, 2), (7, 2), (None, 3)):
        log("polyiop cubic, shift", shift, "blowup", 1 << logb)
        _check(zk, tau, srs, vecs, terms, logb, shift=None if shift is None else ints_to_limbs([shift])[0],
               label="cubic shift=%s" % shift)


@pytest.mark.parametrize("kind", ["boolean", "running_product"])
def test_polyiop_full_size(zk, tau, srs, kind):
    n = 1 << 20
    if kind == "boolean":
        vecs, terms = [_boolean(9100, n)], op.BOOLEAN_CHECK
    else:
        vecs, terms = _running_product(9200, n), RUNNING_PRODUCT
    log("polyiop %s n=2^20 (oracle about a minute)" % kind)
    _check(zk, tau, srs, vecs, terms, 1, label=kind)


def test_polyiop_rejections(zk, srs):
    n = 1 << 6
    ev1 = zk.to_device(ints_to_limbs(_boolean(9300, n)).reshape(1, n, 8))
    bad = [
        (ev1, op.BOOLEAN_CHECK, 0),                       # blowup 1 below the degree 2
        (ev1, [(1, [0, 0, 0])], 1),                       # degree 3 on a 2x coset
        (ev1, [(1, [2])], 1),                             # factor index >= 2N
        (ev1, [(1, [0])] * 17, 1),                        # too many terms
        (ev1, [(1, [0] * 5)], 3),                         # degree above the limit
    ]
    for ev, terms, logb in bad:
        with pytest.raises(zk.ZkError) as ei:
            zk.quotient_polyiop(srs, ev, terms, log_blowup=logb)
        assert ei.value.code == zk.ZK_EINVAL, terms
    ev9 = zk.to_device(np.zeros((9, n, 8), dtype=np.uint32))
    with pytest.raises(zk.ZkError) as ei:
        zk.quotient_polyiop(srs, ev9, [(1, [0])], log_blowup=1)
    assert ei.value.code == zk.ZK_EINVAL
    # a quotient of (d - 1) n coefficients needs that many SRS points
    big = zk.to_device(np.zeros((1, 1 << 20, 8), dtype=np.uint32))
    with pytest.raises(zk.ZkError) as ei:
        zk.quotient_polyiop(srs, big, [(1, [0, 0, 0])], log_blowup=2)
    assert ei.value.code == zk.ZK_EINVAL
