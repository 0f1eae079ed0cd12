"""GPU parity of the Lagrange-basis SRS (zk_srs_lagrange_setup) and of
commitments to evaluation vectors over it, against the oracle: every point
at 2^4 (also with tau on H), sampled points at 2^20, and commitments equal
to [f(tau)]_1 with f(tau) evaluated barycentrically from the vector (no
inverse transform), for uniform and quantized vectors, and equal to the
monomial-basis commitment of the interpolant.
"""
import numpy as np
import pytest

from oracle import field, g1, ntt as ontt, srs as osrs
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


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def test_lagrange_points_small(zk, tau):
    log("lagrange setup 2^4")
    pts = points_from_host(_host(zk, zk.srs_lagrange_setup(tau[0], 4)))
    assert pts == osrs.lagrange_srs(tau[1], 16)
    # tau on H: the basis is the unit vector at that root
    w5 = pow(ontt.root_of_unity(16), 5, R)
    pts_h = points_from_host(_host(zk, zk.srs_lagrange_setup(ints_to_limbs([w5])[0], 4)))
    assert pts_h == [g1.G if j == 5 else None for j in range(16)]
    one = points_from_host(_host(zk, zk.srs_lagrange_setup(tau[0], 0)))
    assert one == [g1.G]


def test_lagrange_commit_matches_barycentric_and_monomial(zk, tau):
    import torch
    n = 1 << 12
    v = gen.uniform_fr(9100, n)
    log("lagrange commit 2^12")
    lag = zk.SRS(zk.srs_lagrange_setup(tau[0], 12))
    mono = zk.SRS(zk.srs_setup(tau[0], n))
    dv = zk.to_device(v)
    com_l = points_from_host(_host(zk, zk.msm_srs(lag, dv)))[0]
    want = g1.gen_mul(ontt.barycentric_eval(fr_from_host(v), tau[1]))
    assert com_l == want
    _, com_m, _ = zk.commit_job(mono, dv.clone(), log_blowup=1)
    assert points_from_host(_host(zk, com_m))[0] == want
    lag.close()
    mono.close()
    torch.cuda.synchronize()


def test_lagrange_full_size(zk, tau):
    import torch
    L = 20
    n = 1 << L
    log("lagrange setup 2^20")
    pts = zk.srs_lagrange_setup(tau[0], L)
    torch.cuda.synchronize()
    rng = np.random.default_rng(20)
    idx = [0, 1, n - 1] + [int(i) for i in rng.integers(0, n, 9)]
    ph = _host(zk, pts)
    for j in idx:
        assert points_from_host(ph[j:j + 1])[0] == g1.gen_mul(osrs.lagrange_basis_at(tau[1], n, j)), j
    lag = zk.SRS(pts)
    for name, v in (("quantized", gen.quantized_fr(gen.CONFIG_SEEDS["quantized"], n)),
                    ("uniform", gen.uniform_fr(9200, n))):
        log("lagrange commit 2^20", name)
        com = points_from_host(_host(zk, zk.msm_srs(lag, zk.to_device(v))))[0]
        assert com == g1.gen_mul(ontt.barycentric_eval(fr_from_host(v), tau[1])), name
    lag.close()
    torch.cuda.synchronize()
