"""zk_msm_srs_noalloc, the MSM for callers that cannot allocate, through the
C ABI: bit-exact against zk_msm_srs and the oracle's closed form on two calls
in a row (the second smaller, so it runs over the first call's leftovers in
the shared scratch array), the empty MSM, and a request larger than the
fixed array refused with ZK_EUNSUPPORTED before any work.  The call takes
no scratch from the library's block cache.
"""
import numpy as np
import pytest

from oracle import msm as omsm
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import limbs_to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_07031_amd import zk as m
    return m


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def test_noalloc_msm_matches_msm_srs(zk):
    import torch
    tau = gen.tau_scalar()
    t = limbs_to_ints(tau[None, :])[0]
    log("no-alloc msm: srs setup 2^19")
    srs = zk.SRS(zk.srs_setup(tau, 1 << 19))
    out = torch.empty((1, 16), dtype=torch.int32, device="cuda")
    try:
        for n in (1 << 18, 1000, 0):
            s_h = gen.uniform_fr(9950 + n, max(n, 1))[:max(n, 1)]
            s = zk.to_device(s_h)
            held = zk.scratch_held()
            log("no-alloc msm n=%d" % n)
            zk.msm_srs_noalloc(srs, s, out, n=n)
            got = _host(zk, out).copy()
            assert zk.scratch_held() == held, "the no-alloc call took library scratch"
            ref = _host(zk, zk.msm_srs(srs, s, n=n))
            assert np.array_equal(got, ref), n
            want = omsm.srs_msm_closed_form(t, fr_from_host(s_h)[:n])
            assert points_from_host(got)[0] == want, n
        # beyond the fixed array: refused before any work, output untouched
        big = zk.to_device(gen.uniform_fr(9960, 1 << 19))
        out.fill_(7)
        log("no-alloc msm: oversize request")
        with pytest.raises(zk.ZkError) as ei:
            zk.msm_srs_noalloc(srs, big, out)
        assert ei.value.code == zk.ZK_EUNSUPPORTED
        assert "scratch" in str(ei.value)
        assert bool((out == 7).all())
    finally:
        srs.close()
