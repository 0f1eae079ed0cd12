"""GPU tests of the scratch budget (zk_set_scratch_budget / ZK_EBUDGET): a
call whose scratch would exceed the budget fails before enqueuing its work
and leaves its output untouched; within the budget results are bit-identical
to unbudgeted calls; a budget below the cached bytes frees the cache first.
"""
import numpy as np
import pytest

from tests.gpu_helpers import log
from workloads import generators as gen

pytestmark = pytest.mark.gpu
MiB = 1 << 20


@pytest.fixture(scope="module")
def zk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_07031_amd import zk as m
    m.set_scratch_budget(0)
    yield m
    m.set_scratch_budget(0)


@pytest.fixture(scope="module")
def srs(zk):
    h = zk.SRS(zk.srs_setup(gen.tau_scalar(), 1 << 16))
    yield h
    h.close()


def test_budget_refuses_and_admits(zk, srs):
    import torch
    x = zk.to_device(gen.uniform_fr(5100, 1 << 20))
    log("budget: unbudgeted reference")
    ref = zk.ntt(x)
    s = zk.to_device(gen.uniform_fr(5101, 1 << 16))
    ref_msm = zk.msm_srs(srs, s)
    torch.cuda.synchronize()
    try:
        zk.release_cached_memory()
        assert zk.scratch_held() == 0
        zk.set_scratch_budget(1 * MiB)
        out = torch.full_like(x, 7)
        log("budget: 2^20 transform over a 1 MiB budget")
        with pytest.raises(zk.ZkError) as ei:
            zk.ntt(x, out=out)
        assert ei.value.code == zk.ZK_EBUDGET
        torch.cuda.synchronize()
        assert bool((out == 7).all())  # nothing was enqueued
        assert zk.scratch_held() <= 1 * MiB
        with pytest.raises(zk.ZkError) as ei:
            zk.msm_srs(srs, s)
        assert ei.value.code == zk.ZK_EBUDGET

        need = zk.ntt_workspace_bytes(20)
        zk.set_scratch_budget(need + 4 * MiB)
        log("budget: 2^20 transform within its budget")
        zk.ntt(x, out=out)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        held = zk.scratch_held()
        assert need <= held <= need + 4 * MiB

        # the cached transform block counts: a budget for the MSM's workspace
        # alone is met by freeing the cache first
        w = zk.msm_srs_workspace_bytes(srs, 1 << 16)
        zk.set_scratch_budget(w + 4 * MiB)
        log("budget: MSM 2^16 after a cached transform block")
        got = zk.msm_srs(srs, s)
        torch.cuda.synchronize()
        assert torch.equal(got, ref_msm)
        assert zk.scratch_held() <= w + 4 * MiB
    finally:
        zk.set_scratch_budget(0)


def test_budget_zero_is_unlimited(zk):
    import torch
    zk.set_scratch_budget(0)
    x = zk.to_device(gen.uniform_fr(5102, 1 << 22))
    log("budget: none, 2^22 transform")
    y = zk.intt(zk.ntt(x))
    torch.cuda.synchronize()
    assert torch.equal(y, x)
    assert zk.scratch_held() >= zk.ntt_workspace_bytes(22)
