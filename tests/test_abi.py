"""The C-ABI library loads, exports every function include/zk.h declares, and
rejects bad arguments before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "zk.h")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:zk_status|const char\*|uint64_t|uint32_t)\s+(zk_\w+)\(", text, re.M)))


@pytest.fixture(scope="module")
def zk():
    from paper_2507_07031_amd import zk as m
    return m


def test_header_lists_the_hot_path_calls():
    names = declared_functions()
    for required in ("zk_ntt", "zk_intt", "zk_coset_ntt", "zk_msm", "zk_msm_batch", "zk_fold"):
        assert required in names


def test_library_exports_every_declared_symbol(zk):
    raw = ctypes.CDLL(zk.LIB_PATH)
    for name in declared_functions():
        assert hasattr(raw, name), name
    assert set(declared_functions()) == set(zk.EXPORTS)


def test_argument_errors_return_before_device_work(zk):
    L = zk.lib
    null = ctypes.c_void_p(0)
    assert L.zk_ntt(null, null, 3, null) == zk.ZK_EINVAL
    assert L.zk_intt(null, null, 3, null) == zk.ZK_EINVAL
    assert "NULL" in L.zk_last_error().decode()
    dummy = ctypes.c_void_p(0x1000)
    assert L.zk_ntt(dummy, dummy, 29, null) == zk.ZK_EUNSUPPORTED
    assert L.zk_coset_ntt(dummy, 24, 5, null, dummy, null) == zk.ZK_EUNSUPPORTED
    assert L.zk_msm(null, null, 4, dummy, null) == zk.ZK_EINVAL
    assert L.zk_msm_srs(null, dummy, 4, dummy, null) == zk.ZK_EINVAL
    assert L.zk_msm_batch(null, dummy, dummy, 1, dummy, null) == zk.ZK_EINVAL
    assert L.zk_fold(dummy, null, 3, 1, dummy, null) == zk.ZK_EINVAL
    assert L.zk_fold(dummy, dummy, 0, 1, dummy, null) == zk.ZK_EINVAL
    assert L.zk_msm_srs_ex(null, dummy, 4, dummy, null, null) == zk.ZK_EINVAL
    assert L.zk_commit_job(null, dummy, 4, 2, null, dummy, dummy, dummy, null) == zk.ZK_EINVAL
    assert L.zk_commit_job(dummy, dummy, 4, 2, null, dummy, null, dummy, null) == zk.ZK_EINVAL
    assert L.zk_commit_job(dummy, dummy, 24, 5, null, dummy, dummy, dummy, null) == zk.ZK_EUNSUPPORTED
    assert L.zk_set_validate(0) == zk.ZK_OK
    # the scratch budget is per device: without one the call reports the device error
    assert L.zk_set_scratch_budget(0) in (zk.ZK_OK, zk.ZK_EDEVICE)
    assert zk.ZK_EBUDGET == -4
    assert L.zk_kzg_open(null, dummy, 4, dummy, dummy, null, dummy, null) == zk.ZK_EINVAL
    assert L.zk_quotient_mul(null, dummy, dummy, dummy, 4, 1, null, dummy, dummy, null) == zk.ZK_EINVAL
    assert L.zk_quotient_mul(dummy, dummy, dummy, dummy, 4, 0, null, dummy, dummy, null) == zk.ZK_EINVAL
    assert L.zk_kzg_open_batch(dummy, dummy, 0, 4, dummy, dummy, dummy, null, dummy, null) == zk.ZK_EINVAL
    assert L.zk_kzg_open_batch(dummy, dummy, 2, 4, dummy, null, dummy, null, dummy, null) == zk.ZK_EINVAL
    assert L.zk_srs_size(null) == 0
    assert L.zk_srs_destroy(null) == zk.ZK_OK
    # tau >= r is rejected
    bad = (ctypes.c_uint32 * 8)(*([0xFFFFFFFF] * 8))
    assert L.zk_srs_setup(ctypes.cast(bad, ctypes.c_void_p), 4, dummy, null) == zk.ZK_EINVAL
    assert "canonical" in L.zk_last_error().decode()
    assert L.zk_srs_lagrange_setup(ctypes.cast(bad, ctypes.c_void_p), 4, dummy, null) == zk.ZK_EINVAL
    assert L.zk_srs_lagrange_setup(null, 4, dummy, null) == zk.ZK_EINVAL
    assert L.zk_transcript_challenge(null, 4, dummy, null) == zk.ZK_EINVAL
    assert L.zk_acc_fold(1, dummy, dummy, 0, dummy, dummy, null, 0, null, null, 0, null, null, null, dummy, dummy,
                         dummy, null, null, null) == zk.ZK_EINVAL
    assert L.zk_acc_fold(1, dummy, dummy, 2, dummy, dummy, null, 0, null, null, 0, null, null, null, dummy, dummy,
                         dummy, null, null, null) == zk.ZK_EINVAL
