"""The commitment does not depend on the table policy (window size), and the
autotuner produces a valid policy: commitments on the small-multiples table
and under forced 12-, 16- and 20-bit-window tables equal each other and the
closed form [f(tau)]_1."""
import pytest

from oracle import msm as omsm
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import limbs_to_ints

pytestmark = pytest.mark.gpu
NEVER = 1 << 62


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
    log("srs setup 2^21 (all three tables)")
    h = zk.SRS(zk.srs_setup(tau[0], 1 << 21))
    torch.cuda.synchronize()
    yield h
    h.close()


def _commit(zk, srs, s, n):
    import torch
    out = zk.msm_srs(srs, s, n=n)
    torch.cuda.synchronize()
    return points_from_host(zk.to_host(out))[0]


@pytest.mark.parametrize("n", [1, 777, 5000, (1 << 14) + 3, (1 << 16) - 1, (1 << 21) - 1])
def test_result_independent_of_window_size(zk, tau, srs, n):
    s_h = gen.uniform_fr(9300 + n, n)
    s = zk.to_device(s_h)
    want = omsm.srs_msm_closed_form(tau[1], fr_from_host(s_h))
    seen = []
    # 4: the small-multiples table (up to 4096 points); 12/16/20: the
    # pre-shifted tables with the small-multiples path off
    paths = {4: (4096, 0, 1 << 21), 12: (0, 1 << 16, NEVER), 16: (0, 0, NEVER), 20: (0, 0, 0)}
    for bits, (tiny_max, small_max, large_min) in paths.items():
        zk.srs_set_tiny_max(srs, tiny_max)
        zk.srs_set_table_policy(srs, small_max, large_min)
        if zk.srs_window_bits(srs, n) != bits:
            continue
        log("msm n=%d window bits %d" % (n, bits))
        assert _commit(zk, srs, s, n) == want, bits
        seen.append(bits)
    zk.srs_set_tiny_max(srs, 4096)
    zk.srs_set_table_policy(srs, 0, 1 << 21)
    assert len(seen) >= 2


def test_autotuner_policy(zk, tau, srs):
    from paper_2507_07031_amd import autotune
    s_h = gen.uniform_fr(9400, 1 << 16)
    s = zk.to_device(s_h)
    log("autotune 2^10..2^16")
    policy = autotune.tune(zk, srs, s, min_log=10, max_log=16, reps=2)
    assert 0 <= policy["small_max"] <= 1 << 16 and 0 <= policy["tiny_max"] <= 4096
    assert set(policy["timings"]) == {str(1 << k) for k in range(10, 17)}
    assert "4" in policy["timings"][str(1 << 10)] and "4" not in policy["timings"][str(1 << 13)]
    for n in (1 << 12, (1 << 16) - 5):
        assert _commit(zk, srs, s, n) == omsm.srs_msm_closed_form(tau[1], fr_from_host(s_h[:n]))
    with pytest.raises(zk.ZkError):
        zk.srs_set_table_policy(srs, (1 << 16) + 1, NEVER)
    zk.srs_set_table_policy(srs, 0, 1 << 21)
    zk.srs_set_tiny_max(srs, 4096)


def test_result_independent_of_schedule(zk, tau, srs):
    # every candidate value of every launch-schedule knob (one at a time, the
    # others at their built-in values) gives the identical commitment (2^16
    # and 2^20 + 3 points, against the closed form), batch and transforms
    import numpy as np
    import torch
    from paper_2507_07031_amd import autotune
    s_h = gen.uniform_fr(9500, (1 << 20) + 3)
    s = zk.to_device(s_h)
    sv = fr_from_host(s_h)
    want = {n: omsm.srs_msm_closed_form(tau[1], sv[:n]) for n in (1 << 16, (1 << 20) + 3)}
    off = np.array([0, 3000, 3000 + (1 << 15), 3000 + (1 << 15) + 70000], dtype=np.uint64)
    ev = zk.to_device(gen.uniform_fr(9501, 1 << 20))
    zk.set_schedule(None)
    ref_batch = zk.to_host(zk.msm_batch(srs, s, off)).copy()
    ref_ntt = zk.to_host(zk.ntt(ev)).copy()
    ref_coset = zk.to_host(zk.coset_ntt(ev, 2)).copy()
    try:
        for knob, values in autotune.SCHEDULE_CANDIDATES.items():
            for v in values:
                zk.set_schedule({knob: v})
                assert zk.get_schedule()[knob] == v
                log("schedule %s=%d" % (knob, v))
                for n, w in want.items():
                    assert _commit(zk, srs, s, n) == w, (knob, v, n)
                assert np.array_equal(zk.to_host(zk.msm_batch(srs, s, off)), ref_batch), (knob, v)
                assert np.array_equal(zk.to_host(zk.ntt(ev)), ref_ntt), (knob, v)
                assert np.array_equal(zk.to_host(zk.coset_ntt(ev, 2)), ref_coset), (knob, v)
        with pytest.raises(zk.ZkError) as ei:
            zk.set_schedule({"sort_chunk": 1000})
        assert ei.value.code == zk.ZK_EINVAL
    finally:
        zk.set_schedule(None)
        torch.cuda.synchronize()


def test_schedule_tuner_runs(zk, srs):
    from paper_2507_07031_amd import autotune
    s = zk.to_device(gen.uniform_fr(9600, 1 << 20))
    ev = zk.to_device(gen.uniform_fr(9601, 1 << 20))
    log("schedule tuner (one round)")
    try:
        res = autotune.tune_schedule(zk, srs, s, ev, reps=1)
        assert set(res["schedule"]) == set(zk.SCHEDULE_FIELDS)
        assert res["mix_ms"] <= res["default_mix_ms"]
        assert zk.get_schedule() == res["schedule"]
    finally:
        zk.set_schedule(None)


@pytest.mark.parametrize("log_n", [10, 13, 14, 17, 20, 21, 25])
def test_transforms_independent_of_tile(zk, log_n):
    # every transform tile (2^10..2^12 points) and stages per LDS round trip
    # (2 or 3) gives the identical NTT, iNTT and 4x coset evaluations; where a
    # tile cannot hold a pass's transforms (2^21 and up for 2^10-point tiles)
    # the planner takes the smallest tile that does; 2^25 runs three passes
    import torch
    n = 1 << log_n
    if log_n <= 21:
        ev = zk.to_device(gen.uniform_fr(9600 + log_n, n))
    else:
        # canonical values made on the device: random words below 2^253 < r
        g = torch.Generator(device="cuda")
        g.manual_seed(9600 + log_n)
        ev = torch.randint(-(1 << 31), (1 << 31) - 1, (n, 8), dtype=torch.int32, device="cuda", generator=g)
        ev[:, 7] &= 0x1FFFFFFF
    zk.set_schedule(None)
    fns = (zk.ntt, zk.intt, lambda x: zk.coset_ntt(x, 2))
    refs = [f(ev).clone() for f in fns]
    try:
        for tile in (10, 11, 12):
            for unit in (2, 3):
                zk.set_schedule({"ntt_tile_log": tile, "ntt_unit_log": unit, "ntt_overlap_tile_log": tile})
                log("transforms 2^%d tile 2^%d unit %d" % (log_n, tile, unit))
                for f, r in zip(fns, refs):
                    got = f(ev)
                    assert torch.equal(got, r), (log_n, tile, unit)
                    del got
        with pytest.raises(zk.ZkError) as ei:
            zk.set_schedule({"ntt_tile_log": 9})
        assert ei.value.code == zk.ZK_EINVAL
    finally:
        zk.set_schedule(None)
        torch.cuda.synchronize()
        del refs
        torch.cuda.empty_cache()
        zk.release_cached_memory()
