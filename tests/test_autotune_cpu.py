"""The autotuner's threshold derivation and cache on the CPU (timings given)."""
import json

from paper_2507_07031_amd import autotune


class FakeZk:
    def __init__(self):
        self.policy = None

        self.tiny = None

    def srs_set_table_policy(self, srs, small_max, large_min):
        self.policy = (small_max, large_min)

    def srs_set_tiny_max(self, srs, tiny_max):
        self.tiny = tiny_max


def test_save_load_roundtrip(tmp_path):
    p = tmp_path / "tune.json"
    autotune.save({"small_max": 100, "large_min": 5}, str(p), "devA")
    autotune.save({"small_max": 7, "large_min": 9}, str(p), "devB")
    assert autotune.load(str(p), "devA") == {"small_max": 100, "large_min": 5}
    assert json.load(open(p))["devB"]["large_min"] == 9


def test_apply_sets_policy():
    z = FakeZk()
    autotune.apply(z, object(), {"small_max": 1024, "large_min": 1 << 20})
    assert z.policy == (1024, 1 << 20) and z.tiny == autotune.TINY_CAP
    autotune.apply(z, object(), {"tiny_max": 0, "small_max": 0, "large_min": 1 << 21})
    assert z.tiny == 0


def test_derive_policy_follows_timings():
    t = {1024: {12: 0.1, 16: 0.2}, 2048: {12: 0.15, 16: 0.2}, 4096: {12: 0.3, 16: 0.25},
         1 << 16: {16: 1.0, 20: 1.2}, 1 << 20: {16: 2.0, 20: 1.9}, 1 << 21: {16: 4.0, 20: 3.1}}
    assert autotune.derive_policy(t) == {"tiny_max": 0, "small_max": 2049, "large_min": 1 << 20}
    # 20-bit never fastest at the top: no large threshold; 12-bit never fastest: 0
    t2 = {1024: {12: 0.3, 16: 0.2}, 1 << 21: {16: 3.0, 20: 3.1}}
    assert autotune.derive_policy(t2) == {"tiny_max": 0, "small_max": 0, "large_min": autotune.NEVER}
    # the small-table threshold never passes the table's 2^16 points
    t3 = {1 << 16: {12: 0.1, 16: 0.2}}
    assert autotune.derive_policy(t3)["small_max"] == 1 << 16


def test_derive_policy_small_multiples():
    # fastest up to 2048, then the tables win: tiny_max 2048, and the table
    # thresholds are derived among the tables alone
    t = {1024: {4: 0.1, 12: 0.3, 16: 0.35}, 2048: {4: 0.2, 12: 0.31, 16: 0.36},
         4096: {4: 0.5, 12: 0.33, 16: 0.4}, 8192: {12: 0.5, 16: 0.45}}
    assert autotune.derive_policy(t) == {"tiny_max": 2048, "small_max": 4097, "large_min": autotune.NEVER}
    # not fastest at the smallest size: off, whatever happens above
    t2 = {1024: {4: 0.5, 16: 0.4}, 2048: {4: 0.1, 16: 0.4}}
    assert autotune.derive_policy(t2)["tiny_max"] == 0
    # never above the table's 4096 points
    t3 = {4096: {4: 0.1, 16: 0.4}}
    assert autotune.derive_policy(t3)["tiny_max"] == 4096


class FakeZkSchedule(FakeZk):
    def __init__(self):
        super().__init__()
        self.schedule = None

    def set_schedule(self, values):
        self.schedule = values


def test_apply_sets_schedule():
    z = FakeZkSchedule()
    autotune.apply(z, object(), {"small_max": 0, "large_min": 1 << 21, "schedule": {"sort_chunk": 2048}})
    assert z.policy == (0, 1 << 21) and z.schedule == {"sort_chunk": 2048}


def test_schedule_candidates_are_valid():
    # the built-in value comes first, and every value is inside the range
    # zk_set_schedule accepts
    c = autotune.SCHEDULE_CANDIDATES
    assert c["acc_max_slice"][0] == 256 and all(16 <= v <= 4096 for v in c["acc_max_slice"])
    assert c["acc_blocks_per_cu"][0] == 2 and all(1 <= v <= 4 for v in c["acc_blocks_per_cu"])
    assert c["reduce_chunk"][0] == 0 and all(v == 0 or (v & (v - 1)) == 0 and v <= 64 for v in c["reduce_chunk"])
    assert c["sort_chunk"][0] == 1024 and all((v & (v - 1)) == 0 and 256 <= v <= 16384 for v in c["sort_chunk"])
    assert all((v & (v - 1)) == 0 and 1 << 10 <= v <= 1 << 20 for v in c["sort_bin_entries"])
    assert c["ntt_tile_log"] == [11, 12, 10] and c["ntt_unit_log"] == [3, 2]
    assert c["ntt_overlap_tile_log"] == [11, 12, 10]
