"""Autotuner for the commitment MSM's window size and bucket/tile schedule.

Two kinds of knobs, neither of which changes any result (the GPU tests check
this), only times:

* Window size.  A prepared SRS holds three pre-shifted tables (12-, 16- and
  20-bit windows); which one serves an n-point commitment is a per-SRS
  threshold policy (`zk_srs_set_table_policy`).  The 12-bit table has a
  short reduction (2048 buckets) but more windows, the 20-bit one fewer
  additions but 16 times the buckets.  Up to 4096 points a commitment can
  also run on the table of small multiples (4-bit digits summed by trees,
  no buckets; `zk_srs_set_tiny_max`).  `tune` times every feasible path on
  the running GPU for power-of-two sizes and picks the thresholds that
  follow the measurements.
* Launch schedule (`zk_set_schedule`, per device): the accumulation slice
  cap and workgroups per compute unit, the bucket reduction's chunk length,
  the coarse-sort workgroup size and coarse-bin target, and the transform
  tile and stages per LDS round trip.  `tune_schedule` runs a coordinate descent over candidate values,
  timing a mix of the library's work (commitments of 2^16 and 2^20 points
  and the 2^20 commit job with its transforms), and keeps each value that
  lowers the mix's time.

`apply` installs a result on an SRS and the current device; `save` / `load`
keep results as a JSON cache keyed by the device name.

    python -m paper_2507_07031_amd.autotune --out tune.json [--max-log 22] [--schedule]
"""
import argparse
import json

SMALL_CAP = 1 << 16      # the small table covers the first 2^16 points
TINY_CAP = 1 << 12       # the small-multiples table covers the first 4096 points
TINY, SMALL, MAIN, LARGE = 4, 12, 16, 20   # window bits of the four paths
NEVER = 1 << 62


def _time_ms(zk, srs, scalars, n, out, reps):
    import torch
    zk.msm_srs(srs, scalars, n=n, out=out)
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        zk.msm_srs(srs, scalars, n=n, out=out)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune(zk, srs, scalars, min_log=10, max_log=22, reps=5):
    """Median time of each feasible path for n = 2^min_log .. 2^max_log
    (n <= srs.n, scalars: device (>= n, 8) tensor) and the policy they imply.
    Returns {"tiny_max", "small_max", "large_min", "timings": {n: {window_bits: ms}}}."""
    import torch
    out = torch.empty((1, 16), dtype=torch.int32, device=scalars.device)
    forced = {SMALL: (SMALL_CAP, NEVER), MAIN: (0, NEVER), LARGE: (0, 0)}
    timings = {}
    for lg in range(min_log, max_log + 1):
        n = 1 << lg
        if n > srs.n or n > scalars.shape[0]:
            break
        row = {}
        zk.srs_set_tiny_max(srs, 0)
        for bits, (small_max, large_min) in forced.items():
            if bits == SMALL and n >= SMALL_CAP:
                continue
            zk.srs_set_table_policy(srs, small_max, large_min)
            if zk.srs_window_bits(srs, n) != bits:
                continue  # table not built for this SRS
            row[bits] = _time_ms(zk, srs, scalars, n, out, reps)
        if n <= TINY_CAP:
            zk.srs_set_tiny_max(srs, TINY_CAP)
            if zk.srs_window_bits(srs, n) == TINY:
                row[TINY] = _time_ms(zk, srs, scalars, n, out, reps)
        timings[n] = row
    policy = derive_policy(timings)
    policy["timings"] = {str(n): {str(b): round(t, 4) for b, t in row.items()} for n, row in timings.items()}
    apply(zk, srs, policy)
    return policy


def derive_policy(timings):
    """Thresholds from {n: {window_bits: ms}}: the small-multiples path up to
    the last size of the run of sizes (from the smallest) where it is fastest;
    among the tables, the small one up to the first size where it stops
    being fastest and the 20-bit one from the first size after which it stays
    fastest."""
    tiny_max = 0
    for n in sorted(timings):
        row = timings[n]
        if TINY in row and row[TINY] <= min(row.values()):
            tiny_max = n
        else:
            break
    tables = {n: {b: t for b, t in row.items() if b != TINY} for n, row in timings.items()}
    timings = {n: row for n, row in tables.items() if row}
    small_max = 0
    for n in sorted(timings):
        row = timings[n]
        if SMALL in row and row[SMALL] <= min(row.values()):
            small_max = n + 1
        else:
            break
    large_min = NEVER
    for n in sorted(timings, reverse=True):
        row = timings[n]
        if LARGE in row and row[LARGE] <= min(row.values()):
            large_min = n
        else:
            break
    return {"tiny_max": min(tiny_max, TINY_CAP), "small_max": min(small_max, SMALL_CAP), "large_min": large_min}


# Candidate values per schedule knob (the built-in value first).
SCHEDULE_CANDIDATES = {
    "acc_max_slice": [256, 128, 512, 64],
    "acc_blocks_per_cu": [2, 1, 3],
    "reduce_chunk": [0, 4, 8, 16, 32],
    "sort_chunk": [1024, 512, 2048, 4096],
    "sort_bin_entries": [32768, 8192, 131072],
    "ntt_tile_log": [11, 12, 10],
    "ntt_unit_log": [3, 2],
    "ntt_overlap_tile_log": [11, 12, 10],
}


def _mix_ms(zk, srs, scalars, evals, out, reps):
    """Median time of the mix: commitments of 2^16 and 2^20 points and the
    2^20 commit job (iNTT, commitment, 4x coset transform)."""
    import torch
    n20 = min(1 << 20, srs.n, scalars.shape[0])
    coset = torch.empty((4 * evals.shape[0], 8), dtype=torch.int32, device=evals.device)
    coeffs = torch.empty_like(evals)

    def run():
        zk.msm_srs(srs, scalars, n=min(1 << 16, n20), out=out)
        zk.msm_srs(srs, scalars, n=n20, out=out)
        zk.commit_job(srs, evals, log_blowup=2, coeffs=coeffs, com=out, coset=coset)
    run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    times.sort()
    return times[len(times) // 2]


def tune_schedule(zk, srs, scalars, evals, reps=7, rounds=1, gain=0.02):
    """Coordinate descent over SCHEDULE_CANDIDATES on the current device: a
    value replaces the current one only if the mix's median time drops by
    more than `gain`; at the end the chosen schedule is timed again against
    the built-in one (twice the repetitions) and kept only if it is still
    faster.  Returns {"schedule": {knob: value}, "timings": {knob: {value:
    ms}}, "mix_ms": best, "default_mix_ms": with the built-in schedule}."""
    import torch
    out = torch.empty((1, 16), dtype=torch.int32, device=scalars.device)
    zk.set_schedule(None)
    default = zk.get_schedule()
    best = dict(default)
    best_ms = _mix_ms(zk, srs, scalars, evals, out, reps)
    timings = {}
    for _ in range(rounds):
        for knob, values in SCHEDULE_CANDIDATES.items():
            row = timings.setdefault(knob, {})
            for v in values:
                trial = dict(best)
                trial[knob] = v
                zk.set_schedule(trial)
                ms = _mix_ms(zk, srs, scalars, evals, out, reps)
                row[str(v)] = round(ms, 4)
                if ms < best_ms * (1.0 - gain):
                    best, best_ms = zk.get_schedule(), ms
            zk.set_schedule(best)
    # confirm against the built-in schedule
    zk.set_schedule(default)
    default_ms = _mix_ms(zk, srs, scalars, evals, out, 2 * reps)
    zk.set_schedule(best)
    chosen_ms = _mix_ms(zk, srs, scalars, evals, out, 2 * reps)
    if chosen_ms >= default_ms:
        best, chosen_ms = default, default_ms
    zk.set_schedule(best)
    return {"schedule": best, "timings": timings, "mix_ms": round(chosen_ms, 4),
            "default_mix_ms": round(default_ms, 4)}


def apply(zk, srs, policy):
    zk.srs_set_table_policy(srs, int(policy["small_max"]), int(policy["large_min"]))
    zk.srs_set_tiny_max(srs, int(policy.get("tiny_max", TINY_CAP)))
    if policy.get("schedule"):
        zk.set_schedule(policy["schedule"])


def save(policy, path, device_name):
    try:
        with open(path) as f:
            cache = json.load(f)
    except (OSError, ValueError):
        cache = {}
    cache[device_name] = policy
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)


def load(path, device_name):
    with open(path) as f:
        return json.load(f).get(device_name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="tune.json")
    ap.add_argument("--min-log", type=int, default=10)
    ap.add_argument("--max-log", type=int, default=22)
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--schedule", action="store_true", help="also tune the launch schedule")
    args = ap.parse_args()
    import torch
    from workloads import generators as gen
    from paper_2507_07031_amd import zk
    n = 1 << args.max_log
    srs = zk.SRS(zk.srs_setup(gen.tau_scalar(), n))
    scalars = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=90))
    policy = tune(zk, srs, scalars, args.min_log, args.max_log, args.reps)
    if args.schedule:
        evals = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], min(n, 1 << 20), tag=91))
        sched = tune_schedule(zk, srs, scalars, evals, args.reps)
        policy["schedule"] = sched["schedule"]
        policy["schedule_timings"] = sched["timings"]
        policy["mix_ms"], policy["default_mix_ms"] = sched["mix_ms"], sched["default_mix_ms"]
    name = torch.cuda.get_device_name(0)
    save(policy, args.out, name)
    print(json.dumps({"device": name, "tiny_max": policy["tiny_max"], "small_max": policy["small_max"],
                      "large_min": policy["large_min"],
                      "schedule": policy.get("schedule"), "mix_ms": policy.get("mix_ms"),
                      "default_mix_ms": policy.get("default_mix_ms")}))


if __name__ == "__main__":
    main()
