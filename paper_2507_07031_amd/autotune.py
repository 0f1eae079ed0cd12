"""Autotuner for the commitment MSM's table policy.

A prepared SRS holds three pre-shifted tables (12-, 16- and 20-bit windows);
which one serves an n-point commitment is a per-SRS threshold policy
(`zk_srs_set_table_policy`).  The best thresholds depend on the device: the
12-bit table has a short reduction (2048 buckets) but more windows, the
20-bit one fewer additions but 16 times the buckets.  `tune` times every feasible table
on the running GPU for power-of-two sizes, picks the thresholds that follow
the measurements, and `apply` installs them; `save` / `load` keep them as a
JSON cache keyed by the device name.  The policy never changes a result, only
its time (the GPU tests check this).

    python -m paper_2507_07031_amd.autotune --out tune.json [--max-log 22]
"""
import argparse
import json

SMALL_CAP = 1 << 16      # the small table covers the first 2^16 points
SMALL, MAIN, LARGE = 12, 16, 20   # window bits of the three tables
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
    """Median time of each feasible table for n = 2^min_log .. 2^max_log
    (n <= srs.n, scalars: device (>= n, 8) tensor) and the policy they imply.
    Returns {"small_max", "large_min", "timings": {n: {window_bits: ms}}}."""
    import torch
    out = torch.empty((1, 16), dtype=torch.int32, device=scalars.device)
    forced = {SMALL: (SMALL_CAP, NEVER), MAIN: (0, NEVER), LARGE: (0, 0)}
    timings = {}
    for lg in range(min_log, max_log + 1):
        n = 1 << lg
        if n > srs.n or n > scalars.shape[0]:
            break
        row = {}
        for bits, (small_max, large_min) in forced.items():
            if bits == SMALL and n >= SMALL_CAP:
                continue
            zk.srs_set_table_policy(srs, small_max, large_min)
            if zk.srs_window_bits(srs, n) != bits:
                continue  # table not built for this SRS
            row[bits] = _time_ms(zk, srs, scalars, n, out, reps)
        timings[n] = row
    policy = derive_policy(timings)
    policy["timings"] = {str(n): {str(b): round(t, 4) for b, t in row.items()} for n, row in timings.items()}
    apply(zk, srs, policy)
    return policy


def derive_policy(timings):
    """Thresholds from {n: {window_bits: ms}}: the small table up to the first
    size where it stops being fastest; the 20-bit table from the first size
    after which it stays fastest."""
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
    return {"small_max": min(small_max, SMALL_CAP), "large_min": large_min}


def apply(zk, srs, policy):
    zk.srs_set_table_policy(srs, int(policy["small_max"]), int(policy["large_min"]))


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
    args = ap.parse_args()
    import torch
    from workloads import generators as gen
    from paper_2507_07031_amd import zk
    n = 1 << args.max_log
    srs = zk.SRS(zk.srs_setup(gen.tau_scalar(), n))
    scalars = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=90))
    policy = tune(zk, srs, scalars, args.min_log, args.max_log, args.reps)
    name = torch.cuda.get_device_name(0)
    save(policy, args.out, name)
    print(json.dumps({"device": name, "small_max": policy["small_max"], "large_min": policy["large_min"]}))


if __name__ == "__main__":
    main()
