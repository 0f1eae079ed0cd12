#!/usr/bin/env python3
"""Benchmark of the KZG commit / fold hot path on one MI355X.

One step = the large basic-block commit job, inputs resident in HBM:
2^20 uniform Fr evaluations -> inverse NTT -> MSM of the 2^20 coefficients
against the prepared SRS [tau^i]_1 -> 4x coset NTT (2^20 -> 2^22).
`value` is that job's throughput in committed points per second.

Printed as one JSON line, with
* per-operation throughputs (MSM points/s, NTT / iNTT / coset elements/s),
* the quantized-activation MSM at 2^22 against uniform scalars at 2^22,
* 256 uneven MSMs (log-uniform 2^8..2^18) batched vs one call each, and the
  fold of 64 of the resulting commitments,
* small commitments (2^8..2^14) on the small-multiples table and as bucket
  runs,
* `roofline` of the dominant kernel (bucket accumulation) from HIP events
  recorded by the library on its launch stream over the timed region,
* a Poisson stream of commit jobs (2^10..2^22 points) through the serving
  loop: p50 / p99 latency and jobs/s, continuous admission vs serial,
* the same job with its host transfers (evaluations in from pinned memory,
  commitment back), beside the device-resident figure,
* `cpu_baseline`: the CPU oracle on a bounded sample of the same job.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from workloads import generators as gen  # noqa: E402

PEAK_HBM_GBS = 8000.0
# v_mad_u64_u32 issues once per lane per cycle: 256 CUs x 64 lanes x 2.4 GHz
PEAK_MAD_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic word products of one 256-bit Montgomery product with 32-bit
# words (operand-scanning CIOS: 8x8 for a*b, 8x8 for m*q, 8 for the m_i)
MADS_PER_MONT = 136
# Fq products of a mixed XYZZ addition (8M + 2S)
MONT_PER_MADD = 10
# Fq products of a mixed G2 XYZZ addition: 8 Fq2 products x 3 + 2 Fq2 squares x 2
G2_FQ_PER_MADD = 28
# HBM bytes of one accumulate dispatch of this workload, from rocprofv3
# FETCH_SIZE / WRITE_SIZE scaled by a plain-copy calibration (x2.0 / x1.0);
# valid only for the kernel sources whose hash is recorded with it.
ACCUMULATE_TRAFFIC = {"sources_sha256_16": "82f7235ce059198c", "bytes": 2725963396}
TRAFFIC_SOURCES = ("msm_accumulate.hip", "msm_store.h", "msm.h", "curve.h", "field.h", "field_constants.h")


def kernel_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2507_07031_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def nonzero_digits(scalars_u32, c):
    """Exact number of nonzero signed c-bit digits after the negation trick:
    the number of mixed additions bucket accumulation must perform."""
    s = np.array(scalars_u32, dtype=np.uint64)
    r = np.array([(gen.FR_MODULUS >> (32 * i)) & 0xFFFFFFFF for i in range(8)], dtype=np.uint64)
    half = np.array([((gen.FR_MODULUS - 1) // 2 >> (32 * i)) & 0xFFFFFFFF for i in range(8)], dtype=np.uint64)
    gt = np.zeros(s.shape[0], dtype=bool)
    eq = np.ones(s.shape[0], dtype=bool)
    for i in range(7, -1, -1):
        gt |= eq & (s[:, i] > half[i])
        eq &= s[:, i] == half[i]
    neg = s.copy()
    borrow = np.zeros(s.shape[0], dtype=np.uint64)
    for i in range(8):
        d = r[i] - s[:, i] - borrow
        borrow = (r[i] < s[:, i] + borrow).astype(np.uint64)
        neg[:, i] = d & 0xFFFFFFFF
    s = np.where(gt[:, None], neg, s)
    s = np.concatenate([s, np.zeros((s.shape[0], 1), dtype=np.uint64)], axis=1)
    W = (254 + c - 1) // c
    carry = np.zeros(s.shape[0], dtype=np.int64)
    count = 0
    for w in range(W):
        o = c * w
        j, sh = o // 32, o % 32
        two = s[:, j] | (s[:, j + 1] << np.uint64(32))
        d = ((two >> np.uint64(sh)) & np.uint64((1 << c) - 1)).astype(np.int64) + carry
        big = d > (1 << (c - 1))
        mag = np.where(big, (1 << c) - d, d)
        carry = big.astype(np.int64)
        count += int(np.count_nonzero(mag))
    return count


def g2_nonzero_digits(scalars_u32):
    """Nonzero signed 8-bit digits of the G2 MSM's recoding (32 windows, no
    negation trick): the number of mixed G2 additions it performs."""
    b = np.ascontiguousarray(np.asarray(scalars_u32, dtype=np.uint32)).view(np.uint8).reshape(-1, 32)
    carry = np.zeros(b.shape[0], dtype=np.int64)
    count = 0
    for w in range(32):
        v = b[:, w].astype(np.int64) + carry
        big = v > 128
        carry = big.astype(np.int64)
        count += int(np.count_nonzero(np.where(big, v - 256, v)))
    return count


# ----------------------------------------------------------------- CPU oracle

def _oracle_srs_chunk(args):
    tau, lo, hi = args
    from oracle import srs as osrs
    return [osrs.srs_point(tau, i) for i in range(lo, hi)]


def _oracle_naive_sum(args):
    pts, scal = args
    from oracle import g1, msm as omsm
    return g1.encode(omsm.naive_msm(pts, scal))


def cpu_baseline(tau_int, log_n=12):
    """The oracle on a 2^12-point commit job: inverse transform, naive MSM over
    the oracle's own SRS (split over every host core), 4x coset evaluation."""
    from oracle import g1, msm as omsm, ntt as ontt
    n = 1 << log_n
    cores = len(os.sched_getaffinity(0))
    evals = gen.limbs_to_ints(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=99))
    chunks = [(i * n // cores, (i + 1) * n // cores) for i in range(cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        srs_parts = pool.map(_oracle_srs_chunk, [(tau_int, lo, hi) for lo, hi in chunks])  # setup, untimed
        t0 = time.perf_counter()
        coeffs = ontt.ifft(evals)
        parts = pool.map(_oracle_naive_sum, [(srs_parts[k], coeffs[lo:hi]) for k, (lo, hi) in enumerate(chunks)])
        acc = None
        for p in parts:
            acc = g1.add(acc, g1.decode(p))
        ontt.coset_evals(coeffs, 2, 5)
        dt = time.perf_counter() - t0
    base = {"value": n / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "2^12-point commit job (oracle iNTT 2^12, naive MSM of 2^12 points split over %d "
                      "processes, 4x coset 2^12->2^14); %.1f s wall" % (cores, dt)}
    # single-core figures of the oracle's routines: the naive MSM at 2^10
    # (linear in n, so its 2^20 time is an extrapolation and labelled so),
    # the DFT at 2^12 and the recursive FFT at 2^20, timed directly
    pts = [p for part in srs_parts for p in part][:1 << 10]
    sc = gen.limbs_to_ints(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1 << 10, tag=98))
    t0 = time.perf_counter()
    omsm.naive_msm(pts, sc)
    t_msm = time.perf_counter() - t0
    a12 = gen.limbs_to_ints(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1 << 12, tag=97))
    t0 = time.perf_counter()
    ontt.dft(a12)
    t_dft = time.perf_counter() - t0
    a20 = gen.limbs_to_ints(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1 << 20, tag=96))
    t0 = time.perf_counter()
    ontt.fft(a20)
    t_fft = time.perf_counter() - t0
    detail = {"cores": 1,
              "naive_msm_2^10_s": round(t_msm, 3), "naive_msm_points_per_s": round((1 << 10) / t_msm, 1),
              "naive_msm_2^20_s_extrapolated": round(t_msm * 1024, 1),
              "dft_2^12_s": round(t_dft, 3), "fft_2^20_s": round(t_fft, 3),
              "fft_2^20_elems_per_s": round((1 << 20) / t_fft, 1)}
    return base, detail


# ----------------------------------------------------------------- GPU

def serving_runs(zk, srs, srs_pts, count):
    """Poisson streams of commit-and-fold jobs (sizes log-uniform 2^10..2^22;
    each job commits its witness and folds the commitment into its input
    accumulator) through the continuous-admission loop, swept over the
    offered rate: 4 stream slots against one slot (plain per-call serial
    execution of the same stream), both at a 64 GiB budget, plus 4 slots at
    a tight 4 GiB budget at the workload's 200 jobs/s.  Each record gives
    achieved jobs/s, p50/p99 latency and the peak HBM the jobs held (caller
    buffers, and the library's scratch including its cache)."""
    from paper_2507_07031_amd.serve import GpuExecutor, Job, serve, summarize
    import torch
    seed = gen.CONFIG_SEEDS["serving"]
    sizes = gen.log_uniform_sizes(seed, count, 10, 22)
    pool_n = 1 << 23
    pool = zk.to_device(gen.uniform_fr(seed, pool_n, tag=1))
    acc_pool = srs_pts[:4096].contiguous()
    rng = gen.rng_for(seed, 2)
    offs = rng.integers(0, pool_n - (1 << 22), size=count)
    accs = rng.integers(0, 4096, size=count)
    out = {"jobs_per_point": count, "size_log2_range": [10, 22], "job": "commit (iNTT, MSM, 4x coset) + fold",
           "points": []}
    runs = [(rate, "continuous_4slots", 4, 64 << 30) for rate in (200.0, 400.0, 800.0, 1600.0)]
    runs += [(rate, "serial_1slot", 1, 64 << 30) for rate in (200.0, 400.0, 800.0, 1600.0)]
    runs += [(200.0, "continuous_4slots_4GiB", 4, 4 << 30)]
    for rate, mode, slots, budget in runs:
        arrivals = gen.poisson_arrivals(seed, count, rate)
        jobs = [Job(i, int(n), float(a), int(o), int(c))
                for i, (n, a, o, c) in enumerate(zip(sizes, arrivals, offs, accs))]
        zk.release_cached_memory()
        torch.cuda.synchronize()
        ex = GpuExecutor(zk, srs, pool, slots, acc_pool=acc_pool, budget=budget)
        fin, rej, wall = serve(jobs, ex, budget, slots)
        torch.cuda.synchronize()
        rec = summarize(fin, wall)
        rec.update({"offered_jobs_per_s": rate, "mode": mode, "slots": slots, "budget_gib": budget >> 30,
                    "rejected": len(rej), "peak_scratch_held_mb": round(ex.peak_scratch / 2 ** 20, 1),
                    "peak_caller_mb": round(ex.peak_caller / 2 ** 20, 1), "busy_refusals": ex.busy_events})
        out["points"].append({k: (round(v, 4) if isinstance(v, float) else v) for k, v in rec.items()})
        log("serving %s %.0f/s: %.1f jobs/s p99 %.2f ms" % (mode, rate, rec.get("jobs_per_s", 0),
                                                             rec.get("p99_ms", 0)))
    zk.set_scratch_budget(0)
    for mode in ("continuous_4slots", "serial_1slot"):
        pts = [p for p in out["points"] if p["mode"] == mode]
        out["saturation_jobs_per_s_" + mode] = max(p.get("jobs_per_s", 0) for p in pts)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=1000)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy and a 2^24-element Fr fold (counter calibration)")
    ap.add_argument("--mad-calibration", action="store_true",
                    help="only measure the sustained v_mad_u64_u32 rate (the integer roof's basis)")
    ap.add_argument("--transforms-only", action="store_true",
                    help="only run the commit workload's transforms (NTT, iNTT 2^20, 4x coset 2^20 -> 2^22), "
                         "for counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(requested --gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_07031_amd import zk

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written per dispatch
        src = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        # a second kernel of known traffic: the accumulation step's Fr part
        # v'' = gamma v + v' over 2^24 elements (fr_rlc_kernel reads 64 B and
        # writes 32 B per element: 1 GiB in, 0.5 GiB out per dispatch)
        ln = 1 << 24
        va = zk.to_device(gen.uniform_fr(7, ln, tag=1))
        vb = zk.to_device(gen.uniform_fr(7, ln, tag=2))
        gam = zk.to_device(gen.uniform_fr(7, 1, tag=3))
        pt = zk.srs_setup(gen.tau_scalar(), 1)
        for _ in range(3):
            zk.acc_fold(gam, pt, pt, pt, pt, None, va, vb)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30, "dispatches": 3,
                          "fr_rlc_read_bytes": 64 * ln, "fr_rlc_write_bytes": 32 * ln, "fr_rlc_dispatches": 3}))
        return
    if args.mad_calibration:
        # 2048 workgroups x 256 threads x 8 dependent chains x 4096 x 16 steps
        rates = [zk.calibrate_mad_rate(2048, 4096) for _ in range(5)]
        best = max(rates)
        print(json.dumps({"mad_rate_tops": [round(r / 1e12, 3) for r in rates], "best_tops": round(best / 1e12, 3),
                          "issue_peak_tops": round(PEAK_MAD_TOPS, 3),
                          "sustained_over_issue_peak": round(best / 1e12 / PEAK_MAD_TOPS, 4),
                          "products_per_run": 2048 * 256 * 4096 * 16 * 8}))
        return
    n = 1 << 20
    if args.transforms_only:
        # the transforms of the 2^20 commit workload, each called `steps` times
        x = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n))
        y = torch.empty_like(x)
        cos = torch.empty((4 * n, 8), dtype=torch.int32, device=dev)
        res = {}
        for name, fn in (("ntt_2^20", lambda: zk.ntt(x, out=y)), ("intt_2^20", lambda: zk.intt(x, out=y)),
                         ("coset_2^20->2^22", lambda: zk.coset_ntt(x, 2, out=cos))):
            fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                fn()
            torch.cuda.synchronize()
            res[name + "_ms"] = round((time.perf_counter() - t0) * 1e3 / args.steps, 4)
        print(json.dumps({"transforms_only": res, "calls_each": args.steps + 1}))
        return
    tau = gen.tau_scalar()
    tau_int = gen.limbs_to_ints(tau[None, :])[0]

    log("setup: SRS 2^22 + prepared table")
    srs_pts = zk.srs_setup(tau, 1 << 22)
    srs = zk.SRS(srs_pts)
    evals_h = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n)
    evals = zk.to_device(evals_h)
    coeffs = torch.empty_like(evals)
    coset = torch.empty((4 * n, 8), dtype=torch.int32, device=dev)
    com = torch.empty((1, 16), dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    # one commit job per step: the library runs the coset transform on a
    # companion stream beside the MSM's latency-bound reduction
    def step():
        zk.commit_job(srs, evals, log_blowup=2, coeffs=coeffs, com=com, coset=coset)

    log("warmup", args.warmup)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # inside the timed region only the dominant kernel is bracketed by events
    # (every recorded region adds two timestamp events to its stream)
    zk.profile_read("msm.accumulate")
    zk.profile_only("msm.accumulate")
    zk.profile_enable(True)
    log("timed", args.steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    zk.profile_enable(False)
    zk.profile_only(None)
    ms_step = (t1 - t0) * 1e3 / args.steps
    acc_ms, acc_n = zk.profile_read("msm.accumulate")

    # the other regions, from a separate (untimed) profiled run of the step
    for reg in ("msm.sort", "msm.accumulate", "msm.reduce", "ntt.pass"):
        zk.profile_read(reg)
    prof_steps = min(args.steps, 10)
    zk.profile_enable(True)
    for _ in range(prof_steps):
        step()
    torch.cuda.synchronize()
    zk.profile_enable(False)
    region = {reg: zk.profile_read(reg) for reg in ("msm.sort", "msm.accumulate", "msm.reduce", "ntt.pass")}

    # algorithmic work of one accumulation launch
    coeffs_h = zk.to_host(coeffs)
    # the window width the SRS's table policy picks for this size
    c_bits = zk.srs_window_bits(srs, n)
    madds = nonzero_digits(coeffs_h, c_bits)
    acc_avg_s = acc_ms / max(acc_n, 1) / 1e3
    achieved = madds * MONT_PER_MADD * MADS_PER_MONT / acc_avg_s / 1e12
    traffic = ACCUMULATE_TRAFFIC["bytes"] if kernel_sources_hash() == ACCUMULATE_TRAFFIC["sources_sha256_16"] else None
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_MAD_TOPS, 3),
                "unit": "TOP/s", "frac": round(achieved / PEAK_MAD_TOPS, 4), "traffic": traffic,
                "kernel": "msm.accumulate", "launch_ms": round(acc_avg_s * 1e3, 4),
                "work_per_launch": "%d mixed additions x %d Fq products x %d word mads"
                                   % (madds, MONT_PER_MADD, MADS_PER_MONT)}

    extras = {"profiled_step_regions_ms": {
        "msm.sort": round(region["msm.sort"][0] / prof_steps, 4),
        "msm.accumulate": round(region["msm.accumulate"][0] / prof_steps, 4),
        "msm.reduce": round(region["msm.reduce"][0] / prof_steps, 4),
        "ntt.pass(all)": round(region["ntt.pass"][0] / prof_steps, 4),
        "ntt.pass launches/step": region["ntt.pass"][1] / prof_steps}}

    def timed(fn, reps=10):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    if not args.no_extras:
        log("per-op")
        t_intt = timed(lambda: zk.intt(evals, out=coeffs))
        t_ntt = timed(lambda: zk.ntt(coeffs, out=evals))
        zk.intt(evals, out=coeffs)
        torch.cuda.synchronize()
        zk.profile_enable(True)
        t_msm = timed(lambda: zk.msm_srs(srs, coeffs, out=com))
        zk.profile_enable(False)
        phases = {}
        for reg in ("msm.sort", "msm.accumulate", "msm.reduce"):
            ms_tot, cnt = zk.profile_read(reg)
            phases[reg] = round(ms_tot / max(cnt, 1), 4)
        t_coset = timed(lambda: zk.coset_ntt(coeffs, 2, out=coset))
        extras["ops_2^20"] = {
            "intt_ms": round(t_intt, 4), "ntt_ms": round(t_ntt, 4), "msm_ms": round(t_msm, 4),
            "coset_4x_ms": round(t_coset, 4), "msm_phases_ms_standalone": phases,
            "msm_points_per_s": n / (t_msm / 1e3), "ntt_elems_per_s": n / (t_ntt / 1e3),
            "intt_elems_per_s": n / (t_intt / 1e3), "coset_out_elems_per_s": 4 * n / (t_coset / 1e3),
            "ntt_hbm_frac_2pass": round(2 * 2 * 32 * n / (t_ntt / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        # both roofs of the transforms: algorithmic HBM bytes (two passes, each
        # reading and writing the data once) and algorithmic word products
        # ((N/2) log2 N butterflies, one Fr product of MADS_PER_MONT each)
        roofs = {}
        for name, t_ms, N_in, N_out in (("ntt_2^20", t_ntt, n, n), ("intt_2^20", t_intt, n, n),
                                        ("coset_2^20->2^22", t_coset, n, 4 * n)):
            lg = N_out.bit_length() - 1
            hbm_bytes = 32 * (N_in + N_out) + 2 * 32 * N_out
            mads = (N_out // 2) * lg * MADS_PER_MONT
            roofs[name] = {"ms": round(t_ms, 4),
                           "hbm_gbs": round(hbm_bytes / (t_ms / 1e3) / 1e9, 1),
                           "hbm_frac": round(hbm_bytes / (t_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                           "int_tops": round(mads / (t_ms / 1e3) / 1e12, 3),
                           "int_frac": round(mads / (t_ms / 1e3) / 1e12 / PEAK_MAD_TOPS, 4),
                           "bound": "alu"}
        extras["ntt_rooflines"] = roofs

        # per-step latency distribution of the commit job (each step bracketed
        # by its own events; separate from the timed throughput run)
        lat = []
        for _ in range(max(20, args.steps)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            step()
            e1.record()
            torch.cuda.synchronize()
            lat.append(e0.elapsed_time(e1))
        lat = np.array(lat)
        extras["step_latency_ms"] = {"median": round(float(np.median(lat)), 4),
                                     "p90": round(float(np.percentile(lat, 90)), 4),
                                     "min": round(float(lat.min()), 4), "reps": int(lat.size)}

        log("commit job with host transfers")
        # end to end with the host transfers: the 2^20 evaluations copied in
        # from pinned host memory, the commit job, the commitment copied back
        # (the coset evaluations stay resident for the next prover step);
        # reported beside the device-resident figure, never in its place
        ev_pin = torch.empty(evals.shape, dtype=torch.int32, pin_memory=True)
        ev_pin.copy_(evals.cpu())
        com_pin = torch.empty(com.shape, dtype=torch.int32, pin_memory=True)
        evals_in = torch.empty_like(evals)
        com_ref = com.clone()

        def e2e():
            evals_in.copy_(ev_pin, non_blocking=True)
            zk.commit_job(srs, evals_in, log_blowup=2, coeffs=coeffs, com=com, coset=coset)
            com_pin.copy_(com, non_blocking=True)

        t_e2e = timed(e2e, reps=20)
        same = bool(torch.equal(com_pin, com_ref.cpu()))
        t_h2d = timed(lambda: evals_in.copy_(ev_pin, non_blocking=True), reps=20)

        # a stream of such jobs: the next job's evaluations are copied in on a
        # copy stream (default priority) while the current job computes, into
        # one of two input buffers
        copy_s = torch.cuda.Stream()
        main_s = torch.cuda.current_stream()
        bufs = [evals_in, torch.empty_like(evals)]
        ready = [torch.cuda.Event(), torch.cuda.Event()]
        free = [torch.cuda.Event(), torch.cuda.Event()]
        coms = torch.empty((2, 16), dtype=torch.int32, pin_memory=True)

        def copy_in(k):
            with torch.cuda.stream(copy_s):
                if k >= 2:
                    copy_s.wait_event(free[k % 2])
                bufs[k % 2].copy_(ev_pin, non_blocking=True)
                ready[k % 2].record(copy_s)

        def pipelined(jobs):
            copy_in(0)
            for k in range(jobs):
                if k + 1 < jobs:
                    copy_in(k + 1)
                main_s.wait_event(ready[k % 2])
                zk.commit_job(srs, bufs[k % 2], log_blowup=2, coeffs=coeffs, com=com, coset=coset)
                free[k % 2].record(main_s)
                coms[k % 2].copy_(com[0], non_blocking=True)

        pipelined(4)
        torch.cuda.synchronize()
        jobs = 20
        t0p = time.perf_counter()
        pipelined(jobs)
        torch.cuda.synchronize()
        t_pipe = (time.perf_counter() - t0p) * 1e3 / jobs
        same = same and bool(torch.equal(coms[(jobs - 1) % 2], com_ref.cpu()[0]))
        extras["commit_job_with_host_transfers"] = {
            "ms": round(t_e2e, 4), "points_per_s": n / (t_e2e / 1e3),
            "pipelined_ms_per_job": round(t_pipe, 4), "pipelined_points_per_s": n / (t_pipe / 1e3),
            "h2d_ms": round(t_h2d, 4), "h2d_gbs": round(32 * n / (t_h2d / 1e3) / 1e9, 1),
            "device_resident_ms": round(ms_step, 4), "commitment_matches": same}
        del ev_pin, com_pin, evals_in, com_ref, bufs, coms

        log("kzg opening 2^20")
        # KZG opening of the committed polynomial at a point (quotient by
        # X - x, then its MSM), and a batched opening of 8 polynomials at one
        # point; the division scan is HBM-bound: 32 B per coefficient read per
        # polynomial plus 32 B per quotient coefficient written
        xw = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1, tag=11)[0]
        gw = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1, tag=12)[0]
        y1 = torch.empty((1, 8), dtype=torch.int32, device=dev)
        pi = torch.empty((1, 16), dtype=torch.int32, device=dev)
        zk.intt(evals, out=coeffs)
        torch.cuda.synchronize()
        kzg = {}
        for m_open in (1, 8):
            if m_open == 1:
                def run_open():
                    zk.kzg_open(srs, coeffs, xw, y=y1, proof=pi)
            else:
                polys = torch.stack([zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=20 + i))
                                     for i in range(m_open)])
                ys8 = torch.empty((m_open, 8), dtype=torch.int32, device=dev)

                def run_open():
                    zk.kzg_open_batch(srs, polys, xw, gw, ys=ys8, proof=pi)
            t_open = timed(run_open, reps=10)
            # each call bracketed by its own events: shows whether time above
            # the kernels' sum sits in every call or in a few
            per_call = []
            for _ in range(10):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                run_open()
                e1.record()
                torch.cuda.synchronize()
                per_call.append(e0.elapsed_time(e1))
            for reg in ("open.scan", "msm.sort", "msm.accumulate", "msm.reduce"):
                zk.profile_read(reg)
            zk.profile_enable(True)
            for _ in range(10):
                run_open()
            torch.cuda.synchronize()
            zk.profile_enable(False)
            scan_ms, scan_n = zk.profile_read("open.scan")
            scan_ms /= max(scan_n, 1)
            msm_ms = sum(zk.profile_read(reg)[0] for reg in ("msm.sort", "msm.accumulate", "msm.reduce")) / 10
            alg_bytes = 32 * m_open * n + 32 * (n - 1)
            products = (2 * m_open - 1) * n
            kzg["open_m%d" % m_open] = {
                "polys": m_open, "coeffs": n, "ms": round(t_open, 4), "openings_per_s": round(1e3 / t_open, 2),
                "call_ms_median": round(float(np.median(per_call)), 4),
                "call_ms_min": round(float(np.min(per_call)), 4), "call_ms_max": round(float(np.max(per_call)), 4),
                "scan_ms": round(scan_ms, 4), "msm_ms_profiled": round(msm_ms, 4),
                "scan_hbm_gbs": round(alg_bytes / (scan_ms / 1e3) / 1e9, 1),
                "scan_hbm_frac": round(alg_bytes / (scan_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                "scan_int_frac": round(products * MADS_PER_MONT / (scan_ms / 1e3) / 1e12 / PEAK_MAD_TOPS, 4),
                "scan_alg_bytes": alg_bytes, "scan_min_fr_products": products}
            if m_open > 1:
                del polys, ys8
        extras["kzg_open_2^20"] = kzg

        log("quotient 2^20")
        # Mul-block quotient t = (f h - g)/(X^n - 1) from three 2^20 witness
        # vectors (c = a*b), on cosets of 2x and 4x the domain, and its commitment
        qa_h = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=31)
        qb_h = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=32)
        qc_h = gen.ints_to_limbs([x * y % gen.FR_MODULUS for x, y in
                                  zip(gen.limbs_to_ints(qa_h), gen.limbs_to_ints(qb_h))]).reshape(n, 8)
        qa, qb, qc = zk.to_device(qa_h), zk.to_device(qb_h), zk.to_device(qc_h)
        qt = torch.empty_like(qa)
        quot = {}
        for lb in (1, 2):
            t_q = timed(lambda: zk.quotient_mul(srs, qa, qb, qc, log_blowup=lb, t=qt, com=com), reps=5)
            for reg in ("quot.pointwise", "ntt.pass", "msm.sort", "msm.accumulate", "msm.reduce"):
                zk.profile_read(reg)
            zk.profile_enable(True)
            for _ in range(5):
                zk.quotient_mul(srs, qa, qb, qc, log_blowup=lb, t=qt, com=com)
            torch.cuda.synchronize()
            zk.profile_enable(False)
            pw_ms = zk.profile_read("quot.pointwise")[0] / 5
            ntt_ms = zk.profile_read("ntt.pass")[0] / 5
            msm_q = sum(zk.profile_read(reg)[0] for reg in ("msm.sort", "msm.accumulate", "msm.reduce")) / 5
            big = n << lb
            quot["blowup_%d" % (1 << lb)] = {
                "ms": round(t_q, 4), "quotients_per_s": round(1e3 / t_q, 2),
                "transforms_ms": round(ntt_ms, 4), "msm_ms": round(msm_q, 4),
                "pointwise_ms": round(pw_ms, 4),
                "pointwise_hbm_frac": round(4 * 32 * big / (pw_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                "pointwise_int_frac": round(3 * big * MADS_PER_MONT / (pw_ms / 1e3) / 1e12 / PEAK_MAD_TOPS, 4)}
        extras["quotient_mul_2^20"] = quot
        del qa, qb, qc, qt

        log("poly-iop quotient 2^20")
        # the Poly-IOP quotient Q = R(f(x), f(omega x)) / (X^n - 1) on a 2x
        # coset for two constraints over 2^20-point witnesses: BooleanCheck
        # R = f (1 - f) (one witness) and a running product
        # R = z(omega x) - z(x) f(x) (two witnesses, one read omega-shifted)
        pseed = gen.CONFIG_SEEDS["commit"]
        Rm = gen.FR_MODULUS
        bits = gen.rng_for(pseed, 41).integers(0, 2, size=n).astype(np.uint32)
        bool_h = np.zeros((1, n, 8), dtype=np.uint32)
        bool_h[0, :, 0] = bits
        fv = [v or 1 for v in gen.limbs_to_ints(gen.uniform_fr(pseed, n, tag=42))]
        prod = 1
        for v in fv[:-1]:
            prod = prod * v % Rm
        fv[-1] = pow(prod, -1, Rm)
        zv = [gen.limbs_to_ints(gen.uniform_fr(pseed, 1, tag=43))[0] or 1]
        for i in range(n - 1):
            zv.append(zv[-1] * fv[i] % Rm)
        rp_h = np.stack([gen.ints_to_limbs(zv), gen.ints_to_limbs(fv)])
        cases = {"boolean_check": (zk.to_device(bool_h), [(1, [0]), (Rm - 1, [0, 0])]),
                 "running_product": (zk.to_device(rp_h), [(1, [2]), (Rm - 1, [0, 1])])}
        piop = {}
        for name, (ev_d, terms) in cases.items():
            qbuf = torch.empty((n, 8), dtype=torch.int32, device=dev)
            t_p = timed(lambda: zk.quotient_polyiop(srs, ev_d, terms, log_blowup=1, q=qbuf, com=com), reps=5)
            for reg in ("quot.pointwise", "ntt.pass", "msm.sort", "msm.accumulate", "msm.reduce"):
                zk.profile_read(reg)
            zk.profile_enable(True)
            for _ in range(5):
                zk.quotient_polyiop(srs, ev_d, terms, log_blowup=1, q=qbuf, com=com)
            torch.cuda.synchronize()
            zk.profile_enable(False)
            pw = zk.profile_read("quot.pointwise")[0] / 5
            nt = zk.profile_read("ntt.pass")[0] / 5
            ms_ = sum(zk.profile_read(reg)[0] for reg in ("msm.sort", "msm.accumulate", "msm.reduce")) / 5
            nwit = int(ev_d.shape[0])
            big = 2 * n
            piop[name] = {"witnesses": nwit, "ms": round(t_p, 4), "quotients_per_s": round(1e3 / t_p, 2),
                          "transforms_ms": round(nt, 4), "msm_ms": round(ms_, 4), "pointwise_ms": round(pw, 4),
                          "pointwise_hbm_frac": round((nwit + 1) * 32 * big / (pw / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
            del qbuf
        extras["polyiop_quotient_2^20"] = piop
        del cases, bool_h, rp_h, zv, fv

        log("lagrange commit 2^20")
        # commitments to a 2^20 vector of quantized activations as evaluations
        # on H: against the Lagrange-basis SRS (the vector's entries are the
        # MSM scalars, small) and through the monomial SRS (iNTT first, full
        # size coefficients)
        lag = zk.SRS(zk.srs_lagrange_setup(tau, 20))
        qv = zk.to_device(gen.quantized_fr(gen.CONFIG_SEEDS["quantized"], n, tag=3))
        qcoef = torch.empty_like(qv)
        t_lag = timed(lambda: zk.msm_srs(lag, qv, out=com), reps=10)

        def mono_commit():
            zk.intt(qv, out=qcoef)
            zk.msm_srs(srs, qcoef, out=com)
        t_mono = timed(mono_commit, reps=10)
        extras["lagrange_commit_2^20"] = {
            "vector": "quantized activations (int16, 30% zeros)", "lagrange_ms": round(t_lag, 4),
            "monomial_intt_msm_ms": round(t_mono, 4), "speedup": round(t_mono / t_lag, 3),
            "lagrange_points_per_s": n / (t_lag / 1e3)}
        lag.close()
        del qv, qcoef

        log("accumulation step")
        # one full fold of two accumulators: 64 commitments, a degree-2
        # relation (one correction term E_1), 2^20-element Fr parts and error
        # vectors; the challenge from the device transcript of the instances
        ka, la = 64, n
        Cs = [zk.srs_setup(gen.uniform_fr(gen.CONFIG_SEEDS["batched"], 1, tag=40 + i)[0], ka) for i in range(2)]
        Es = [zk.srs_setup(gen.uniform_fr(gen.CONFIG_SEEDS["batched"], 1, tag=50 + i)[0], 1) for i in range(3)]
        vs = [zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["batched"], la, tag=60 + i)) for i in range(5)]
        tr = torch.cat([Cs[0].flatten(), Es[0].flatten(), Cs[1].flatten(), Es[1].flatten(), Es[2].flatten()])
        gam = torch.empty((1, 8), dtype=torch.int32, device=dev)
        t_tr = timed(lambda: zk.transcript_challenge(tr, out=gam), reps=10)

        def acc_step():
            zk.transcript_challenge(tr, out=gam)
            zk.acc_fold(gam, Cs[0], Cs[1], Es[0], Es[1], Es[2], vs[0], vs[1], vs[2], vs[3],
                        vs[4].reshape(1, la, 8))
        t_acc = timed(acc_step, reps=5)
        for reg in ("acc.fold_g1", "acc.fr_rlc"):
            zk.profile_read(reg)
        zk.profile_enable(True)
        for _ in range(5):
            acc_step()
        torch.cuda.synchronize()
        zk.profile_enable(False)
        g1_ms = zk.profile_read("acc.fold_g1")[0] / 5
        rlc_ms, rlc_n = zk.profile_read("acc.fr_rlc")
        # fr_rlc launches per step: v'' (2 vectors in, 1 out) and e'' (3 in, 1 out)
        rlc_bytes = 32 * la * (3 + 4)
        extras["acc_fold_step"] = {
            "commitments": ka, "degree": 2, "fr_len": la, "ms": round(t_acc, 4), "transcript_ms": round(t_tr, 4),
            "g1_fold_ms": round(g1_ms, 4), "fr_rlc_ms": round(rlc_ms / 5, 4),
            "fr_rlc_hbm_frac": round(rlc_bytes / (rlc_ms / 5 / 1e3) / 1e9 / PEAK_HBM_GBS, 4)}
        del Cs, Es, vs, tr

        log("g2 msm")
        # G2 commitments (MulScalar / Mul / MatMul send G2 commitments beside
        # the G1 ones): MSMs over a prepared 2^20-point G2 SRS
        g2pts = zk.srs_g2_setup(tau, n)
        g2srs = zk.SRSG2(g2pts)
        g2out = torch.empty((1, 32), dtype=torch.int32, device=dev)
        g2 = {}
        for lg in (16, 20):
            sc2_h = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1 << lg, tag=70 + lg)
            sc2 = zk.to_device(sc2_h)
            t_g2 = timed(lambda: zk.msm_g2_srs(g2srs, sc2, out=g2out), reps=3)
            zk.profile_read("g2.accumulate")
            zk.profile_enable(True)
            for _ in range(3):
                zk.msm_g2_srs(g2srs, sc2, out=g2out)
            torch.cuda.synchronize()
            zk.profile_enable(False)
            acc_ms, acc_n = zk.profile_read("g2.accumulate")
            acc_ms /= max(acc_n, 1)
            # one mixed G2 addition per nonzero signed 8-bit digit: 8 Fq2
            # products (3 Fq products each) and 2 Fq2 squares (2 each)
            g2_madds = g2_nonzero_digits(sc2_h)
            g2_tops = g2_madds * G2_FQ_PER_MADD * MADS_PER_MONT / (acc_ms / 1e3) / 1e12
            g2["msm_2^%d" % lg] = {"ms": round(t_g2, 4), "points_per_s": (1 << lg) / (t_g2 / 1e3),
                                   "accumulate_ms": round(acc_ms, 4), "mixed_additions": g2_madds,
                                   "accumulate_int_frac": round(g2_tops / PEAK_MAD_TOPS, 4)}
            del sc2
        extras["g2_msm"] = g2
        g2srs.close()
        del g2pts

        log("quantized 2^22")
        N22 = 1 << 22
        q = zk.to_device(gen.quantized_fr(gen.CONFIG_SEEDS["quantized"], N22))
        u = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["quantized"], N22, tag=5))
        q8 = zk.to_device(gen.quantized_fr(gen.CONFIG_SEEDS["quantized"], N22, bits=8))
        t_q = timed(lambda: zk.msm_srs(srs, q, out=com), reps=5)
        t_q8 = timed(lambda: zk.msm_srs(srs, q8, out=com), reps=5)
        t_u = timed(lambda: zk.msm_srs(srs, u, out=com), reps=3)
        extras["quantized_2^22"] = {"msm_ms": round(t_q, 4), "points_per_s": N22 / (t_q / 1e3),
                                    "int8_msm_ms": round(t_q8, 4), "int8_points_per_s": N22 / (t_q8 / 1e3),
                                    "uniform_msm_ms": round(t_u, 4), "uniform_points_per_s": N22 / (t_u / 1e3),
                                    "speedup_vs_uniform": round(t_u / t_q, 3)}
        del q, q8, u

        log("batched 256")
        sizes = gen.log_uniform_sizes(gen.CONFIG_SEEDS["batched"], 256, 8, 18)
        off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
        sc = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["batched"], int(off[-1]), tag=1))
        outs = torch.empty((256, 16), dtype=torch.int32, device=dev)
        t_batch = timed(lambda: zk.msm_batch(srs, sc, off, out=outs), reps=3)
        views = [sc[int(off[b]):int(off[b + 1])] for b in range(256)]

        def per_call():
            for b in range(256):
                zk.msm_srs(srs, views[b], out=outs[b:b + 1])
        t_call = timed(per_call, reps=3)
        per_call_outs = zk.to_host(outs).copy()
        # the same 256 commitments as zk_msm_srs_noalloc calls (no allocation,
        # no host synchronisation): run directly, and captured once into a
        # HIP graph (torch.cuda.graph on one stream) and replayed
        cap = torch.empty((256, 16), dtype=torch.int32, device=dev)

        def noalloc_calls():
            for b in range(256):
                zk.msm_srs_noalloc(srs, views[b], cap[b:b + 1])
        t_noalloc = timed(noalloc_calls, reps=3)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            noalloc_calls()
        torch.cuda.synchronize()
        cap.fill_(0)
        t_graph = timed(graph.replay, reps=3)
        graph_same = bool(np.array_equal(zk.to_host(cap), per_call_outs))
        del graph
        tot = int(off[-1])
        extras["batched_256"] = {"total_points": tot, "batched_ms": round(t_batch, 3),
                                 "per_call_ms": round(t_call, 3), "batched_points_per_s": tot / (t_batch / 1e3),
                                 "per_call_points_per_s": tot / (t_call / 1e3),
                                 "batched_over_per_call": round(t_call / t_batch, 3),
                                 "noalloc_per_call_ms": round(t_noalloc, 3),
                                 "graph_replay_ms": round(t_graph, 3),
                                 "graph_points_per_s": tot / (t_graph / 1e3),
                                 "graph_matches_per_call": graph_same}
        log("fold 64")
        inst = outs[:64].contiguous().reshape(64, 1, 16)
        gam = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["batched"], 63, tag=2))
        fout = torch.empty((1, 16), dtype=torch.int32, device=dev)
        t_fold = timed(lambda: zk.fold(inst, gam, out=fout), reps=5)
        extras["fold_64"] = {"latency_ms": round(t_fold, 4)}
        del sc, outs

        # small commitments: the small-multiples table (up to 4096 points)
        # against the bucket run of the same commitment
        log("small commitments")
        small = {}
        sc = zk.to_device(gen.uniform_fr(gen.CONFIG_SEEDS["batched"], 1 << 14, tag=5))
        for lg in (8, 10, 12, 14):
            row = {}
            for label, tmax in (("small_multiples_ms", 4096), ("bucket_ms", 0)):
                zk.srs_set_tiny_max(srs, tmax)
                if tmax and (1 << lg) > tmax:
                    continue
                row[label] = round(timed(lambda: zk.msm_srs(srs, sc, n=1 << lg, out=com), reps=20), 4)
            small["2^%d" % lg] = row
        zk.srs_set_tiny_max(srs, 4096)
        extras["msm_small"] = small
        del sc

        log("serving")
        extras["serving"] = serving_runs(zk, srs, srs_pts, args.serve_jobs)
        # the largest transform, 2^28 points (three LDS passes), on a dense
        # input of canonical values (top word cut to 29 bits, below r's); run
        # last, so that no other timed section follows the release of its
        # 24 GB of buffers
        log("ntt 2^28")
        N28 = 1 << 28
        big = torch.randint(-2 ** 31, 2 ** 31 - 1, (N28, 8), dtype=torch.int32, device="cuda")
        big[:, 7] &= 0x1FFFFFFF
        big_out = torch.empty_like(big)
        t28 = timed(lambda: zk.ntt(big, out=big_out), reps=5)
        t28i = timed(lambda: zk.intt(big_out, out=big), reps=5)
        for name, t_ms in (("ntt_2^28", t28), ("intt_2^28", t28i)):
            hbm_bytes = 3 * 2 * 32 * N28
            mads = (N28 // 2) * 28 * MADS_PER_MONT
            extras["ntt_rooflines"][name] = {"ms": round(t_ms, 4), "passes": 3,
                                             "hbm_gbs": round(hbm_bytes / (t_ms / 1e3) / 1e9, 1),
                                             "hbm_frac": round(hbm_bytes / (t_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 4),
                                             "int_tops": round(mads / (t_ms / 1e3) / 1e12, 3),
                                             "int_frac": round(mads / (t_ms / 1e3) / 1e12 / PEAK_MAD_TOPS, 4),
                                             "bound": "alu"}
        del big, big_out
        torch.cuda.empty_cache()
        zk.release_cached_memory()

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, oracle_timings = cpu_baseline(tau_int)
        extras["oracle_timings"] = oracle_timings

    rec = {
        "metric": "MSM points/s (2^20) + NTT elems/s; batched vs per-call throughput, p99 latency",
        "value": n / (ms_step / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32 limbs (BN254 Fr/Fq, exact)",
        "data": "synthetic: seeded uniform Fr evaluations; SRS [tau^i]G from a seeded tau",
        "config": {"workload": "commit job: iNTT 2^20 -> MSM 2^20 vs SRS -> 4x coset NTT 2^20->2^22",
                   "n": n, "curve": "BN254", "msm_window_bits": c_bits},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    rec.update(extras)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
