"""GPU parity: the HIP path through the C-ABI against the CPU oracle, bit-exact.

Inputs are seeded (workloads); expected values come only from oracle/.
Sizes span one and two NTT passes and several MSM workgroups with ragged
tails; the largest cases use the full workload sizes and check sampled
outputs (Horner) or closed forms the oracle evaluates exactly.
"""
import numpy as np
import pytest

from oracle import field, fold as ofold, g1, msm as omsm, ntt as ontt, srs as osrs
from tests.gpu_helpers import fr_from_host, log, points_from_host, points_to_host
from workloads import generators as gen
from workloads import limbs_to_ints

pytestmark = pytest.mark.gpu
R, P = field.R, field.P


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
def srs_big(zk, tau):
    import torch
    log("srs setup 2^22")
    pts = zk.srs_setup(tau[0], 1 << 22)
    h = zk.SRS(pts)
    torch.cuda.synchronize()
    yield pts, h
    h.close()


def _dev(zk, arr):
    return zk.to_device(arr)


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


# ------------------------------------------------------------------ NTT

@pytest.mark.parametrize("logn", [0, 1, 2, 3, 5, 8, 12])
def test_ntt_small_exact(zk, logn):
    n = 1 << logn
    a = gen.uniform_fr(100 + logn, n)
    log("ntt small", logn)
    x = _dev(zk, a)
    fwd = fr_from_host(_host(zk, zk.ntt(x)))
    ref = ontt.dft(fr_from_host(a)) if logn <= 8 else ontt.fft(fr_from_host(a))
    assert fwd == ref
    inv = fr_from_host(_host(zk, zk.intt(x)))
    assert inv == (ontt.idft(fr_from_host(a)) if logn <= 8 else ontt.ifft(fr_from_host(a)))


@pytest.mark.parametrize("logn", [13, 14, 17])
def test_ntt_two_pass_exact(zk, logn):
    n = 1 << logn
    a = gen.uniform_fr(200 + logn, n)
    log("ntt two-pass", logn)
    x = _dev(zk, a)
    fwd = _host(zk, zk.ntt(x))
    av = fr_from_host(a)
    assert fr_from_host(fwd) == ontt.fft(av)
    inv = _host(zk, zk.intt(x))
    assert fr_from_host(inv) == ontt.ifft(av)


def test_ntt_tiny_workload_dft(zk):
    # 2^12 uniform Fr: NTT then iNTT of its output, against the O(n^2) definition
    n = 1 << 12
    a = gen.uniform_fr(gen.CONFIG_SEEDS["tiny"], n, tag=1)
    log("ntt 2^12 vs dft")
    x = _dev(zk, a)
    A = zk.ntt(x)
    back = zk.intt(A)
    Ah = fr_from_host(_host(zk, A))
    assert Ah == ontt.dft(fr_from_host(a))
    assert fr_from_host(_host(zk, back)) == fr_from_host(a)


@pytest.mark.parametrize("logn", [20, 22])
def test_ntt_large_roundtrip_and_samples(zk, logn):
    n = 1 << logn
    a = gen.uniform_fr(300 + logn, n)
    av = fr_from_host(a)
    log("ntt large", logn)
    x = _dev(zk, a)
    A = zk.ntt(x)
    back = zk.intt(A)
    Ah = fr_from_host(_host(zk, A))
    assert np.array_equal(_host(zk, back), a)
    # Sum protocol identity: sum_j A_j = n a_0
    assert sum(Ah) % R == n * av[0] % R
    w = ontt.root_of_unity(n)
    rng = np.random.default_rng(logn)
    for j in [0, 1, n - 1] + [int(v) for v in rng.integers(0, n, 3)]:
        assert Ah[j] == ontt.horner(av, pow(w, j, R)), j


def test_ntt_in_place(zk):
    for logn in (10, 16):
        n = 1 << logn
        a = gen.uniform_fr(400 + logn, n)
        x = _dev(zk, a)
        ref = _host(zk, zk.ntt(x))
        zk.ntt(x, out=x)
        assert np.array_equal(_host(zk, x), ref)
        zk.intt(x, out=x)
        assert np.array_equal(_host(zk, x), a)


@pytest.mark.parametrize("logn,logb", [(0, 2), (3, 2), (4, 2), (10, 2), (7, 6), (12, 2)])
def test_coset_exact(zk, logn, logb):
    n = 1 << logn
    c = gen.uniform_fr(500 + logn, n)
    log("coset", logn, logb)
    E = fr_from_host(_host(zk, zk.coset_ntt(_dev(zk, c), logb)))
    assert E == ontt.coset_evals(fr_from_host(c), logb, 5)


def test_coset_custom_shift(zk):
    n = 1 << 6
    c = gen.uniform_fr(600, n)
    g = 7
    sh = np.zeros(8, dtype=np.uint32)
    sh[0] = g
    E = fr_from_host(_host(zk, zk.coset_ntt(_dev(zk, c), 2, shift=sh)))
    assert E == ontt.coset_evals(fr_from_host(c), 2, g)
    # shift 1 and blowup 0 is the plain transform
    one = np.zeros(8, dtype=np.uint32)
    one[0] = 1
    E1 = fr_from_host(_host(zk, zk.coset_ntt(_dev(zk, c), 0, shift=one)))
    assert E1 == ontt.fft(fr_from_host(c))


def test_coset_large_samples(zk):
    # the commit workload's coset: 2^20 coefficients -> 2^22 evaluations
    n = 1 << 20
    c = gen.uniform_fr(700, n)
    cv = fr_from_host(c)
    log("coset 2^20 -> 2^22")
    E = _host(zk, zk.coset_ntt(_dev(zk, c), 2))
    Ev = fr_from_host(E)
    rng = np.random.default_rng(7)
    for j in [0, 1, 4 * n - 1] + [int(v) for v in rng.integers(0, 4 * n, 3)]:
        assert Ev[j] == ontt.coset_eval_at(cv, 2, j, 5), j


# ------------------------------------------------------------------ SRS / MSM

def test_srs_points_match_oracle(zk, tau, srs_big):
    pts, _ = srs_big
    rng = np.random.default_rng(11)
    idx = [0, 1, 2, (1 << 22) - 1] + [int(v) for v in rng.integers(0, 1 << 22, 6)]
    host = _host(zk, pts[idx])
    for i, pt in zip(idx, points_from_host(host)):
        assert pt == osrs.srs_point(tau[1], i), i


def test_msm_tiny_workload_vs_naive(zk, tau, srs_big):
    # 2^10 SRS points x uniform scalars, against the naive sum over the
    # oracle's own SRS and against the closed form
    n = 1 << 10
    s = gen.uniform_fr(gen.CONFIG_SEEDS["tiny"], n)
    sv = fr_from_host(s)
    pts, h = srs_big
    log("msm 2^10 generic + srs")
    got_generic = points_from_host(_host(zk, zk.msm(pts[:n].contiguous(), _dev(zk, s))))[0]
    got_srs = points_from_host(_host(zk, zk.msm_srs(h, _dev(zk, s))))[0]
    expect = omsm.naive_msm(osrs.srs(tau[1], n), sv)
    assert expect == omsm.srs_msm_closed_form(tau[1], sv)
    assert got_generic == expect
    assert got_srs == expect


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 255, 4097, 16383, 16384, 65537])
def test_msm_sizes_closed_form(zk, tau, srs_big, n):
    s = gen.uniform_fr(800 + n, n)
    sv = fr_from_host(s)
    pts, h = srs_big
    log("msm n", n)
    expect = omsm.srs_msm_closed_form(tau[1], sv)
    assert points_from_host(_host(zk, zk.msm_srs(h, _dev(zk, s))))[0] == expect
    if n <= 4097:
        assert points_from_host(_host(zk, zk.msm(pts[:n].contiguous(), _dev(zk, s))))[0] == expect


def test_msm_large_commit_workload(zk, tau, srs_big):
    n = 1 << 20
    s = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=7)
    _, h = srs_big
    log("msm 2^20 srs")
    got = points_from_host(_host(zk, zk.msm_srs(h, _dev(zk, s))))[0]
    assert got == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))


@pytest.mark.parametrize("n", [(1 << 21) + 12345, 1 << 22])
def test_msm_large_window_table(zk, tau, srs_big, n):
    # from 2^21 points the commitment runs on the 20-bit-window table
    # (13 windows, 2^19 shared buckets): uniform scalars, ragged and full size
    s = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=11)
    _, h = srs_big
    log("msm large-window table", n)
    got = points_from_host(_host(zk, zk.msm_srs(h, _dev(zk, s))))[0]
    assert got == omsm.srs_msm_closed_form(tau[1], fr_from_host(s))


def test_msm_quantized_full_size(zk, tau, srs_big):
    n = 1 << 22
    q = gen.quantized_fr(gen.CONFIG_SEEDS["quantized"], n)
    x = gen.quantized_values(gen.CONFIG_SEEDS["quantized"], n)
    _, h = srs_big
    log("msm 2^22 quantized")
    got = points_from_host(_host(zk, zk.msm_srs(h, _dev(zk, q))))[0]
    assert got == omsm.srs_msm_closed_form(tau[1], [int(v) % R for v in x])


def test_msm_edge_scalars_and_bases(zk, tau, srs_big):
    pts, h = srs_big
    t = tau[1]
    n = 40
    base = pts[:n].contiguous()
    cases = {
        "zeros": [0] * n,
        "ones": [1] * n,
        "r-1": [R - 1] * n,
        "powers": [1 << (i * 6 % 254) for i in range(n)],
        "half": [(R - 1) // 2 + (i % 3) for i in range(n)],
        "mixed": [0, 1, R - 1, 2, R - 2, 12345] * 6 + [5, 6, 7, 8],
    }
    for name, sv in cases.items():
        s = gen.ints_to_limbs([v % R for v in sv])
        log("msm edge", name)
        expect = omsm.srs_msm_closed_form(t, sv)
        assert points_from_host(_host(zk, zk.msm(base, _dev(zk, s))))[0] == expect, name
        assert points_from_host(_host(zk, zk.msm_srs(h, _dev(zk, s), n=n)))[0] == expect, name
    # duplicate bases (P + P inside a bucket), P and -P, infinity bases
    host = _host(zk, base).copy()
    dup = host.copy()
    dup[1] = dup[0]
    dup[2] = dup[0]
    negy = P - limbs_to_ints(host[3, 8:16][None, :])[0]
    dup[4, :8] = host[3, :8]
    dup[4, 8:] = gen.ints_to_limbs([negy])[0]
    dup[5] = 0
    logs = [pow(t, i, R) for i in range(n)]
    logs[1] = logs[2] = logs[0]
    logs[4] = (R - logs[3]) % R
    logs[5] = 0
    for sv in ([7] * n, [3, 3, 3, 9, 9, 4] + [1] * (n - 6)):
        s = gen.ints_to_limbs(sv)
        expect = omsm.gen_msm_closed_form(logs, sv)
        got = points_from_host(_host(zk, zk.msm(_dev(zk, dup), _dev(zk, s))))[0]
        assert got == expect


@pytest.mark.parametrize("logn", [0, 10, 16, 20])
def test_commit_step_overlapped(zk, tau, srs_big, logn):
    # the commit step with the coset transform on a second stream, released by
    # the event that zk_msm_srs_ex records after bucket accumulation: the
    # commitment and the coset evaluations must equal the serial calls and the
    # oracle (small table below 2^15 points, SRS table above)
    import torch
    n = 1 << logn
    _, h = srs_big
    ev = _dev(zk, gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=30 + logn))
    side = torch.cuda.Stream()
    main_s = torch.cuda.current_stream()
    acc_done = torch.cuda.Event()
    log("commit step overlapped", logn)
    coeffs = zk.intt(ev)
    com = zk.msm_srs_overlap(h, coeffs, acc_done)
    side.wait_event(acc_done)
    with torch.cuda.stream(side):
        coset = zk.coset_ntt(coeffs, 2)
    main_s.wait_stream(side)
    com_h, coset_h = _host(zk, com), _host(zk, coset)
    assert np.array_equal(com_h, _host(zk, zk.msm_srs(h, coeffs)))
    assert np.array_equal(coset_h, _host(zk, zk.coset_ntt(coeffs, 2)))
    cv = fr_from_host(_host(zk, coeffs))
    assert points_from_host(com_h)[0] == omsm.srs_msm_closed_form(tau[1], cv)
    Ev = fr_from_host(coset_h)
    for j in sorted({0, 1, 4 * n - 1, (7 * n) // 3}):
        assert Ev[j] == ontt.coset_eval_at(cv, 2, j, 5), j


@pytest.mark.parametrize("logn,logb,custom", [(0, 2, False), (3, 0, False), (12, 2, False), (13, 2, True),
                                               (16, 2, False), (20, 2, False)])
def test_commit_job(zk, tau, srs_big, logn, logb, custom):
    # the fused commit job (iNTT, commitment, coset evaluations overlapped on
    # a companion stream) equals the three separate calls and the oracle
    n = 1 << logn
    _, h = srs_big
    ev = _dev(zk, gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n, tag=50 + logn))
    shift = None
    g = 5
    if custom:
        g = 7
        shift = np.zeros(8, dtype=np.uint32)
        shift[0] = g
    log("commit job", logn, logb, custom)
    coeffs, com, coset = zk.commit_job(h, ev, log_blowup=logb, shift=shift)
    cf_ref = zk.intt(ev)
    com_h, cos_h, cf_h = _host(zk, com), _host(zk, coset), _host(zk, coeffs)
    assert np.array_equal(cf_h, _host(zk, cf_ref))
    assert np.array_equal(com_h, _host(zk, zk.msm_srs(h, cf_ref)))
    assert np.array_equal(cos_h, _host(zk, zk.coset_ntt(cf_ref, logb, shift=shift)))
    cv = fr_from_host(cf_h)
    assert points_from_host(com_h)[0] == omsm.srs_msm_closed_form(tau[1], cv)
    # the commitment straight from the evaluations: [f(tau)]_1 with f(tau) in
    # barycentric form, independent of any inverse transform (about 25 s of
    # oracle time at 2^20, the benchmarked size)
    log("commit job", logn, "barycentric")
    assert points_from_host(com_h)[0] == g1.gen_mul(ontt.barycentric_eval(fr_from_host(_host(zk, ev)), tau[1]))
    Ev = fr_from_host(cos_h)
    m = n << logb
    for j in sorted({0, 1, m - 1, (7 * m) // 3 % m}):
        assert Ev[j] == ontt.coset_eval_at(cv, logb, j, g), j
    # in-place: evals and coeffs alias
    ev2 = ev.clone()
    zk.commit_job(h, ev2, log_blowup=logb, shift=shift, coeffs=ev2)
    assert np.array_equal(_host(zk, ev2), cf_h)


def test_msm_empty(zk, srs_big):
    import torch
    pts, h = srs_big
    s = torch.zeros((1, 8), dtype=torch.int32, device="cuda")
    assert points_from_host(_host(zk, zk.msm(pts[:1].contiguous(), s, n=0)))[0] is None
    assert points_from_host(_host(zk, zk.msm_srs(h, s, n=0)))[0] is None
    ev = torch.cuda.Event()
    assert points_from_host(_host(zk, zk.msm_srs_overlap(h, s, ev, n=0)))[0] is None
    assert ev.query()


def test_msm_batch_uneven(zk, tau, srs_big):
    _, h = srs_big
    sizes = [1, 300, 5000, 20000, 70000, 2]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    s = gen.uniform_fr(900, int(off[-1]))
    sv = fr_from_host(s)
    log("msm batch", sizes)
    out = points_from_host(_host(zk, zk.msm_batch(h, _dev(zk, s), off)))
    for b in range(len(sizes)):
        assert out[b] == omsm.srs_msm_closed_form(tau[1], sv[off[b]:off[b + 1]]), b


def test_msm_batch_many_segments(zk, tau, srs_big):
    # more MSMs than one kernel-argument block of segment offsets, with empty
    # and one-point MSMs among them
    _, h = srs_big
    rng = np.random.default_rng(5)
    sizes = [int(v) for v in rng.integers(0, 400, 300)]
    sizes[3] = 0
    sizes[129] = 0
    sizes[130] = 1
    sizes[-1] = 40000
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    s = gen.uniform_fr(901, int(off[-1]))
    sv = fr_from_host(s)
    log("msm batch", len(sizes), "segments")
    out = points_from_host(_host(zk, zk.msm_batch(h, _dev(zk, s), off)))
    for b in range(len(sizes)):
        assert out[b] == omsm.srs_msm_closed_form(tau[1], sv[off[b]:off[b + 1]]), b


def test_msm_batch_quantized_segments(zk, tau, srs_big):
    _, h = srs_big
    sizes = [1 << 16, 1000, 1 << 18]
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    x = gen.quantized_values(77, int(off[-1]))
    q = gen.quantized_fr(77, int(off[-1]))
    out = points_from_host(_host(zk, zk.msm_batch(h, _dev(zk, q), off)))
    xv = [int(v) % R for v in x]
    for b in range(len(sizes)):
        assert out[b] == omsm.srs_msm_closed_form(tau[1], xv[off[b]:off[b + 1]]), b


# ------------------------------------------------------------------ fold

# per-term path up to 1024 instances and 2^16 points (one block of 64 terms,
# several, and the limit), Pippenger beyond either bound
@pytest.mark.parametrize("m,k", [(1, 1), (2, 3), (3, 1), (5, 2), (64, 1), (65, 2), (1024, 1), (1025, 1),
                                 (300, 250)])
def test_fold_matches_tree(zk, tau, srs_big, m, k):
    pts, _ = srs_big
    t = tau[1]
    rng = np.random.default_rng(m * 10 + k)
    idx = [int(v) for v in rng.integers(0, 1 << 22, m * k)]
    inst = pts[idx].contiguous().reshape(m, k, 16)
    gam = gen.uniform_fr(1000 + m, max(m - 1, 1))[: m - 1]
    gv = fr_from_host(gam) if m > 1 else []
    log("fold", m, k)
    out = points_from_host(_host(zk, zk.fold(inst, _dev(zk, gam) if m > 1 else None)))
    sig = ofold.flat_coefficients(m, gv)
    for j in range(k):
        logsum = sum(sig[i] * pow(t, idx[i * k + j], R) for i in range(m)) % R
        assert out[j] == g1.gen_mul(logsum), j
    if m <= 5:
        inst_pts = [[osrs.srs_point(t, idx[i * k + j]) for j in range(k)] for i in range(m)]
        assert out == ofold.tree_fold(inst_pts, gv)


def test_fold_with_points_at_infinity(zk, tau, srs_big):
    pts, _ = srs_big
    t = tau[1]
    m, k = 6, 2
    idx = [5 + 3 * i for i in range(m * k)]
    host = zk.to_host(pts[idx].contiguous()).reshape(m * k, 16).copy()
    zero = {1, 4, 11}  # (0, 0) entries
    host[list(zero)] = 0
    inst = zk.to_device(host).reshape(m, k, 16)
    gam = gen.uniform_fr(1077, m - 1)
    log("fold with infinity entries")
    out = points_from_host(_host(zk, zk.fold(inst, _dev(zk, gam))))
    sig = ofold.flat_coefficients(m, fr_from_host(gam))
    for j in range(k):
        logsum = sum(sig[i] * pow(t, idx[i * k + j], R) for i in range(m) if i * k + j not in zero) % R
        assert out[j] == g1.gen_mul(logsum), j


# ------------------------------------------------------------------ input validation

def test_validation_rejects_out_of_range_inputs(zk, tau, srs_big):
    # zk_set_validate: non-canonical scalars and off-curve bases are refused
    # with ZK_EINVAL before any work; valid inputs give unchanged results
    pts, h = srs_big
    n = 64
    s = gen.uniform_fr(gen.CONFIG_SEEDS["tiny"], n, tag=90)
    base = pts[:n].contiguous()
    ref = _host(zk, zk.msm(base, _dev(zk, s)))
    bad_s = s.copy()
    bad_s[5] = gen.ints_to_limbs([R])[0]            # r itself: not canonical
    host_pts = _host(zk, base).copy()
    bad_p = host_pts.copy()
    bad_p[7, 8] ^= 1                                 # y changed: off the curve
    zk.set_validate(True)
    try:
        assert np.array_equal(_host(zk, zk.msm(base, _dev(zk, s))), ref)
        assert np.array_equal(_host(zk, zk.msm_srs(h, _dev(zk, s))), _host(zk, zk.msm_srs(h, _dev(zk, s))))
        for call in (lambda: zk.msm(base, _dev(zk, bad_s)),
                     lambda: zk.msm(_dev(zk, bad_p), _dev(zk, s)),
                     lambda: zk.msm_srs(h, _dev(zk, bad_s)),
                     lambda: zk.ntt(_dev(zk, bad_s)),
                     lambda: zk.intt(_dev(zk, bad_s)),
                     lambda: zk.coset_ntt(_dev(zk, bad_s), 2),
                     lambda: zk.commit_job(h, _dev(zk, bad_s)),
                     lambda: zk.msm_batch(h, _dev(zk, bad_s), np.array([0, 10, n], dtype=np.uint64)),
                     lambda: zk.SRS(_dev(zk, bad_p))):
            with pytest.raises(zk.ZkError) as ei:
                call()
            assert ei.value.code == zk.ZK_EINVAL
        # infinity (0, 0) is a valid base
        inf_p = host_pts.copy()
        inf_p[3] = 0
        zk.msm(_dev(zk, inf_p), _dev(zk, s))
    finally:
        zk.set_validate(False)
    # off again: the same non-canonical input is not checked
    zk.ntt(_dev(zk, bad_s))


# ------------------------------------------------------------------ serving

def test_serving_mix_equals_alone(zk, tau, srs_big):
    # commit-and-fold jobs admitted while others run overlap on the device;
    # every result (commitment, coset evaluations, folded accumulator) must be
    # bit-identical to the same job run alone, including a 2^22 job
    from paper_2507_07031_amd.serve import GpuExecutor, Job, serve
    pts, h = srs_big
    pool = _dev(zk, gen.uniform_fr(gen.CONFIG_SEEDS["serving"], 1 << 23, tag=1))
    acc_pool = pts[:4096].contiguous()
    sizes = [1000, 1 << 12, 70000, 1 << 18, 333, 1 << 16, 5000, 1 << 20, 1, 2, (1 << 21) + 77, 3000]
    rng = np.random.default_rng(3)
    offs = [int(rng.integers(0, (1 << 23) - (1 << 22))) for _ in sizes]
    accs = [int(rng.integers(0, 4096)) for _ in sizes]

    def mk():
        return [Job(i, n, 1e-4 * i, o, a) for i, (n, o, a) in enumerate(zip(sizes, offs, accs))]

    log("serving mix")
    ex = GpuExecutor(zk, h, pool, slots=4, acc_pool=acc_pool, budget=64 << 30, keep_results=True)
    fin, rej, _ = serve(mk(), ex, 64 << 30, 4)
    assert not rej and len(fin) == len(sizes)
    assert all(j.error is None for j in fin)
    mixed = {j.jid: j.result for j in fin}
    assert max(j.start for j in fin) < max(j.finish for j in fin)
    zk.set_scratch_budget(0)
    for job in mk():
        ex1 = GpuExecutor(zk, h, pool, slots=1, acc_pool=acc_pool, keep_results=True)
        f1, _, _ = serve([job], ex1, 64 << 30, 1)
        for a, b in zip(f1[0].result, mixed[job.jid]):
            assert np.array_equal(a, b), job.jid
    # the smallest padded job against the oracle: commitment straight from the
    # evaluations (barycentric), coset samples from the coefficients, and the
    # fold gamma * acc + com with gamma the transcript of (acc, com)
    from oracle import transcript as otr
    j = 0
    N = 1024
    ev = fr_from_host(_host(zk, pool[offs[j]:offs[j] + sizes[j]])) + [0] * (N - sizes[j])
    com = points_from_host(mixed[j][0])[0]
    assert com == g1.gen_mul(ontt.barycentric_eval(ev, tau[1]))
    coeffs = ontt.ifft(ev)
    cos = fr_from_host(mixed[j][1])
    for k in (0, 5, 4 * N - 1):
        assert cos[k] == ontt.coset_eval_at(coeffs, 2, k, 5)
    acc = osrs.srs_point(tau[1], accs[j])
    gamma = otr.challenge(np.concatenate([points_to_host([acc]), points_to_host([com])]).tobytes())
    assert points_from_host(mixed[j][2])[0] == ofold.tree_fold([[acc], [com]], [gamma])[0]
