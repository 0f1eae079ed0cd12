"""Element-by-element parity on the inputs and launch shapes that bench.py
times, against the oracle.

Each test rebuilds a benchmarked workload from the same seeded generators
and calls the library the way the benchmark does (same sizes, same prepared
SRS of 2^22 points, caller-owned outputs where the benchmark passes them),
then compares every output with the oracle:

* the 2^20 commit job: all 2^20 coefficients against the oracle's inverse
  FFT of the evaluations, the commitment against [f(tau)]_1, and all 2^22
  coset evaluations against the oracle's coset FFT; the forward transform of
  the benchmark's per-operation leg must give the evaluations back exactly;
* forward transforms of 2^20 and 2^22 uniform elements against the oracle's
  FFT, every output;
* the 256-MSM batch (log-uniform sizes 2^8..2^18, 11.95M points): all 256
  commitments against their closed forms, the batch against 256 single
  calls, and the fold of the first 64 commitments;
* the 2^22 MSMs over int16 and int8 activations and uniform scalars;
* the G2 MSMs at 2^16 and 2^20 over a 2^20-point G2 SRS;
* the accumulation step with 64 commitments and 2^20-element Fr parts.

The oracle's transforms are plain Python (about 30 s for 2^22 points on the
MI355X host), so this file takes a few minutes.
"""
import numpy as np
import pytest

from oracle import field, fold as ofold, g1, g2 as og2, msm as omsm, ntt as ontt, transcript as otr
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R
N20 = 1 << 20
N22 = 1 << 22


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
    log("srs setup 2^22 (the benchmark's SRS)")
    pts = zk.srs_setup(tau[0], N22)
    h = zk.SRS(pts)
    torch.cuda.synchronize()
    yield h
    h.close()
    del pts
    torch.cuda.empty_cache()


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def _assert_fr_equal(got_words, want_ints, what):
    """Every element of a device result (words) equals the oracle's list."""
    got = fr_from_host(got_words)
    assert len(got) == len(want_ints), what
    if got != want_ints:
        bad = [i for i, (a, b) in enumerate(zip(got, want_ints)) if a != b]
        raise AssertionError("%s: %d of %d elements differ, first at %d" % (what, len(bad), len(got), bad[0]))


def test_commit_job_benchmarked_elementwise(zk, tau, srs_big):
    import torch
    n = N20
    evals_h = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], n)
    evals = zk.to_device(evals_h)
    coeffs = torch.empty_like(evals)
    coset = torch.empty((4 * n, 8), dtype=torch.int32, device=evals.device)
    com = torch.empty((1, 16), dtype=torch.int32, device=evals.device)
    log("commit job 2^20 (benchmark step)")
    zk.commit_job(srs_big, evals, log_blowup=2, coeffs=coeffs, com=com, coset=coset)
    cf_h, com_h, cos_h = _host(zk, coeffs), _host(zk, com), _host(zk, coset)
    log("oracle: inverse FFT 2^20")
    ev = fr_from_host(evals_h)
    cf = ontt.ifft(ev)
    _assert_fr_equal(cf_h, cf, "coefficients")
    assert points_from_host(com_h)[0] == omsm.srs_msm_closed_form(tau[1], cf)
    log("oracle: coset FFT 2^20 -> 2^22")
    _assert_fr_equal(cos_h, ontt.coset_evals(cf, 2, 5), "coset evaluations")
    # the per-operation legs of the benchmark: the standalone coset call and
    # the forward transform of the coefficients (which must return the
    # evaluations, element by element)
    log("per-op legs: coset and forward NTT 2^20")
    assert np.array_equal(_host(zk, zk.coset_ntt(coeffs, 2, out=coset)), cos_h)
    back = torch.empty_like(evals)
    zk.ntt(coeffs, out=back)
    assert np.array_equal(_host(zk, back), evals_h)


@pytest.mark.parametrize("logn", [20, 22])
def test_ntt_forward_elementwise(zk, logn):
    n = 1 << logn
    a = gen.uniform_fr(300 + logn, n)
    log("ntt forward", logn)
    x = zk.to_device(a)
    A = zk.ntt(x)
    A_h = _host(zk, A)
    assert np.array_equal(_host(zk, zk.intt(A)), a)
    log("oracle: FFT", logn)
    _assert_fr_equal(A_h, ontt.fft(fr_from_host(a)), "forward transform 2^%d" % logn)


def test_batched_256_benchmarked(zk, tau, srs_big):
    import torch
    sizes = gen.log_uniform_sizes(gen.CONFIG_SEEDS["batched"], 256, 8, 18)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(off[-1])
    sc_h = gen.uniform_fr(gen.CONFIG_SEEDS["batched"], total, tag=1)
    sc = zk.to_device(sc_h)
    outs = torch.empty((256, 16), dtype=torch.int32, device=sc.device)
    log("batched 256 MSMs, %d points" % total)
    zk.msm_batch(srs_big, sc, off, out=outs)
    batched = _host(zk, outs).copy()
    log("per-call 256 MSMs")
    single = torch.empty_like(outs)
    for b in range(256):
        zk.msm_srs(srs_big, sc[int(off[b]):int(off[b + 1])], out=single[b:b + 1])
    assert np.array_equal(_host(zk, single), batched)
    log("oracle: 256 closed forms")
    sv = limbs_to_ints(sc_h)
    del sc_h
    want = [omsm.srs_msm_closed_form(tau[1], sv[int(off[b]):int(off[b + 1])]) for b in range(256)]
    got = points_from_host(batched)
    for b in range(256):
        assert got[b] == want[b], b
    # the fold of the first 64 commitments, as the benchmark runs it, against
    # the oracle's tree of pairwise folds over the oracle's commitments
    inst = outs[:64].contiguous().reshape(64, 1, 16)
    gam_h = gen.uniform_fr(gen.CONFIG_SEEDS["batched"], 63, tag=2)
    log("fold of 64 commitments")
    fout = zk.fold(inst, zk.to_device(gam_h))
    want_fold = ofold.tree_fold([[p] for p in want[:64]], fr_from_host(gam_h))
    assert points_from_host(_host(zk, fout)) == want_fold


@pytest.mark.parametrize("kind", ["int16", "int8", "uniform"])
def test_msm_2e22_benchmarked(zk, tau, srs_big, kind):
    seed = gen.CONFIG_SEEDS["quantized"]
    if kind == "uniform":
        s_h = gen.uniform_fr(seed, N22, tag=5)
        sv = fr_from_host(s_h)
    else:
        bits = 16 if kind == "int16" else 8
        s_h = gen.quantized_fr(seed, N22, bits=bits)
        sv = [int(v) % R for v in gen.quantized_values(seed, N22, bits=bits)]
    log("msm 2^22", kind)
    got = points_from_host(_host(zk, zk.msm_srs(srs_big, zk.to_device(s_h))))[0]
    assert got == omsm.srs_msm_closed_form(tau[1], sv)


def test_g2_msm_benchmarked(zk, tau):
    import torch
    log("g2 srs setup 2^20")
    pts = zk.srs_g2_setup(tau[0], N20)
    h = zk.SRSG2(pts)
    try:
        for lg in (16, 20):
            s_h = gen.uniform_fr(gen.CONFIG_SEEDS["commit"], 1 << lg, tag=70 + lg)
            log("g2 msm 2^%d" % lg)
            out = _host(zk, zk.msm_g2_srs(h, zk.to_device(s_h)))
            v = limbs_to_ints(out.reshape(-1, 8))
            assert og2.decode(tuple(v[:4])) == og2.srs_msm_closed_form(tau[1], fr_from_host(s_h)), lg
    finally:
        h.close()
        del pts
        torch.cuda.empty_cache()


def test_acc_fold_step_benchmarked(zk):
    # the benchmark's accumulation step: 64 commitments [t^j]_1 per
    # instance, E terms, 2^20-element Fr parts and error vectors, gamma from
    # the device transcript of the two instances
    import torch
    seed = gen.CONFIG_SEEDS["batched"]
    ka, la = 64, N20
    ts = [limbs_to_ints(gen.uniform_fr(seed, 1, tag=40 + i))[0] for i in range(2)]
    Cs = [zk.srs_setup(gen.uniform_fr(seed, 1, tag=40 + i)[0], ka) for i in range(2)]
    Es = [zk.srs_setup(gen.uniform_fr(seed, 1, tag=50 + i)[0], 1) for i in range(3)]
    vs_h = [gen.uniform_fr(seed, la, tag=60 + i) for i in range(5)]
    vs = [zk.to_device(v) for v in vs_h]
    tr = torch.cat([Cs[0].flatten(), Es[0].flatten(), Cs[1].flatten(), Es[1].flatten(), Es[2].flatten()])
    log("accumulation step: 64 commitments, 2^20 Fr parts")
    gam = zk.transcript_challenge(tr)
    C_out, E_out, v_out, e_out = zk.acc_fold(gam, Cs[0], Cs[1], Es[0], Es[1], Es[2], vs[0], vs[1], vs[2], vs[3],
                                             vs[4].reshape(1, la, 8))
    g = otr.challenge(_host(zk, tr).tobytes())
    assert fr_from_host(_host(zk, gam))[0] == g
    # commitments by their discrete logs: [t^j]_1; each E term is [t^0]_1 = G
    logs_c = [[pow(t, j, R) for j in range(ka)] for t in ts]
    want_c = [g1.gen_mul(x) for x in ofold.fold_fr(g, logs_c[0], logs_c[1])]
    assert points_from_host(_host(zk, C_out)) == want_c
    assert points_from_host(_host(zk, E_out))[0] == g1.gen_mul(ofold.fold_errors_fr(g, [1], [1], [[1]])[0])
    log("oracle: Fr parts 2^20")
    v = [fr_from_host(x) for x in vs_h]
    _assert_fr_equal(_host(zk, v_out), ofold.fold_fr(g, v[0], v[1]), "v''")
    _assert_fr_equal(_host(zk, e_out), ofold.fold_errors_fr(g, v[2], v[3], [v[4]]), "e''")
