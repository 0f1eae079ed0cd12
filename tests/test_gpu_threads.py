"""Library calls from several host threads at once, each thread on its own
stream: every result must equal the same call made alone.

ctypes releases the GIL around foreign calls, so the threads really do enter
the library together: the device-context set-up, the scratch-block cache
(blocks freed on one stream and taken on another wait on the block's last
use) and the per-thread error state are shared paths.  Streams are created at
the default priority.
"""
import threading

import pytest

from tests.gpu_helpers import log
from workloads import generators as gen

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_07031_amd import zk as m
    return m


def _step(zk, srs, ev):
    coeffs = zk.intt(ev)
    com = zk.msm_srs(srs, coeffs)
    coset = zk.coset_ntt(coeffs, 2)
    return coeffs, com, coset


def test_threads_on_separate_streams(zk):
    import torch
    logs = (12, 14, 16, 18)
    srs = zk.SRS(zk.srs_setup(gen.tau_scalar(), 1 << max(logs)))
    evs = [zk.to_device(gen.uniform_fr(7000 + L, 1 << L)) for L in logs]
    log("threads: references, one call at a time")
    refs = [_step(zk, srs, ev) for ev in evs]
    torch.cuda.synchronize()

    iters = 6
    errors = []
    results = [[None] * iters for _ in logs]
    barrier = threading.Barrier(len(logs))

    def work(t):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                barrier.wait()
                for k in range(iters):
                    results[t][k] = _step(zk, srs, evs[t])
            s.synchronize()
        except Exception as e:  # reported below, in the main thread
            errors.append((t, repr(e)))

    log("threads: %d threads x %d steps, sizes %s" % (len(logs), iters, [1 << L for L in logs]))
    th = [threading.Thread(target=work, args=(t,)) for t in range(len(logs))]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not any(x.is_alive() for x in th), "a thread did not finish"
    torch.cuda.synchronize()
    assert not errors, errors
    for t in range(len(logs)):
        for k in range(iters):
            for got, want in zip(results[t][k], refs[t]):
                assert torch.equal(got, want), (logs[t], k)
    srs.close()


def test_errors_stay_on_their_thread(zk):
    # a failing call on one thread leaves the other thread's last error alone
    msgs = {}
    barrier = threading.Barrier(2)

    def bad():
        barrier.wait()
        st = zk.lib.zk_ntt(None, None, 3, None)
        msgs["bad"] = (st, zk.lib.zk_last_error().decode())

    def good():
        barrier.wait()
        st = zk.lib.zk_set_validate(0)
        msgs["good"] = (st, zk.lib.zk_last_error().decode())

    th = [threading.Thread(target=bad), threading.Thread(target=good)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=30)
    assert msgs["bad"][0] == zk.ZK_EINVAL and "NULL" in msgs["bad"][1]
    assert msgs["good"][0] == zk.ZK_OK and "NULL" not in msgs["good"][1]


def test_validation_findings_stay_on_their_call(zk):
    # with validation on, two threads on their own streams enter the library
    # together many times: one always passes a non-canonical Fr input, the
    # other canonical inputs.  Each validated call has its own flag word, so
    # the bad call is refused every time and the good call never is.
    import numpy as np
    import torch
    n = 1 << 14
    good_h = gen.uniform_fr(7100, n)
    bad_h = good_h.copy()
    bad_h[n // 2] = gen.ints_to_limbs([gen.FR_MODULUS])[0]   # r itself
    good, bad = zk.to_device(good_h), zk.to_device(bad_h)
    ref = zk.to_host(zk.ntt(good))
    iters = 40
    status = {"good": [], "bad": []}
    errors = []
    barrier = threading.Barrier(2)

    def work(name, x):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                out = torch.empty_like(x)
                barrier.wait()
                for _ in range(iters):
                    st = zk.lib.zk_ntt(zk._ptr(x), zk._ptr(out), 14, zk._stream(x))
                    status[name].append(st)
                    if name == "good" and st == zk.ZK_OK:
                        s.synchronize()
                        if not np.array_equal(zk.to_host(out), ref):
                            errors.append("good output differs")
        except Exception as e:  # reported below, in the main thread
            errors.append(repr(e))

    log("threads: validated calls, one bad input thread and one good")
    zk.set_validate(True)
    try:
        th = [threading.Thread(target=work, args=("good", good)), threading.Thread(target=work, args=("bad", bad))]
        for x in th:
            x.start()
        for x in th:
            x.join(timeout=120)
        assert not any(x.is_alive() for x in th), "a thread did not finish"
    finally:
        zk.set_validate(False)
    torch.cuda.synchronize()
    assert not errors, errors
    assert status["good"] == [zk.ZK_OK] * iters
    assert status["bad"] == [zk.ZK_EINVAL] * iters
