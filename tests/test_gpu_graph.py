"""HIP graph capture of batched commitments: the 256 uneven MSMs of the
batched workload (log-uniform 2^8..2^18 points over one prepared SRS), each
a zk_msm_srs_noalloc call, captured once into a graph on one stream and
replayed.  Every replay must equal the direct per-call results bit for bit;
the replays are separated by the program's own eager library work and
synchronisations, and one replay runs after the scalars were overwritten in
place (the graph computes on the live buffers).  The first outputs are also
checked against the oracle's closed form.
"""
import numpy as np
import pytest

from oracle import msm as omsm
from tests.gpu_helpers import fr_from_host, log, points_from_host
from workloads import generators as gen
from workloads import limbs_to_ints

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def zk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_07031_amd import zk as m
    return m


def _host(zk, t):
    import torch
    torch.cuda.synchronize()
    return zk.to_host(t)


def test_captured_batch_replays_match_direct_calls(zk):
    import torch
    tau = gen.tau_scalar()
    t = limbs_to_ints(tau[None, :])[0]
    log("graph: srs setup 2^18")
    srs = zk.SRS(zk.srs_setup(tau, 1 << 18))
    sizes = gen.log_uniform_sizes(gen.CONFIG_SEEDS["batched"], 256, 8, 18)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint64)
    total = int(off[-1])
    sc_a = gen.uniform_fr(gen.CONFIG_SEEDS["batched"], total, tag=1)
    sc_b = gen.uniform_fr(gen.CONFIG_SEEDS["batched"], total, tag=3)
    sc = zk.to_device(sc_a)
    views = [sc[int(off[b]):int(off[b + 1])] for b in range(256)]

    def direct():
        ref = torch.empty((256, 16), dtype=torch.int32, device="cuda")
        for b in range(256):
            zk.msm_srs(srs, views[b], out=ref[b:b + 1])
        return _host(zk, ref).copy()

    log("graph: direct per-call references")
    ref_a = direct()
    outs = torch.zeros((256, 16), dtype=torch.int32, device="cuda")
    # the first call of the process sets kernel attributes: not during capture
    zk.msm_srs_noalloc(srs, views[0], outs[0:1])
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    log("graph: capture 256 no-alloc MSMs")
    with torch.cuda.graph(g):
        for b in range(256):
            zk.msm_srs_noalloc(srs, views[b], outs[b:b + 1])
    torch.cuda.synchronize()
    other = zk.to_device(gen.uniform_fr(77, 1 << 12))
    for rep in range(3):
        outs.fill_(0)
        log("graph: replay", rep)
        g.replay()
        got = _host(zk, outs).copy()
        assert np.array_equal(got, ref_a), rep
        # eager work between replays
        zk.msm_srs(srs, other)
        zk.ntt(other)
        torch.cuda.synchronize()
    # new scalars in the same buffer: the replay computes on them
    sc.copy_(zk.to_device(sc_b))
    ref_b = direct()
    outs.fill_(0)
    g.replay()
    assert np.array_equal(_host(zk, outs), ref_b)
    assert not np.array_equal(ref_a, ref_b)
    for b in (0, 1, 255):
        seg = fr_from_host(sc_b[int(off[b]):int(off[b + 1])])
        assert points_from_host(ref_b[b:b + 1])[0] == omsm.srs_msm_closed_form(t, seg), b
    del g
    srs.close()
