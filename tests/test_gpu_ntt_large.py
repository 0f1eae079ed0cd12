"""GPU parity of transforms above 2^24 points (three LDS passes), up to the
largest radix-2 domain of Fr, 2^28 (its 2-adicity).

Inputs are run-structured: a few hundred constant runs of random lengths with
random values, overwritten at scattered single positions (index 0 and N - 1
among them) by other random values.  Every input element is read, and every
output is a sum over all runs and points, so sampled outputs are checked
bit-exact against the oracle's geometric-sum form of the transform's
definition.  The samples cover both ends, N/2 and the boundaries of the three
factors.  A dense uniform input is checked by the inverse round trip, in place
and out of place.
"""
import numpy as np
import pytest

from oracle import field, ntt as ontt
from tests.gpu_helpers import fr_from_host, log
from workloads import generators as gen

pytestmark = pytest.mark.gpu
R = field.R


@pytest.fixture(scope="module")
def zk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2507_07031_amd import zk as m
    yield m
    torch.cuda.empty_cache()
    m.release_cached_memory()


def _runs_input(seed, n, nruns=200, npts=40):
    """Device tensor of n elements made of constant runs plus single values,
    and the (runs, points) description the oracle takes."""
    import torch
    rng = gen.rng_for(seed, tag=3)
    cuts = np.sort(rng.choice(n - 1, nruns - 1, replace=False).astype(np.int64) + 1)
    edges = np.concatenate([[0], cuts, [n]]).astype(np.int64)
    lengths = np.diff(edges)
    vals = gen.uniform_fr(seed, nruns + npts, tag=4)
    vals[nruns // 2] = 0  # one run of zeros
    pos = rng.choice(n - 2, npts - 2, replace=False).astype(np.int64) + 1
    pos = np.concatenate([[0, n - 1], pos]).astype(np.int64)
    dev_vals = torch.from_numpy(vals[:nruns].view(np.int32)).cuda()
    dev_cuts = torch.from_numpy(cuts).cuda()
    x = torch.empty((n, 8), dtype=torch.int32, device="cuda")
    step = 1 << 24  # torch's own kernels take at most this many rows at once here
    for c0 in range(0, n, step):
        rows = torch.arange(c0, min(n, c0 + step), dtype=torch.int64, device="cuda")
        x[c0:c0 + rows.numel()] = dev_vals.index_select(0, torch.bucketize(rows, dev_cuts, right=True))
    x[torch.from_numpy(pos).cuda()] = torch.from_numpy(vals[nruns:].view(np.int32)).cuda()
    ints = fr_from_host(vals)
    runs = [(int(edges[t]), int(lengths[t]), ints[t]) for t in range(nruns)]
    points = {int(p): ints[nruns + t] for t, p in enumerate(pos)}
    assert x.shape == (n, 8) and x.is_contiguous()
    return x, runs, points


def _samples(L, seed):
    N = 1 << L
    mA = (L + 2) // 3
    mB = L - mA
    p2 = (mB + 1) // 2
    ks = {0, 1, 2, N // 2, N - 1, N - 2}
    for b in (mA, mA + p2):
        ks |= {(1 << b) - 1, 1 << b, (1 << b) + 1}
    rng = gen.rng_for(seed, tag=5)
    ks |= {int(v) for v in rng.integers(0, N, 16)}
    return sorted(ks)


def _gather(t, ks):
    import torch
    idx = torch.tensor(ks, dtype=torch.int64, device=t.device)
    torch.cuda.synchronize()
    return fr_from_host(t.index_select(0, idx).cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("L", [25, 26, 27, 28])
def test_ntt_three_pass_forward(zk, L):
    log("ntt three-pass forward 2^%d" % L)
    x, runs, points = _runs_input(4000 + L, 1 << L)
    out = zk.ntt(x)
    ks = _samples(L, L)
    got = _gather(out, ks)
    for k, v in zip(ks, got):
        assert v == ontt.ntt_runs_at(runs, points, L, k), (L, k)
    del x, out


@pytest.mark.parametrize("L", [25, 28])
def test_intt_three_pass(zk, L):
    log("intt three-pass 2^%d" % L)
    x, runs, points = _runs_input(4100 + L, 1 << L)
    out = zk.intt(x)
    ks = _samples(L, 100 + L)
    got = _gather(out, ks)
    for k, v in zip(ks, got):
        assert v == ontt.ntt_runs_at(runs, points, L, k, inverse=True), (L, k)
    del x, out


@pytest.mark.parametrize("log_n,lb", [(23, 2), (22, 3), (26, 2)])
def test_coset_ntt_three_pass(zk, log_n, lb):
    L = log_n + lb
    log("coset ntt three-pass 2^%d x %d" % (log_n, 1 << lb))
    x, runs, points = _runs_input(4200 + L, 1 << log_n)
    out = zk.coset_ntt(x, lb)
    assert out.shape[0] == 1 << L
    ks = _samples(L, 200 + L)
    got = _gather(out, ks)
    for k, v in zip(ks, got):
        assert v == ontt.ntt_runs_at(runs, points, L, k, shift=field.GENERATOR_FR), (log_n, lb, k)
    del x, out


def _dense_input(seed, L):
    """2^L distinct elements below r: a seeded uniform block of 2^16 tiled,
    the low word of element i set to i and the top word cut to 29 bits (every
    value with a top word below r's, 0x30644e72, is below r)."""
    import torch
    blk = torch.from_numpy(gen.uniform_fr(seed, 1 << 16).view(np.int32)).cuda()
    x = blk.repeat(1 << (L - 16), 1)
    x[:, 0] = torch.arange(1 << L, dtype=torch.int64, device="cuda").to(torch.int32)
    x[:, 7] &= 0x1FFFFFFF
    return x.contiguous()


def _sum_mod_r(t):
    # sum of the 256-bit values (rows of eight 32-bit limbs) reduced mod r:
    # limb columns summed in 64 bits (2^25 * 2^32 < 2^63), then combined
    import torch
    cols = (t.to(torch.int64) & 0xFFFFFFFF).sum(dim=0).cpu().tolist()
    return sum(int(c) << (32 * j) for j, c in enumerate(cols)) % R


def test_ntt_three_pass_dense_roundtrip(zk):
    import torch
    L = 25
    log("ntt three-pass dense round trip 2^%d" % L)
    x = _dense_input(4300, L)
    A = zk.ntt(x)
    back = zk.intt(A)
    torch.cuda.synchronize()
    assert torch.equal(back, x)
    # in place: in == out for both directions
    y = x.clone()
    zk.ntt(y, out=y)
    torch.cuda.synchronize()
    assert torch.equal(y, A)
    zk.intt(y, out=y)
    torch.cuda.synchronize()
    assert torch.equal(y, x)
    # the Sum identity on the dense input: sum_j A_j = N a_0
    a0 = fr_from_host(x[:1].cpu().numpy().view(np.uint32))[0]
    assert _sum_mod_r(A) == (1 << L) * a0 % R
    del x, A, back, y


def test_ntt_workspace_bytes(zk):
    assert zk.ntt_workspace_bytes(28) == 32 << 28
    assert zk.ntt_workspace_bytes(29) == 0
