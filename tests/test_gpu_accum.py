"""GPU parity of the accumulation step (zk_acc_fold) and the transcript
challenge (zk_transcript_challenge) against the oracle, bit-exact: the
FIPS 180-4 example messages, transcripts of several lengths (padding
boundaries), and folds with k commitments, relation degrees d = 1..5,
points at infinity, gamma = 0 and 1, and long Fr vectors; then a two-level
tree of full folds whose challenges come from the device transcript.
"""
import os

import numpy as np
import pytest

from oracle import field, fold as ofold, g1, transcript as otr
from tests.gpu_helpers import fr_from_host, log, points_from_host, points_to_host
from workloads import generators as gen
from workloads import ints_to_limbs, limbs_to_ints

pytestmark = pytest.mark.gpu
R = field.R
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sha256_fips180_4.txt")


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


def _bytes_dev(zk, b):
    import torch
    return torch.tensor(list(b), dtype=torch.uint8, device="cuda")


def test_transcript_fips_and_lengths(zk):
    import torch
    msgs = []
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            msgs.append(line.split()[0].encode())
    rng = np.random.default_rng(5)
    # lengths around the 55/56/64-byte padding boundaries (one prefix byte added)
    msgs += [bytes(rng.integers(0, 256, L, dtype=np.uint8)) for L in (0, 1, 54, 55, 56, 63, 64, 119, 1000, 4099)]
    for m in msgs:
        log("transcript", len(m))
        if m:
            out = zk.transcript_challenge(_bytes_dev(zk, m))
        else:
            out = zk.transcript_challenge(torch.empty(0, dtype=torch.uint8, device="cuda"))
        assert fr_from_host(_host(zk, out))[0] == otr.challenge(m)


def _rand_points(seed, n, with_inf=False):
    ks = limbs_to_ints(gen.uniform_fr(seed, n, tag=4))
    pts = [g1.gen_mul(k) for k in ks]
    if with_inf and n:
        pts[0] = None
    return pts


def _dev_pts(zk, pts):
    return zk.to_device(points_to_host(pts))


@pytest.mark.parametrize("k,d,len_v,len_e,gkind", [
    (1, 1, 0, 0, "rand"), (3, 2, 5, 4, "rand"), (17, 3, 1000, 257, "rand"), (2, 5, 3, 3, "zero"),
    (5, 4, 7, 9, "one"), (64, 2, 1 << 16, 1 << 12, "rand"),
    (16, 15, 3, 2, "rand"), (33, 7, 0, 0, "minus1"),
])
def test_acc_fold_exact(zk, k, d, len_v, len_e, gkind):
    seed = 9400 + 7 * k + d
    gam = {"zero": 0, "one": 1, "minus1": R - 1}.get(gkind)
    if gam is None:
        gam = limbs_to_ints(gen.uniform_fr(seed, 1, tag=8))[0]
    C = _rand_points(seed, k, with_inf=True)
    C2 = _rand_points(seed + 1, k)
    E, E2 = _rand_points(seed + 2, 2, with_inf=(d == 2))
    Ej = _rand_points(seed + 3, d - 1)
    v = gen.uniform_fr(seed, len_v, tag=1)
    v2 = gen.uniform_fr(seed, len_v, tag=2)
    e = gen.uniform_fr(seed, len_e, tag=3)
    e2 = gen.uniform_fr(seed, len_e, tag=5)
    ej = gen.uniform_fr(seed, (d - 1) * len_e, tag=6)
    log("acc fold k=%d d=%d len_v=%d len_e=%d gamma=%s" % (k, d, len_v, len_e, gkind))
    dv = (lambda a: zk.to_device(a) if len(a) else None)
    C_out, E_out, v_out, e_out = zk.acc_fold(
        zk.to_device(ints_to_limbs([gam]).reshape(1, 8)), _dev_pts(zk, C), _dev_pts(zk, C2), _dev_pts(zk, [E]),
        _dev_pts(zk, [E2]), _dev_pts(zk, Ej) if d > 1 else None, dv(v), dv(v2), dv(e), dv(e2),
        zk.to_device(ej).reshape(d - 1, len_e, 8) if d > 1 and len_e else None)
    ejv = fr_from_host(ej) if len(ej) else []
    want = ofold.acc_fold(gam, C, C2, E, E2, Ej, fr_from_host(v) if len_v else [], fr_from_host(v2) if len_v else [],
                          fr_from_host(e) if len_e else [], fr_from_host(e2) if len_e else [],
                          [ejv[j * len_e:(j + 1) * len_e] for j in range(d - 1)])
    assert points_from_host(_host(zk, C_out)) == want[0]
    assert points_from_host(_host(zk, E_out))[0] == want[1]
    if len_v:
        assert fr_from_host(_host(zk, v_out)) == want[2]
    if len_e:
        assert fr_from_host(_host(zk, e_out)) == want[3]


def test_acc_fold_tree_with_device_transcript(zk):
    # four accumulators folded as a two-level tree; each challenge is the
    # device transcript of the two instances' commitments and E terms
    import torch
    k, d, n = 4, 2, 300
    accs = []
    for i in range(4):
        C = _rand_points(9500 + 10 * i, k)
        E = _rand_points(9501 + 10 * i, 1)[0]
        v = fr_from_host(gen.uniform_fr(9502 + 10 * i, n))
        accs.append((C, E, v))
    Ej_all = [_rand_points(9600 + j, 1) for j in range(3)]
    dev = [(_dev_pts(zk, C), _dev_pts(zk, [E]), zk.to_device(ints_to_limbs(v).reshape(n, 8))) for C, E, v in accs]

    def fold_two(a, b, ej, dev_a, dev_b):
        tr = torch.cat([dev_a[0].flatten(), dev_a[1].flatten(), dev_b[0].flatten(), dev_b[1].flatten(),
                        _dev_pts(zk, ej).flatten()]).contiguous()
        gam_dev = zk.transcript_challenge(tr)
        torch.cuda.synchronize()
        gam = otr.challenge(tr.cpu().numpy().tobytes())
        assert fr_from_host(_host(zk, gam_dev))[0] == gam
        C_out, E_out, v_out, _ = zk.acc_fold(gam_dev, dev_a[0], dev_b[0], dev_a[1], dev_b[1], _dev_pts(zk, ej),
                                             dev_a[2], dev_b[2])
        want = ofold.acc_fold(gam, a[0], b[0], a[1], b[1], ej, a[2], b[2], [], [], [])
        return (want[0], want[1], want[2]), (C_out, E_out, v_out)

    l0, d0 = fold_two(accs[0], accs[1], Ej_all[0], dev[0], dev[1])
    l1, d1 = fold_two(accs[2], accs[3], Ej_all[1], dev[2], dev[3])
    top, dtop = fold_two(l0, l1, Ej_all[2], d0, d1)
    assert points_from_host(_host(zk, dtop[0])) == top[0]
    assert points_from_host(_host(zk, dtop[1]))[0] == top[1]
    assert fr_from_host(_host(zk, dtop[2])) == top[2]
