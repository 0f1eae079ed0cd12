"""Pins for the oracle's commit (MSM), SRS and fold.

Polynomial Commitment: com = [f(tau)]_1 = sum_i f_i [tau^i]_1.
Parallel Accumulation, prover step 5 (v'' = gamma v + v'), run as a tree;
the knowledge-soundness appendix recovers an instance from two folds of the
same pair with different challenges, which the extractor test below repeats.
"""
import pytest

from oracle import field, fold, g1, msm, srs

R = field.R


def test_srs_points(rng):
    tau = rng.randrange(1, R)
    pts = srs.srs(tau, 12)
    assert pts[0] == g1.G
    for i, pt in enumerate(pts):
        assert g1.on_curve(pt)
        assert srs.srs_point(tau, i) == pt
        if i:
            assert g1.mul(tau, pts[i - 1]) == pt


def test_naive_msm_equals_closed_form_on_srs(rng):
    tau = rng.randrange(1, R)
    n = 48
    pts = srs.srs(tau, n)
    s = [rng.randrange(R) for _ in range(n)]
    assert msm.naive_msm(pts, s) == msm.srs_msm_closed_form(tau, s)


def test_msm_brute_force_small_scalars(rng):
    ks = [rng.randrange(R) for _ in range(6)]
    pts = [g1.gen_mul(k) for k in ks]
    s = [0, 1, 2, 3, 5, 4]
    acc = None
    for pt, c in zip(pts, s):
        for _ in range(c):
            acc = g1.add(acc, pt)
    assert msm.naive_msm(pts, s) == acc
    assert msm.gen_msm_closed_form(ks, s) == acc


def test_msm_unit_vectors_and_linearity(rng):
    ks = [rng.randrange(R) for _ in range(8)]
    pts = [g1.gen_mul(k) for k in ks]
    for i in range(8):
        e = [0] * 8
        e[i] = 1
        assert msm.naive_msm(pts, e) == pts[i]
    a = [rng.randrange(R) for _ in range(8)]
    b = [rng.randrange(R) for _ in range(8)]
    ab = [(x + y) % R for x, y in zip(a, b)]
    assert msm.naive_msm(pts, ab) == g1.add(msm.naive_msm(pts, a), msm.naive_msm(pts, b))


def test_msm_edge_cases(rng):
    k = rng.randrange(R)
    pt = g1.gen_mul(k)
    # duplicate bases, P and -P, zero scalars, r-1
    assert msm.naive_msm([pt, pt], [3, 4]) == g1.mul(7, pt)
    assert msm.naive_msm([pt, g1.neg(pt)], [5, 5]) is None
    assert msm.naive_msm([pt] * 3, [0, 0, 0]) is None
    assert msm.naive_msm([pt], [R - 1]) == g1.neg(pt)
    assert msm.naive_msm([], []) is None


def test_fold_pair_is_gamma_left_plus_right(rng):
    a = [g1.gen_mul(rng.randrange(R)) for _ in range(3)]
    b = [g1.gen_mul(rng.randrange(R)) for _ in range(3)]
    gam = rng.randrange(R)
    out = fold.fold_pair(gam, a, b)
    # on the logs: gamma * log(a) + log(b)
    for o, x, y in zip(out, a, b):
        assert o == g1.add(g1.mul(gam, x), y)
    assert fold.tree_fold([a, b], [gam]) == out


@pytest.mark.parametrize("m", [1, 2, 3, 5, 8, 13])
def test_tree_equals_flat_on_points(rng, m):
    logs = [rng.randrange(R) for _ in range(m)]
    inst = [[g1.gen_mul(x)] for x in logs]
    gam = [rng.randrange(R) for _ in range(m - 1)]
    t = fold.tree_fold(inst, gam)
    assert t == fold.flat_fold(inst, gam)
    sig = fold.flat_coefficients(m, gam)
    assert t[0] == g1.gen_mul(sum(s * x for s, x in zip(sig, logs)))


def test_tree_equals_flat_64_scalars(rng):
    # On Fr (the logs of the points) the tree schedule and the flat sum agree.
    m = 64
    vals = [rng.randrange(R) for _ in range(m)]
    gam = [rng.randrange(R) for _ in range(m - 1)]
    level = list(vals)
    gi = 0
    while len(level) > 1:
        nxt = [(gam[gi + j // 2] * level[j] + level[j + 1]) % R for j in range(0, len(level) - 1, 2)]
        gi += len(level) // 2
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    sig = fold.flat_coefficients(m, gam)
    assert level[0] == sum(s * v for s, v in zip(sig, vals)) % R
    # a full binary tree of depth 6: every sigma is a product of between 0 and 6 challenges
    assert sig[-1] == 1


def test_extractor_identity(rng):
    # two folds of the same pair with alpha1 != alpha2 give back the left instance
    a = [g1.gen_mul(rng.randrange(R))]
    b = [g1.gen_mul(rng.randrange(R))]
    a1, a2 = rng.randrange(R), rng.randrange(R)
    f1 = fold.fold_pair(a1, a, b)[0]
    f2 = fold.fold_pair(a2, a, b)[0]
    diff = g1.add(f1, g1.neg(f2))
    assert g1.mul(pow(a1 - a2, -1, R), diff) == a[0]


def test_fold_wrong_gamma_count():
    inst = [[g1.G]] * 4
    with pytest.raises(ValueError):
        fold.tree_fold(inst, [1, 2])
