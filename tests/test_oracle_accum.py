"""Pins for the oracle's full accumulation step and transcript challenge.

Prover step 5 of Parallel Accumulation: v'' = gamma v + v' and
E'' = E' + sum_j gamma^j E_j + gamma^d E (likewise e'').  Checked against:
the two-term case d = 1; the homomorphism of the commitment (committing
the folded Fr vector equals folding the commitments); G1 against Fr on
known discrete logs; and the special-soundness extraction of the error
polynomial from d + 1 folds with distinct challenges (Lagrange
interpolation recovers e', e_1, ..., e).  The transcript's hash is pinned
to the FIPS 180-4 example digests.
"""
import hashlib
import os

from oracle import field, fold, g1, msm, srs, transcript

R = field.R
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "sha256_fips180_4.txt")


def test_two_term_case(rng):
    E, E2 = g1.gen_mul(rng.randrange(R)), g1.gen_mul(rng.randrange(R))
    gam = rng.randrange(R)
    assert fold.fold_errors_g1(gam, E, E2, []) == g1.add(E2, g1.mul(gam, E))
    assert fold.fold_errors_g1(gam, E, E2, []) == fold.fold_pair(gam, [E], [E2])[0]


def test_commitment_homomorphism(rng):
    tau = rng.randrange(R)
    pts = srs.srs(tau, 6)
    v = [rng.randrange(R) for _ in range(6)]
    v2 = [rng.randrange(R) for _ in range(6)]
    gam = rng.randrange(R)
    lhs = msm.naive_msm(pts, fold.fold_fr(gam, v, v2))
    rhs = fold.fold_pair(gam, [msm.naive_msm(pts, v)], [msm.naive_msm(pts, v2)])[0]
    assert lhs == rhs


def test_g1_errors_match_fr_errors_on_logs(rng):
    d = 4
    xs = [rng.randrange(R) for _ in range(d + 1)]   # logs of E', E_1..E_(d-1), E
    gam = rng.randrange(R)
    E2, Ej, E = g1.gen_mul(xs[0]), [g1.gen_mul(x) for x in xs[1:d]], g1.gen_mul(xs[d])
    want = fold.fold_errors_fr(gam, [xs[d]], [xs[0]], [[x] for x in xs[1:d]])[0]
    assert fold.fold_errors_g1(gam, E, E2, Ej) == g1.gen_mul(want)


def test_error_polynomial_extraction(rng):
    # d + 1 folds with distinct challenges determine e', e_1..e_(d-1), e
    d, n = 3, 4
    e = [rng.randrange(R) for _ in range(n)]
    e2 = [rng.randrange(R) for _ in range(n)]
    ej = [[rng.randrange(R) for _ in range(n)] for _ in range(d - 1)]
    gams = [rng.randrange(R) for _ in range(d + 1)]
    outs = [fold.fold_errors_fr(g, e, e2, ej) for g in gams]
    coeffs = [e2] + ej + [e]
    for i in range(n):
        for deg in range(d + 1):
            # coefficient `deg` of the interpolant through (gamma_t, outs[t][i])
            c = 0
            for t, gt in enumerate(gams):
                num, den = [1], 1
                for u, gu in enumerate(gams):
                    if u != t:
                        num = [(a - gu * b) % R for a, b in zip([0] + num, num + [0])]
                        den = den * (gt - gu) % R
                c = (c + outs[t][i] * num[deg] * pow(den, -1, R)) % R
            assert c == coeffs[deg][i]


def test_acc_fold_bundles_the_parts(rng):
    gam = rng.randrange(R)
    C = [g1.gen_mul(rng.randrange(R)) for _ in range(3)]
    C2 = [g1.gen_mul(rng.randrange(R)) for _ in range(3)]
    E, E2, Ej = (g1.gen_mul(rng.randrange(R)) for _ in range(3))
    v, v2, e, e2 = ([rng.randrange(R) for _ in range(5)] for _ in range(4))
    ej = [[rng.randrange(R) for _ in range(5)]]
    out = fold.acc_fold(gam, C, C2, E, E2, [Ej], v, v2, e, e2, ej)
    assert out[0] == fold.fold_pair(gam, C, C2)
    assert out[1] == g1.add(g1.add(E2, g1.mul(gam, Ej)), g1.mul(gam * gam % R, E))
    assert out[2] == fold.fold_fr(gam, v, v2)
    assert out[3] == fold.fold_errors_fr(gam, e, e2, ej)


def test_sha256_fips_examples():
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        msg, digest = line.split()
        assert hashlib.sha256(msg.encode()).hexdigest() == digest


def test_challenge_in_field_and_input_sensitive():
    a = transcript.challenge(b"instance")
    assert 0 <= a < R
    assert a != transcript.challenge(b"instancf")
    assert transcript.challenge(b"") < R
