"""Pins for the oracle's KZG opening and batch opening.

Polynomial Commitment: open returns y = f(x) and [q(tau)]_1 with
q = (f - y) / (X - x); a batch at one point uses h = sum_i gamma^i
(f_i - f_i(x)) / (X - x).  The pins check the division against what fixes
it independently: multiplying back, the explicit coefficient sum, special
points (0, 1, a root), a hand-worked example, and the verifier's equation
with the trapdoor known, evaluated in G1 by the oracle's group law.
"""
from oracle import field, g1, kzg, msm, srs
from oracle.ntt import horner, root_of_unity

R = field.R


def _poly_mul(a, b):
    """Schoolbook product of coefficient lists."""
    if not a or not b:
        return []
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] = (out[i + j] + x * y) % R
    return out


def _trim(p):
    p = [c % R for c in p]
    while p and p[-1] == 0:
        p.pop()
    return p


def test_hand_worked_example():
    # f = 1 + 2X + 3X^2 at x = 2: y = 17, f - 17 = 3X^2 + 2X - 16 = (X - 2)(3X + 8)
    y, q = kzg.open_at([1, 2, 3], 2)
    assert y == 17
    assert q == [8, 3]


def test_division_multiplies_back(rng):
    for n in (1, 2, 3, 7, 20):
        f = [rng.randrange(R) for _ in range(n)]
        x = rng.randrange(R)
        q, rem = kzg.divide_by_linear(f, x)
        assert len(q) == n - 1
        back = _poly_mul(q, [(-x) % R, 1]) if q else []
        back = back + [0] * (n - len(back))
        back[0] = (back[0] + rem) % R
        assert back == [c % R for c in f]
        assert rem == horner(f, x)  # remainder theorem


def test_quotient_explicit_sum(rng):
    f = [rng.randrange(R) for _ in range(9)]
    x = rng.randrange(R)
    _, q = kzg.open_at(f, x)
    for i in range(len(f) - 1):
        assert q[i] == sum(f[j] * pow(x, j - i - 1, R) for j in range(i + 1, len(f))) % R


def test_special_points(rng):
    f = [rng.randrange(R) for _ in range(11)]
    y0, q0 = kzg.open_at(f, 0)
    assert y0 == f[0] and q0 == f[1:]
    y1, q1 = kzg.open_at(f, 1)
    assert y1 == sum(f) % R
    assert q1 == [sum(f[i + 1:]) % R for i in range(len(f) - 1)]
    # x a root: f = (X - a) p divides exactly
    a = rng.randrange(R)
    p = [rng.randrange(R) for _ in range(6)]
    fa = _poly_mul([(-a) % R, 1], p)
    ya, qa = kzg.open_at(fa, a)
    assert ya == 0 and qa == p
    # a root of unity of the evaluation domain
    w = root_of_unity(16)
    yw, qw = kzg.open_at(f, w)
    assert yw == horner(f, w)
    z = rng.randrange(R)
    assert (horner(f, z) - yw) % R == (z - w) * horner(qw, z) % R


def test_degenerate_lengths():
    assert kzg.open_at([], 5) == (0, [])
    assert kzg.open_at([7], 5) == (7, [])
    assert kzg.batch_open_at([[], [4]], 3, 9) == ([0, 4], [])


def test_identity_at_random_points(rng):
    f = [rng.randrange(R) for _ in range(33)]
    x = rng.randrange(R)
    y, q = kzg.open_at(f, x)
    for _ in range(4):
        z = rng.randrange(R)
        assert (horner(f, z) - y) % R == (z - x) * horner(q, z) % R


def test_batch_is_gamma_combination_of_single_quotients(rng):
    polys = [[rng.randrange(R) for _ in range(n)] for n in (5, 9, 1, 7)]
    x, gamma = rng.randrange(R), rng.randrange(R)
    ys, h = kzg.batch_open_at(polys, x, gamma)
    want = [0] * 8
    for i, f in enumerate(polys):
        y, q = kzg.open_at(f, x)
        assert ys[i] == y
        for j, c in enumerate(q):
            want[j] = (want[j] + pow(gamma, i, R) * c) % R
    assert h == want
    # gamma = 0 keeps only the first polynomial
    ys0, h0 = kzg.batch_open_at(polys, x, 0)
    assert h0[: len(polys[0]) - 1] == kzg.open_at(polys[0], x)[1]
    assert _trim(h0[len(polys[0]) - 1:]) == []


def test_verifier_equation_with_trapdoor(rng):
    tau = rng.randrange(2, R)
    n = 10
    pts = srs.srs(tau, n)
    f = [rng.randrange(R) for _ in range(n)]
    x = rng.randrange(R)
    y, q = kzg.open_at(f, x)
    com = msm.naive_msm(pts, f)
    pi = msm.naive_msm(pts[: n - 1], q)
    assert pi == kzg.proof_closed_form(tau, q)
    assert kzg.verify_with_trapdoor(tau, com, x, y, pi)
    assert not kzg.verify_with_trapdoor(tau, com, x, (y + 1) % R, pi)
    assert not kzg.verify_with_trapdoor(tau, com, (x + 1) % R, y, pi)
    assert not kzg.verify_with_trapdoor(tau, com, x, y, g1.add(pi, g1.G))


def test_batch_verifier_equation_with_trapdoor(rng):
    tau = rng.randrange(2, R)
    polys = [[rng.randrange(R) for _ in range(6)] for _ in range(3)]
    x, gamma = rng.randrange(R), rng.randrange(R)
    ys, h = kzg.batch_open_at(polys, x, gamma)
    coms = [msm.srs_msm_closed_form(tau, f) for f in polys]
    pi = kzg.proof_closed_form(tau, h)
    assert kzg.batch_verify_with_trapdoor(tau, coms, x, ys, gamma, pi)
    bad = list(ys)
    bad[1] = (bad[1] + 1) % R
    assert not kzg.batch_verify_with_trapdoor(tau, coms, x, bad, gamma, pi)
