"""Pins for the oracle's quotient by X^n - 1 (the Mul block's t = (f h - g) / (X^n - 1)).

Checked against what fixes the division independently: schoolbook
multiplication back, divisibility exactly when c is the entrywise product,
two closed forms (f = 1 and f = X), a hand-derived n = 2 case, and the
identity at random points with f, h, g evaluated barycentrically from the
witness vectors (no inverse transform).
"""
from oracle import field, quotient as oq
from oracle.ntt import barycentric_eval, horner, root_of_unity

R = field.R


def _schoolbook(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] = (out[i + j] + x * y) % R
    return out


def test_fft_product_matches_schoolbook(rng):
    for la, lb in ((1, 1), (3, 5), (8, 8), (13, 4)):
        a = [rng.randrange(R) for _ in range(la)]
        b = [rng.randrange(R) for _ in range(lb)]
        assert oq.poly_mul_fft(a, b) == _schoolbook(a, b)


def test_division_multiplies_back(rng):
    for n, deg in ((1, 5), (4, 3), (4, 12), (8, 15)):
        p = [rng.randrange(R) for _ in range(deg + 1)]
        t, rem = oq.divide_by_vanishing(p, n)
        assert len(rem) == n
        back = _schoolbook(t, [R - 1] + [0] * (n - 1) + [1]) if t else []
        back = back + [0] * (max(len(p), n) - len(back))
        for i, r in enumerate(rem):
            back[i] = (back[i] + r) % R
        assert back[:len(p)] == p and all(v == 0 for v in back[len(p):])


def test_product_witness_divides_exactly(rng):
    for n in (2, 4, 16, 64):
        a = [rng.randrange(R) for _ in range(n)]
        b = [rng.randrange(R) for _ in range(n)]
        c = [x * y % R for x, y in zip(a, b)]
        t, rem, _ = oq.mul_quotient(a, b, c)
        assert rem == [0] * n
        assert len(t) == n and t[n - 1] == 0  # deg t <= n - 2
        bad = list(c)
        bad[n // 2] = (bad[n // 2] + 1) % R
        _, rem_bad, _ = oq.mul_quotient(a, b, bad)
        assert any(rem_bad)


def test_closed_forms(rng):
    n = 16
    w = root_of_unity(n)
    b = [rng.randrange(R) for _ in range(n)]
    # f = 1 (a all ones), g = h: the numerator is zero
    t1, rem1, _ = oq.mul_quotient([1] * n, b, b)
    assert t1 == [0] * n and rem1 == [0] * n
    # f = X (a_i = omega^i): X h - g = h_(n-1) (X^n - 1), so t is the constant
    # h_(n-1) = n^-1 sum_j b_j omega^j, summed directly
    a = [pow(w, i, R) for i in range(n)]
    c = [x * y % R for x, y in zip(a, b)]
    t, rem, _ = oq.mul_quotient(a, b, c)
    top = sum(bj * pow(w, j, R) for j, bj in enumerate(b)) * pow(n, -1, R) % R
    assert t == [top] + [0] * (n - 1) and rem == [0] * n


def test_two_point_domain_by_hand(rng):
    # H = {1, -1}: f = (a0 + a1)/2 + (a0 - a1)/2 X, likewise h; t = f_1 h_1
    a0, a1, b0, b1 = (rng.randrange(R) for _ in range(4))
    half = pow(2, -1, R)
    t, rem, _ = oq.mul_quotient([a0, a1], [b0, b1], [a0 * b0 % R, a1 * b1 % R])
    assert t == [(a0 - a1) * half * (b0 - b1) * half % R, 0]
    assert rem == [0, 0]


def test_identity_at_random_points_barycentric(rng):
    n = 32
    a = [rng.randrange(R) for _ in range(n)]
    b = [rng.randrange(R) for _ in range(n)]
    c = [x * y % R for x, y in zip(a, b)]
    t, _, _ = oq.mul_quotient(a, b, c)
    for _ in range(3):
        z = rng.randrange(R)
        fz, hz, gz = (barycentric_eval(v, z) for v in (a, b, c))
        assert horner(t, z) * oq.vanishing_at(z, n) % R == (fz * hz - gz) % R
