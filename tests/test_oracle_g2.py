"""Pins for the oracle's Fq2 and G2 (BN254 twist).

Fq2 against its definition (u^2 = -1 via explicit integer products, inverse
identity, 9 + u is not a square so the twist is well defined); the generator
on the twist with order r; the group laws on random multiples; scalar
multiplication against repeated addition; and the MSM against its closed form.
"""
from oracle import field, g2

P, R = field.P, field.R


def test_fq2_definition(rng):
    for _ in range(20):
        a = (rng.randrange(P), rng.randrange(P))
        b = (rng.randrange(P), rng.randrange(P))
        # (a0 + a1 u)(b0 + b1 u) = a0 b0 + (a0 b1 + a1 b0) u + a1 b1 u^2, u^2 = -1
        assert g2.f2_mul(a, b) == ((a[0] * b[0] - a[1] * b[1]) % P, (a[0] * b[1] + a[1] * b[0]) % P)
        assert g2.f2_mul(a, g2.f2_inv(a)) == (1, 0)
    # u^2 = -1 and u^4 = 1
    u = (0, 1)
    assert g2.f2_mul(u, u) == (P - 1, 0)
    # 9 + u is a non-square in Fq2: its norm 82 is a non-square in Fq
    assert pow(82, (P - 1) // 2, P) == P - 1
    assert g2.f2_mul(g2.B2, (9, 1)) == (3, 0)


def test_generator_order_r():
    assert g2.on_curve(g2.H)
    assert g2.mul(R, g2.H) is None
    assert g2.mul(R - 1, g2.H) == g2.neg(g2.H)
    assert g2.mul(2, g2.H) == g2.double(g2.H) != g2.H


def test_group_laws(rng):
    pts = [g2.gen_mul(rng.randrange(1, R)) for _ in range(4)]
    a, b, c, _ = pts
    assert all(g2.on_curve(p) for p in pts)
    assert g2.add(a, b) == g2.add(b, a)
    assert g2.add(g2.add(a, b), c) == g2.add(a, g2.add(b, c))
    assert g2.add(a, g2.neg(a)) is None
    assert g2.add(a, a) == g2.double(a)
    k1, k2 = rng.randrange(R), rng.randrange(R)
    assert g2.add(g2.gen_mul(k1), g2.gen_mul(k2)) == g2.gen_mul(k1 + k2)


def test_mul_is_repeated_addition(rng):
    p = g2.gen_mul(rng.randrange(1, R))
    acc = None
    for k in range(20):
        assert g2.mul(k, p) == acc
        acc = g2.add(acc, p)


def test_msm_closed_form(rng):
    tau = rng.randrange(R)
    pts = g2.srs(tau, 6)
    s = [rng.randrange(R) for _ in range(6)]
    assert g2.naive_msm(pts, s) == g2.srs_msm_closed_form(tau, s)
    assert g2.naive_msm(pts, [0] * 6) is None
