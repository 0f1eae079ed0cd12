"""Pins for the oracle's affine G1 (Preliminaries: [x]_1 = xG, group of prime order)."""
from oracle import field, g1


def _rand_point(rng):
    while True:
        pt = g1.lift_x(rng.randrange(field.P))
        if pt is not None:
            return pt


def test_generator_on_curve_and_order_r():
    assert g1.on_curve(g1.G)
    assert g1.mul(field.R, g1.G) is None
    assert g1.mul(field.R - 1, g1.G) == g1.neg(g1.G)
    assert g1.mul(field.R + 1, g1.G) == g1.G
    assert g1.mul(0, g1.G) is None


def test_infinity_encoding_is_off_curve():
    x, y = 0, 0
    assert (y * y - x ** 3 - g1.B) % field.P != 0
    assert g1.encode(None) == (0, 0)
    assert g1.decode((0, 0)) is None
    assert g1.decode(g1.encode(g1.G)) == g1.G


def test_special_cases():
    pt = g1.mul(12345, g1.G)
    assert g1.add(pt, g1.neg(pt)) is None
    assert g1.add(pt, pt) == g1.double(pt)
    assert g1.add(None, pt) == pt and g1.add(pt, None) == pt
    assert g1.double(None) is None


def test_scalar_mult_matches_repeated_addition():
    acc = None
    for k in range(40):
        assert g1.mul(k, g1.G) == acc
        acc = g1.add(acc, g1.G)


def test_group_laws_on_random_points(rng):
    for _ in range(5):
        a, b, c = _rand_point(rng), _rand_point(rng), _rand_point(rng)
        for pt in (a, b, c):
            assert g1.on_curve(pt)
            # cofactor 1: every curve point has order r
            assert g1.mul(field.R, pt) is None
        assert g1.add(a, b) == g1.add(b, a)
        assert g1.add(g1.add(a, b), c) == g1.add(a, g1.add(b, c))
        assert g1.on_curve(g1.add(a, b)) and g1.on_curve(g1.double(a))


def test_distributivity(rng):
    for _ in range(5):
        a, b = rng.randrange(field.R), rng.randrange(field.R)
        assert g1.gen_mul(a + b) == g1.add(g1.gen_mul(a), g1.gen_mul(b))
        assert g1.gen_mul(a * b) == g1.mul(a, g1.gen_mul(b))
