"""Pins for the oracle's BN254 fields (Experimental Setup: BN254, 254-bit prime field)."""
from oracle import field

# The BN254 moduli as published hexadecimal constants, typed independently of
# the BN-polynomial definition the oracle uses.
P_HEX = 0x30644E72E131A029B85045B68181585D97816A916871CA8D3C208C16D87CFD47
R_HEX = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001


def test_moduli_match_published_constants():
    assert field.P == P_HEX
    assert field.R == R_HEX
    assert field.P.bit_length() == 254 and field.R.bit_length() == 254


def test_moduli_are_prime_and_test_rejects_composites():
    assert field.is_probable_prime(field.P)
    assert field.is_probable_prime(field.R)
    # Carmichael number, a square of a prime and a product of two primes.
    assert not field.is_probable_prime(561)
    assert not field.is_probable_prime(1000003 * 1000003)
    assert not field.is_probable_prime(field.P * 1000003)
    assert not field.is_probable_prime(field.R + 1)  # even


def test_two_adicity_and_root_generator():
    assert (field.R - 1) % (1 << 28) == 0
    assert ((field.R - 1) >> 28) % 2 == 1
    # 5 is a quadratic non-residue mod r (Euler's criterion gives -1).
    assert pow(field.GENERATOR_FR, (field.R - 1) // 2, field.R) == field.R - 1


def test_p_is_3_mod_4_and_sqrt(rng):
    assert field.P % 4 == 3
    for _ in range(50):
        a = rng.randrange(field.P)
        s = field.fq_sqrt(a * a % field.P)
        assert s is not None and s * s % field.P == a * a % field.P
    # -1 is a non-residue when p = 3 mod 4
    assert field.fq_sqrt(field.P - 1) is None


def test_inverses_agree_with_fermat(rng):
    for _ in range(50):
        a = rng.randrange(1, field.R)
        assert field.fr_inv(a) == pow(a, field.R - 2, field.R)
        assert field.fr_mul(a, field.fr_inv(a)) == 1
        b = rng.randrange(1, field.P)
        assert field.fq_inv(b) == pow(b, field.P - 2, field.P)
        assert field.fq_mul(b, field.fq_inv(b)) == 1


def test_field_ops_are_reduced(rng):
    for _ in range(50):
        a, b = rng.randrange(field.R), rng.randrange(field.R)
        for v in (field.fr_add(a, b), field.fr_sub(a, b), field.fr_mul(a, b)):
            assert 0 <= v < field.R
        assert field.fr_sub(field.fr_add(a, b), b) == a
