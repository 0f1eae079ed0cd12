"""BN254 prime fields, as Python integers (test oracle only).

The paper fixes the curve as BN254 over a 254-bit prime field (Experimental
Setup).  BN curves are a one-parameter family: with the BN parameter u,

    p(u) = 36u^4 + 36u^3 + 24u^2 + 6u + 1   (base field Fq, point coordinates)
    r(u) = 36u^4 + 36u^3 + 18u^2 + 6u + 1   (group order; the paper's "p" in
                                             Preliminaries, here the scalar
                                             field Fr)

and BN254 is u = 4965661367192848881.  Elements are canonical ints in [0, q).
"""

BN_U = 4965661367192848881

P = 36 * BN_U**4 + 36 * BN_U**3 + 24 * BN_U**2 + 6 * BN_U + 1
R = 36 * BN_U**4 + 36 * BN_U**3 + 18 * BN_U**2 + 6 * BN_U + 1

# Fr's multiplicative group has order r - 1 = 2^28 * odd; 5 is a quadratic
# non-residue mod r, hence 5^((r-1)/2^k) has exact order 2^k for k <= 28.
TWO_ADICITY = 28
GENERATOR_FR = 5


# ---- Fr (scalars, polynomial coefficients, evaluations) -------------------

def fr(x: int) -> int:
    return x % R


def fr_add(a: int, b: int) -> int:
    return (a + b) % R


def fr_sub(a: int, b: int) -> int:
    return (a - b) % R


def fr_mul(a: int, b: int) -> int:
    return (a * b) % R


def fr_pow(a: int, e: int) -> int:
    return pow(a % R, e, R)


def fr_inv(a: int) -> int:
    """a^(-1) mod r (Python's extended-Euclid modular inverse); a must be nonzero."""
    if a % R == 0:
        raise ZeroDivisionError("inverse of 0 in Fr")
    return pow(a % R, -1, R)


# ---- Fq (point coordinates) ------------------------------------------------

def fq_add(a: int, b: int) -> int:
    return (a + b) % P


def fq_sub(a: int, b: int) -> int:
    return (a - b) % P


def fq_mul(a: int, b: int) -> int:
    return (a * b) % P


def fq_inv(a: int) -> int:
    """a^(-1) mod p (Python's extended-Euclid modular inverse); a must be nonzero."""
    if a % P == 0:
        raise ZeroDivisionError("inverse of 0 in Fq")
    return pow(a % P, -1, P)


def fq_sqrt(a: int):
    """Square root in Fq (p = 3 mod 4): a^((p+1)/4) if it squares back, else None."""
    s = pow(a % P, (P + 1) // 4, P)
    return s if (s * s) % P == a % P else None


def is_probable_prime(n: int, rounds: int = 40) -> bool:
    """Miller-Rabin with the first ``rounds`` primes as bases."""
    if n < 2:
        return False
    small = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61,
             67, 71, 73, 79, 83, 89, 97, 101, 103, 107, 109, 113, 127, 131, 137,
             139, 149, 151, 157, 163, 167, 173, 179, 181]
    for q in small:
        if n % q == 0:
            return n == q
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in small[:rounds]:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = pow(x, 2, n)
            if x == n - 1:
                break
        else:
            return False
    return True
