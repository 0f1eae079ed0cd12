"""KZG opening and batch opening (test oracle only).

Polynomial Commitment: to open f at a point x the prover returns y = f(x)
and the proof pi = [q(tau)]_1 for the quotient q(X) = (f(X) - y) / (X - x);
the verifier compares e(pi, [tau - x]_2) with e(com - [y]_1, [1]_2).
Several polynomials opened at the same x are batched with a verifier
challenge gamma: the prover sends every f_i(x) and one proof [h(tau)]_1 for
h(X) = sum_i gamma^i (f_i(X) - f_i(x)) / (X - x).

Polynomials are coefficient lists, lowest degree first, over Fr.

The division is schoolbook long division by the monic linear X - x, i.e.
synthetic division: working down from the leading coefficient, each quotient
coefficient is the next coefficient of f plus x times the previous quotient
coefficient, and what is left at the bottom is the remainder f(x).  The batch
form combines the numerators first and divides once, as the definition of h
reads.  With the trapdoor tau known (tests only), the pairing check reduces
to the G1 identity com - y G = (tau - x) pi, since both sides are the
commitment to f - y = (X - x) q.
"""
from . import g1, msm
from .field import R
from .ntt import horner


def divide_by_linear(coeffs, x: int):
    """(q, rem) with f(X) = q(X) (X - x) + rem; len(q) = len(f) - 1."""
    f = [int(c) % R for c in coeffs]
    if not f:
        return [], 0
    n = len(f)
    q = [0] * (n - 1)
    carry = f[n - 1]
    for i in range(n - 2, -1, -1):
        q[i] = carry
        carry = (f[i] + x * carry) % R
    return q, carry


def open_at(coeffs, x: int):
    """(y, q): y = f(x) and the opening quotient q = (f - y) / (X - x)."""
    y = horner(coeffs, x)
    shifted = [int(c) % R for c in coeffs]
    if shifted:
        shifted[0] = (shifted[0] - y) % R
    q, rem = divide_by_linear(shifted, x)
    if rem != 0:
        raise ArithmeticError("f - f(x) is not divisible by X - x")
    return y, q


def batch_open_at(polys, x: int, gamma: int):
    """(ys, h): ys[i] = f_i(x) and h = sum_i gamma^i (f_i - f_i(x)) / (X - x).

    The polynomials may differ in length; h has max(len) - 1 coefficients."""
    ys = [horner(f, x) for f in polys]
    n = max((len(f) for f in polys), default=0)
    num = [0] * n
    gi = 1
    for f, y in zip(polys, ys):
        for j, c in enumerate(f):
            num[j] = (num[j] + gi * int(c)) % R
        if f:
            num[0] = (num[0] - gi * y) % R
        gi = gi * gamma % R
    h, rem = divide_by_linear(num, x)
    if rem != 0:
        raise ArithmeticError("combined numerator is not divisible by X - x")
    return ys, h


def proof_closed_form(tau: int, q):
    """pi = [q(tau)]_1 over the SRS [tau^i]_1 (closed form of the MSM)."""
    return msm.srs_msm_closed_form(tau, q)


def verify_with_trapdoor(tau: int, com, x: int, y: int, pi) -> bool:
    """The pairing equation with tau known: com - y G == (tau - x) pi."""
    lhs = g1.add(com, g1.neg(g1.gen_mul(y % R)))
    rhs = g1.mul((tau - x) % R, pi)
    return lhs == rhs


def batch_verify_with_trapdoor(tau: int, coms, x: int, ys, gamma: int, pi) -> bool:
    """sum_i gamma^i (com_i - y_i G) == (tau - x) pi."""
    lhs = None
    gi = 1
    for com, y in zip(coms, ys):
        lhs = g1.add(lhs, g1.mul(gi, g1.add(com, g1.neg(g1.gen_mul(y % R)))))
        gi = gi * gamma % R
    return lhs == g1.mul((tau - x) % R, pi)
