"""Quotient by the vanishing polynomial X^n - 1 (test oracle only).

Mul (Foldable basic blocks): the prover shows f(w) h(w) = g(w) on H = {omega^i}
by committing to t = (f h - g) / (X^n - 1), where f, h, g interpolate the
witness vectors a, b, c (c_i = a_i b_i) on H.  The polynomials come from the
evaluations by the inverse transform; the product f h is formed with the
transform (zero-padded to 2n, pointwise product, inverse), and the division
by the monic X^n - 1 is schoolbook long division from the top coefficient
down.  A nonzero remainder means c is not the entrywise product of a and b.
"""
from .field import R
from .ntt import fft, horner, ifft


def poly_mul_fft(f, h):
    """f * h by zero-padded transforms (exact over Fr)."""
    if not f or not h:
        return []
    m = len(f) + len(h) - 1
    size = 1
    while size < m:
        size *= 2
    F = fft(list(f) + [0] * (size - len(f)))
    H = fft(list(h) + [0] * (size - len(h)))
    return ifft([x * y % R for x, y in zip(F, H)])[:m]


def divide_by_vanishing(p, n: int):
    """(t, rem) with p = t (X^n - 1) + rem, deg rem < n."""
    work = [int(c) % R for c in p]
    if len(work) <= n:
        return [], work + [0] * (n - len(work))
    t = [0] * (len(work) - n)
    for i in range(len(work) - 1, n - 1, -1):
        c = work[i]
        if c:
            t[i - n] = (t[i - n] + c) % R
            work[i - n] = (work[i - n] + c) % R   # subtracting c X^(i-n) (X^n - 1) adds c X^(i-n)
            work[i] = 0
    return t, work[:n]


def mul_quotient(a, b, c):
    """(t, rem, (f, h, g)) for witness vectors a, b, c of length n on H:
    t = (f h - g) / (X^n - 1); t is padded to n coefficients (deg t <= n - 2)."""
    n = len(a)
    f, h, g = ifft(a), ifft(b), ifft(c)
    p = poly_mul_fft(f, h)
    for i, gi in enumerate(g):
        p[i] = (p[i] - gi) % R
    t, rem = divide_by_vanishing(p, n)
    t = t + [0] * (n - len(t))
    return t, rem, (f, h, g)


def vanishing_at(z: int, n: int) -> int:
    return (pow(z, n, R) - 1) % R


def quotient_identity_holds(t, f, h, g, z: int, n: int) -> bool:
    """t(z) (z^n - 1) == f(z) h(z) - g(z)."""
    lhs = horner(t, z) * vanishing_at(z, n) % R
    rhs = (horner(f, z) * horner(h, z) - horner(g, z)) % R
    return lhs == rhs
