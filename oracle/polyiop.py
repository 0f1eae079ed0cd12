"""Quotient of a Poly-IOP constraint by the vanishing polynomial (test oracle only).

Basic blocks based on a Poly-IOP: the prover knows witness polynomials
f_1 .. f_N with R(f_1(x), .., f_N(x), f_1(omega x), .., f_N(omega x)) = 0 for
every x in H = {omega^i}, and commits to the quotient Q with

    R(f_1(x), .., f_N(x), f_1(omega x), .., f_N(omega x)) = Q(x) (x^n - 1).

Here the witnesses are given as vectors on H (vector k, element i =
f_k(omega^i)), so f_k is their interpolant, and R as a sum of terms
c * x_a * x_b * ...: a term is (c, [a, b, ...]) where a factor index
a < N names f_(a+1)(x) and N <= a < 2N names f_(a-N+1)(omega x).  The paper's
instances:

* BooleanCheck: N = 1, R = x_1 (1 - x_1)             -> [(1, [0]), (r - 1, [0, 0])]
* Sub Check:    N = 2, R = x_2 + x_1 - x_3           -> [(1, [1]), (1, [0]), (r - 1, [2])]
  (f_1 = g, f_2 = d = g(omega x) - g(x))
* i-thIsZero:   N = 2, R = x_1 x_2 (f_1 = L_i, f_2 = d) -> [(1, [0, 1])]

The constraint polynomial is formed the plain way: each f_k by the inverse
transform, f_k(omega x) by scaling coefficient i by omega^i, every product by
zero-padded transforms (``quotient.poly_mul_fft``), the terms summed; then
schoolbook division by X^n - 1 (``quotient.divide_by_vanishing``).  A
nonzero remainder means the witnesses do not satisfy R on H.  The paper's
blinding (f_k + (x^n - 1) b_k) is not applied: it adds multiples of X^n - 1
that the caller's own terms would carry.
"""
from .field import R
from .ntt import ifft, root_of_unity
from .quotient import divide_by_vanishing, poly_mul_fft

BOOLEAN_CHECK = [(1, [0]), (R - 1, [0, 0])]
SUB_CHECK = [(1, [1]), (1, [0]), (R - 1, [2])]
ITH_IS_ZERO = [(1, [0, 1])]


def degree(terms) -> int:
    """Total degree of R (the largest number of factors in a term)."""
    return max((len(f) for _, f in terms), default=0)


def shifted(coeffs):
    """Coefficients of f(omega x) from those of f (omega = omega_n, n = len)."""
    n = len(coeffs)
    w = root_of_unity(n)
    out = []
    wi = 1
    for c in coeffs:
        out.append(int(c) * wi % R)
        wi = wi * w % R
    return out


def constraint_poly(polys, terms):
    """Coefficients of R(f_1(x), .., f_N(x), f_1(omega x), .., f_N(omega x)),
    with the f_k given by coefficients (all of one length n)."""
    ops = list(polys) + [shifted(p) for p in polys]
    acc = []
    for c, factors in terms:
        c = int(c) % R
        if factors:
            prod = [c * v % R for v in ops[factors[0]]]
        else:
            prod = [c]
        for a in factors[1:]:
            prod = poly_mul_fft(prod, ops[a])
        if len(prod) > len(acc):
            acc += [0] * (len(prod) - len(acc))
        for i, v in enumerate(prod):
            acc[i] = (acc[i] + v) % R
    return acc


def polyiop_quotient(vectors, terms):
    """(Q, rem, polys) for witness vectors (N lists of n values on H):
    Q = R(...) / (X^n - 1), padded to max(d - 1, 1) * n coefficients
    (d = degree(terms); deg Q <= d (n - 1) - n), and the remainder."""
    n = len(vectors[0])
    polys = [ifft(v) for v in vectors]
    p = constraint_poly(polys, terms)
    q, rem = divide_by_vanishing(p, n)
    size = max(degree(terms) - 1, 1) * n
    if len(q) > size and any(q[size:]):
        raise ValueError("quotient longer than the degree bound")
    q = (q + [0] * size)[:size]
    return q, rem, polys


def constraint_at(values, terms) -> int:
    """R at scalar operands: values[a] for factor index a (x_1..x_2N)."""
    acc = 0
    for c, factors in terms:
        t = int(c) % R
        for a in factors:
            t = t * int(values[a]) % R
        acc = (acc + t) % R
    return acc
