"""Affine BN254 G1 arithmetic (test oracle only).

G1 is the curve y^2 = x^3 + 3 over Fq with generator G = (1, 2); its order is
the prime r, cofactor 1 (Preliminaries: [x]_1 = xG).  A point is a pair of
canonical ints (x, y), and the point at infinity O is ``None``.  For byte
exchange O is written (0, 0), which is not on the curve because 0 != 3.

Addition uses the textbook chord-and-tangent formulas with every special case
spelled out (O operand, P + (-P), P + P).  Scalar multiplication is
most-significant-bit-first double-and-add.
"""
from .field import P, R, fq_inv, fq_sqrt

B = 3
G = (1, 2)
O = None


def on_curve(pt) -> bool:
    if pt is None:
        return True
    x, y = pt
    return 0 <= x < P and 0 <= y < P and (y * y - x * x * x - B) % P == 0


def neg(pt):
    if pt is None:
        return None
    x, y = pt
    return (x, (-y) % P)


def add(p1, p2):
    if p1 is None:
        return p2
    if p2 is None:
        return p1
    x1, y1 = p1
    x2, y2 = p2
    if x1 == x2:
        if (y1 + y2) % P == 0:
            return None              # P + (-P), also the tangent at y = 0
        return double(p1)            # P + P
    lam = (y2 - y1) * fq_inv(x2 - x1) % P
    x3 = (lam * lam - x1 - x2) % P
    y3 = (lam * (x1 - x3) - y1) % P
    return (x3, y3)


def double(p1):
    if p1 is None:
        return None
    x1, y1 = p1
    if y1 == 0:
        return None
    lam = 3 * x1 * x1 * fq_inv(2 * y1) % P
    x3 = (lam * lam - 2 * x1) % P
    y3 = (lam * (x1 - x3) - y1) % P
    return (x3, y3)


def mul(k: int, pt):
    """k * pt for any integer k >= 0 (no reduction of k), MSB-first."""
    if k < 0:
        return mul(-k, neg(pt))
    acc = None
    for bit in bin(k)[2:] if k else "":
        acc = double(acc)
        if bit == "1":
            acc = add(acc, pt)
    return acc


def gen_mul(k: int):
    """[k]_1 = kG with k reduced mod r."""
    return mul(k % R, G)


def lift_x(x: int):
    """A curve point with abscissa x (the even-y root), or None if x^3+3 is a non-square."""
    y = fq_sqrt((x * x * x + B) % P)
    if y is None:
        return None
    if y & 1:
        y = P - y
    return (x % P, y)


def encode(pt):
    """Canonical affine encoding; O -> (0, 0)."""
    return (0, 0) if pt is None else (pt[0], pt[1])


def decode(xy):
    x, y = int(xy[0]), int(xy[1])
    return None if (x == 0 and y == 0) else (x, y)
