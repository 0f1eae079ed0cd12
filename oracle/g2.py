"""BN254 G2 over Fq2 (test oracle only).

Several basic blocks commit in G2 as well as G1 (MulScalar's s', Mul's h',
MatMul's B' and D'): [x]_2 = x H for the G2 generator H.  G2 is the order-r
subgroup of the sextic twist E'(Fq2): y^2 = x^3 + b', b' = 3 / (9 + u), with
Fq2 = Fq[u] / (u^2 + 1).  An Fq2 element is a pair (c0, c1) = c0 + c1 u of
canonical ints; a point is a pair of Fq2 elements, and infinity is None.
Addition uses the textbook chord-and-tangent formulas with every special
case written out; scalar multiplication is double-and-add from the top bit.

H is the generator commonly used for BN254 G2 (as in Ethereum's precompiles);
the tests check that it lies on the twist and has order r.
"""
from .field import P, R

# ---- Fq2 ---------------------------------------------------------------------


def f2(a0, a1=0):
    return (a0 % P, a1 % P)


def f2_add(a, b):
    return ((a[0] + b[0]) % P, (a[1] + b[1]) % P)


def f2_sub(a, b):
    return ((a[0] - b[0]) % P, (a[1] - b[1]) % P)


def f2_neg(a):
    return ((-a[0]) % P, (-a[1]) % P)


def f2_mul(a, b):
    """(a0 + a1 u)(b0 + b1 u) with u^2 = -1."""
    return ((a[0] * b[0] - a[1] * b[1]) % P, (a[0] * b[1] + a[1] * b[0]) % P)


def f2_inv(a):
    """1 / a = conj(a) / (a0^2 + a1^2); a nonzero."""
    norm = (a[0] * a[0] + a[1] * a[1]) % P
    if norm == 0:
        raise ZeroDivisionError("inverse of 0 in Fq2")
    ni = pow(norm, -1, P)
    return (a[0] * ni % P, (-a[1]) * ni % P)


B2 = f2_mul(f2(3), f2_inv(f2(9, 1)))

H = (f2(10857046999023057135944570762232829481370756359578518086990519993285655852781,
        11559732032986387107991004021392285783925812861821192530917403151452391805634),
     f2(8495653923123431417604973247489272438418190587263600148770280649306958101930,
        4082367875863433681332203403145435568316851327593401208105741076214120093531))

# ---- points ------------------------------------------------------------------


def on_curve(pt) -> bool:
    if pt is None:
        return True
    x, y = pt
    return f2_mul(y, y) == f2_add(f2_mul(f2_mul(x, x), x), B2)


def neg(pt):
    return None if pt is None else (pt[0], f2_neg(pt[1]))


def double(pt):
    if pt is None:
        return None
    x, y = pt
    if y == (0, 0):
        return None
    lam = f2_mul(f2_mul(f2(3), f2_mul(x, x)), f2_inv(f2_add(y, y)))
    x3 = f2_sub(f2_mul(lam, lam), f2_add(x, x))
    return (x3, f2_sub(f2_mul(lam, f2_sub(x, x3)), y))


def add(p1, p2):
    if p1 is None:
        return p2
    if p2 is None:
        return p1
    (x1, y1), (x2, y2) = p1, p2
    if x1 == x2:
        if f2_add(y1, y2) == (0, 0):
            return None
        return double(p1)
    lam = f2_mul(f2_sub(y2, y1), f2_inv(f2_sub(x2, x1)))
    x3 = f2_sub(f2_sub(f2_mul(lam, lam), x1), x2)
    return (x3, f2_sub(f2_mul(lam, f2_sub(x1, x3)), y1))


def mul(k: int, pt):
    acc = None
    for bit in bin(k)[2:] if k > 0 else "":
        acc = double(acc)
        if bit == "1":
            acc = add(acc, pt)
    return acc


def gen_mul(k: int):
    return mul(k % R, H)


def naive_msm(points, scalars):
    acc = None
    for pt, s in zip(points, scalars):
        acc = add(acc, mul(int(s), pt))
    return acc


def srs_msm_closed_form(tau: int, scalars):
    """sum_i s_i [tau^i]_2 = (sum_i s_i tau^i mod r) H."""
    acc = 0
    for s in reversed(list(scalars)):
        acc = (acc * tau + int(s)) % R
    return gen_mul(acc)


def srs(tau: int, n: int):
    out, t = [], 1
    for _ in range(n):
        out.append(gen_mul(t))
        t = t * tau % R
    return out


def encode(pt):
    """(x0, x1, y0, y1) ints; infinity -> zeros."""
    if pt is None:
        return (0, 0, 0, 0)
    return (pt[0][0], pt[0][1], pt[1][0], pt[1][1])


def decode(v):
    if all(c == 0 for c in v):
        return None
    return ((v[0], v[1]), (v[2], v[3]))
