"""Interval analysis of the lazily-reduced 29-bit-limb field arithmetic.

The HIP kernels keep Fq/Fr elements in nine 29-bit limbs (radix 2^29,
Montgomery radix R = 2^261) and reduce lazily: a Montgomery product is only
guaranteed < V_a V_b / 2^261 + q, and a subtraction a - b is computed as
a + K - b with K a fixed multiple of q written in "borrowed" limbs.  This
script replays every point formula the kernels use on upper bounds of values
and limbs, and checks

* no 64-bit column accumulator of a product can overflow,
* every subtraction's K exceeds its subtrahend (value and every limb), and
  no 32-bit limb overflows before carry normalisation,
* the XYZZ coordinates of a running sum stay inside the invariant box the
  formulas assume (a fixed point), so chains of any length stay bounded.

It imports nothing from the rest of the repository; the constants mirror the
tables in field_constants.h and the sub_k multiples in curve.h, and
tests/test_host_bounds.py checks both against those sources and runs
check_all().
"""
from fractions import Fraction

P = 0x30644E72E131A029B85045B68181585D97816A916871CA8D3C208C16D87CFD47
R_FR = 0x30644E72E131A029B85045B68181585D2833E84879B9709143E1F593F0000001
LIMB = 29
NLIMB = 9
MASK = (1 << LIMB) - 1
MONT_R = 1 << (LIMB * NLIMB)  # 2^261


def digits(x):
    return [(x >> (LIMB * i)) & MASK for i in range(NLIMB)] if x < (1 << (LIMB * NLIMB)) else None


def borrowed(cq):
    """K = cq with limbs 0..7 raised by 2^31 (borrowing 4 from the next limb)."""
    d = digits(cq)
    k = [d[0] + (1 << 31)] + [d[i] + (1 << 31) - 4 for i in range(1, 8)] + [d[8] - 4]
    assert sum(v << (LIMB * i) for i, v in enumerate(k)) == cq
    assert all(v >= 0 for v in k)
    return k


def borrowed30(cq):
    """K = cq with limbs 0..7 raised by 2^30 (borrowing 2 from the next limb)."""
    d = digits(cq)
    k = [d[0] + (1 << 30)] + [d[i] + (1 << 30) - 2 for i in range(1, 8)] + [d[8] - 2]
    assert sum(v << (LIMB * i) for i, v in enumerate(k)) == cq
    assert all(v >= 0 for v in k)
    return k


class V:
    """Upper bounds of a non-negative value and of each of its limbs."""

    def __init__(self, val, limb, top=None):
        self.val = val      # value < val
        self.limb = limb    # limbs 0..7 < limb
        self.top = top if top is not None else min(limb, -(-val // (1 << (LIMB * 8))))

    def __repr__(self):
        return "V(%.3f q, limb 2^%.2f)" % (self.val / Q, self.limb.bit_length() - 1)


Q = P


def norm(val):
    """A normalised element (limbs < 2^29) of value < val."""
    assert val <= (1 << (LIMB * NLIMB)), "value does not fit nine limbs"
    return V(val, 1 << LIMB, (val >> (LIMB * 8)) + 1)


def mul(a, b, q=None):
    q = q or Q
    la, lb = max(a.limb, a.top), max(b.limb, b.top)
    col = 9 * (la - 1) * (lb - 1) + 9 * MASK * MASK + (1 << 64) // (1 << LIMB)
    assert col < (1 << 64), "column accumulator overflow"
    return norm((a.val - 1) * (b.val - 1) // MONT_R + q + 1)


def sub_raw(a, b, c, q=None):
    """a - b computed as a + c*q - b with c*q in 2^30-raised limbs, left
    unnormalised: limb i of the result is below a's limb bound + k_i."""
    q = q or Q
    k = borrowed30(c * q)
    assert c * q >= b.val - 1, "K = %dq does not exceed the subtrahend" % c
    assert all(k[i] >= b.limb - 1 for i in range(8)), "limb borrow too small"
    assert k[8] >= b.top - 1, "top limb borrow too small"
    limb = max(a.limb + k[i] for i in range(8))
    top = a.top + k[8]
    assert limb <= (1 << 32) and top <= (1 << 32), "32-bit limb overflow"
    return V(a.val + c * q, limb, top)


def mul2(a, b, c, d, q=None):
    """(a b + c d) / 2^261 with one reduction: both products' column sums
    share the 64-bit accumulators."""
    q = q or Q
    la, lb = max(a.limb, a.top), max(b.limb, b.top)
    lc, ld = max(c.limb, c.top), max(d.limb, d.top)
    col = 9 * (la - 1) * (lb - 1) + 9 * (lc - 1) * (ld - 1) + 9 * MASK * MASK + (1 << 64) // (1 << LIMB)
    assert col < (1 << 64), "column accumulator overflow"
    return norm(((a.val - 1) * (b.val - 1) + (c.val - 1) * (d.val - 1)) // MONT_R + q + 1)


def add(a, b):
    return V(a.val + b.val - 1, a.limb + b.limb - 1, a.top + b.top - 1)


def addn(a, b):
    """a + b followed by carry normalisation."""
    return norm(a.val + b.val - 1)


def sub(a, b, c, q=None):
    """a - b computed as a + c*q - b (then normalised)."""
    q = q or Q
    k = borrowed(c * q)
    assert c * q >= b.val - 1, "K = %dq does not exceed the subtrahend" % c
    assert all(k[i] >= b.limb - 1 for i in range(8)), "limb borrow too small"
    assert k[8] >= b.top - 1, "top limb borrow too small"
    assert all(a.limb - 1 + k[i] < (1 << 32) for i in range(8)), "32-bit limb overflow"
    assert a.top - 1 + k[8] < (1 << 32)
    return norm(a.val + c * q)


# Subtraction tables used by the kernels (field_constants.h): "K<c>" is c q in
# 2^31-raised limbs (sub_k, normalised result), "H<c>" c q in 2^30-raised
# limbs (sub_raw, unnormalised result).  In the additions Y3 = R (Q - X3) -
# S PPP is one reduction of R (Q - X3) + (K - S) PPP, with "nY1" / "nS1" the
# negation K - S and Q - X3 unnormalised.
SUB_K = {"madd.P": "K8", "madd.R": "K8", "madd.X3": "K4", "madd.QX": "H8", "madd.nY1": "K8",
         "add.P": "K8", "add.R": "K8", "add.X3": "K4", "add.QX": "H8", "add.nS1": "K8",
         "dbl.X3": "K4", "dbl.SX": "K8", "dbl.Y3": "K2"}


def _sub(name, a, b):
    t = SUB_K[name]
    return (sub_raw if t[0] == "H" else sub)(a, b, int(t[1:]))

ZERO = V(1, 1, 1)  # the constant 0 (bounds are exclusive)


def madd(X1, Y1, ZZ1, ZZZ1, x2, y2):
    U2 = mul(x2, ZZ1)
    S2 = mul(y2, ZZZ1)
    Pv = _sub("madd.P", U2, X1)
    Rv = _sub("madd.R", S2, Y1)
    # the signed form: -p gives R = 8q - (S2 + Y1); both must hold, keep the larger
    Rneg = _sub("madd.R", ZERO, add(S2, Y1))
    Rv = Rv if Rv.val >= Rneg.val and Rv.limb >= Rneg.limb and Rv.top >= Rneg.top else Rneg
    PP = mul(Pv, Pv)
    PPP = mul(Pv, PP)
    Qv = mul(X1, PP)
    R2 = mul(Rv, Rv)
    T = add(add(PPP, Qv), Qv)
    X3 = _sub("madd.X3", R2, T)
    QX = _sub("madd.QX", Qv, X3)
    nY1 = _sub("madd.nY1", ZERO, Y1)
    Y3 = mul2(Rv, QX, nY1, PPP)
    return X3, Y3, mul(ZZ1, PP), mul(ZZZ1, PPP)


def add_xyzz(X1, Y1, ZZ1, ZZZ1, X2, Y2, ZZ2, ZZZ2):
    U1 = mul(X1, ZZ2)
    U2 = mul(X2, ZZ1)
    S1 = mul(Y1, ZZZ2)
    S2 = mul(Y2, ZZZ1)
    Pv = _sub("add.P", U2, U1)
    Rv = _sub("add.R", S2, S1)
    PP = mul(Pv, Pv)
    PPP = mul(Pv, PP)
    Qv = mul(U1, PP)
    R2 = mul(Rv, Rv)
    T = add(add(PPP, Qv), Qv)
    X3 = _sub("add.X3", R2, T)
    QX = _sub("add.QX", Qv, X3)
    nS1 = _sub("add.nS1", ZERO, S1)
    Y3 = mul2(Rv, QX, nS1, PPP)
    return X3, Y3, mul(mul(ZZ1, ZZ2), PP), mul(mul(ZZZ1, ZZZ2), PPP)


def dbl_xyzz(X1, Y1, ZZ1, ZZZ1):
    U = add(Y1, Y1)
    Vv = mul(U, U)
    W = mul(U, Vv)
    S = mul(X1, Vv)
    X1sq = mul(X1, X1)
    M = addn(add(X1sq, X1sq), X1sq)
    M2 = mul(M, M)
    X3 = _sub("dbl.X3", M2, add(S, S))
    SX = _sub("dbl.SX", S, X3)
    A = mul(M, SX)
    B = mul(W, Y1)
    Y3 = _sub("dbl.Y3", A, B)
    return X3, Y3, mul(Vv, ZZ1), mul(W, ZZZ1)


# Invariant box for XYZZ coordinates of any running sum.
BOX = (norm(6 * P), norm(4 * P), norm(P + (P >> 2)), norm(P + (P >> 2)))
AFFINE = (norm(P + 1), norm(P + 1))


def inside(pt, box=BOX):
    return all(c.val <= b.val and c.limb <= b.limb and c.top <= b.top for c, b in zip(pt, box))


def check_all():
    """Run every formula on the invariant box; return the output bounds."""
    out = {}
    m = madd(*BOX, *AFFINE)
    assert inside(m), ("madd leaves the box", m)
    out["madd"] = m
    a = add_xyzz(*BOX, *BOX)
    assert inside(a), ("add leaves the box", a)
    out["add"] = a
    d = dbl_xyzz(*BOX)
    assert inside(d), ("dbl leaves the box", d)
    out["dbl"] = d
    # an affine point lifted to XYZZ (ZZ = ZZZ = Montgomery one < q) is inside
    assert inside((AFFINE[0], AFFINE[1], norm(P), norm(P)))
    # Fr butterflies: twiddle products of canonical inputs are < 2r
    t = mul(norm(R_FR), norm(R_FR), R_FR)
    assert t.val <= 2 * R_FR
    return out


if __name__ == "__main__":
    for k, v in check_all().items():
        print(k, v)
