"""KZG commitment as a multi-scalar multiplication (test oracle only).

Polynomial Commitment: the commitment to f is [f(tau)]_1.  With the SRS
[tau^i]_1 and coefficients f_i this is sum_i f_i [tau^i]_1, i.e. the
multi-scalar multiplication sum_i s_i P_i.  The oracle forms that sum the
slowest obvious way -- one double-and-add scalar multiple per term, added up
in affine coordinates -- and, when the trapdoor is known, by the closed form
(sum_i s_i tau^i mod r) G, which needs no SRS at all.
"""
from . import g1
from .field import R


def naive_msm(points, scalars):
    """sum_i scalars[i] * points[i]; scalars are non-negative integers."""
    if len(points) != len(scalars):
        raise ValueError("length mismatch")
    acc = None
    for pt, s in zip(points, scalars):
        acc = g1.add(acc, g1.mul(int(s), pt))
    return acc


def srs_msm_closed_form(tau: int, scalars):
    """sum_i s_i [tau^i]_1 = (sum_i s_i tau^i mod r) G, evaluated by Horner."""
    acc = 0
    for s in reversed(list(scalars)):
        acc = (acc * tau + int(s)) % R
    return g1.gen_mul(acc)


def gen_msm_closed_form(ks, scalars):
    """sum_i s_i [k_i]_1 = (sum_i s_i k_i mod r) G for bases given by their logs k_i."""
    acc = 0
    for k, s in zip(ks, scalars):
        acc = (acc + int(k) * int(s)) % R
    return g1.gen_mul(acc)
