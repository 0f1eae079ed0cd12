"""Structured reference string [tau^0]_1, [tau^1]_1, ... (test oracle only).

Polynomial Commitment: KZG commits against srs = ([tau^i]_1)_i for a uniform
trapdoor tau.  In deployment it comes from a powers-of-tau ceremony; tests
know tau and build it point by point as [tau^i mod r]_1 by double-and-add.
"""
from . import g1
from .field import R


def srs_point(tau: int, i: int):
    return g1.gen_mul(pow(tau, i, R))


def srs(tau: int, n: int):
    out = []
    t = 1
    for _ in range(n):
        out.append(g1.gen_mul(t))
        t = t * tau % R
    return out
