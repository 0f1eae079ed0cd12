"""Structured reference string [tau^0]_1, [tau^1]_1, ... (test oracle only).

Polynomial Commitment: KZG commits against srs = ([tau^i]_1)_i for a uniform
trapdoor tau.  In deployment it comes from a powers-of-tau ceremony; tests
know tau and build it point by point as [tau^i mod r]_1 by double-and-add.
The same trapdoor in the Lagrange basis of H (the vector encoding of
Foldable basic blocks) gives [l_j(tau)]_1, against which a vector of
evaluations on H commits directly.
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


def lagrange_basis_at(tau: int, n: int, j: int) -> int:
    """l_j(tau) for the Lagrange basis of H = {omega_n^i}: the polynomial of
    degree < n that is 1 at omega^j and 0 at the other points of H.  For tau
    outside H this is the barycentric weight (tau^n - 1)/n * omega^j / (tau - omega^j);
    for tau in H it is 1 exactly at tau = omega^j."""
    from .ntt import root_of_unity
    w = pow(root_of_unity(n), j, R)
    if pow(tau, n, R) == 1:
        return 1 if tau % R == w else 0
    return (pow(tau, n, R) - 1) * pow(n, -1, R) % R * w % R * pow(tau - w, -1, R) % R


def lagrange_srs(tau: int, n: int):
    """[l_j(tau)]_1 for j < n (commitments to evaluation vectors on H)."""
    return [g1.gen_mul(lagrange_basis_at(tau, n, j)) for j in range(n)]
