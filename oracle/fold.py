"""Random-linear-combination fold of G1 commitments (test oracle only).

Parallel Accumulation, accumulation prover step 5: from two instances v, v'
and the challenge gamma the prover forms v'' = gamma * v + v'; for the G1 part
of an instance that is C''_i = gamma * C_i + C'_i for every commitment i.  The
paper runs these pairwise folds as a tree, folding the instances of each level
in parallel.

Tree schedule used here (the paper leaves it open): at every level, adjacent
instances (2j, 2j+1) fold as gamma * left + right; an odd last instance is
carried to the next level unchanged; challenges are consumed in breadth-first
order (level by level, left to right).

Because every fold is linear, the tree's result is also the flat sum
sum_i sigma_i C_i, where sigma_i is the product of the challenges of the folds
in which instance i's running value was the left operand.  ``flat_fold`` forms
that sum directly; the two must agree.
"""
from . import g1
from .field import R


def fold_pair(gamma: int, left, right):
    """gamma * left + right, componentwise over a list of points."""
    return [g1.add(g1.mul(gamma % R, a), b) for a, b in zip(left, right)]


def tree_fold(instances, gammas):
    """Fold m instances (each a list of k points) to one with m - 1 challenges."""
    level = [list(inst) for inst in instances]
    if not level:
        raise ValueError("need at least one instance")
    if len(gammas) != len(level) - 1:
        raise ValueError("expected %d challenges, got %d" % (len(level) - 1, len(gammas)))
    gi = 0
    while len(level) > 1:
        nxt = []
        for j in range(0, len(level) - 1, 2):
            nxt.append(fold_pair(gammas[gi], level[j], level[j + 1]))
            gi += 1
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return level[0]


def flat_coefficients(m: int, gammas):
    """sigma_i for the tree schedule above: walk the same tree on scalars."""
    level = [[i] for i in range(m)]
    sig = [1] * m
    gi = 0
    while len(level) > 1:
        nxt = []
        for j in range(0, len(level) - 1, 2):
            for i in level[j]:
                sig[i] = sig[i] * gammas[gi] % R
            nxt.append(level[j] + level[j + 1])
            gi += 1
        if len(level) % 2:
            nxt.append(level[-1])
        level = nxt
    return sig


def flat_fold(instances, gammas):
    """sum_i sigma_i * instances[i], componentwise."""
    m = len(instances)
    k = len(instances[0])
    sig = flat_coefficients(m, gammas)
    out = []
    for c in range(k):
        acc = None
        for i in range(m):
            acc = g1.add(acc, g1.mul(sig[i], instances[i][c]))
        out.append(acc)
    return out


def fold_errors_g1(gamma: int, E, E2, Ej):
    """E'' = E' + sum_(j=1)^(d-1) gamma^j E_j + gamma^d E (prover step 5),
    d = len(Ej) + 1: the committed error polynomial evaluated at gamma."""
    terms = [E2] + list(Ej) + [E]
    acc = None
    for j, pt in enumerate(terms):
        acc = g1.add(acc, g1.mul(pow(gamma, j, R), pt))
    return acc


def fold_errors_fr(gamma: int, e, e2, ej):
    """e'' = e' + sum_j gamma^j e_j + gamma^d e, elementwise over Fr vectors."""
    vecs = [e2] + list(ej) + [e]
    return [sum(pow(gamma, j, R) * int(v[i]) for j, v in enumerate(vecs)) % R for i in range(len(e))]


def fold_fr(gamma: int, v, v2):
    """v'' = gamma v + v' over the Fr parts (mu, pi, r_i, m_i)."""
    return [(gamma * int(a) + int(b)) % R for a, b in zip(v, v2)]


def acc_fold(gamma: int, C, C2, E, E2, Ej, v, v2, e, e2, ej):
    """One accumulation step on two accumulators (C, E, v, e) and
    (C2, E2, v2, e2): (C'', E'', v'', e'')."""
    return (fold_pair(gamma, C, C2), fold_errors_g1(gamma, E, E2, Ej), fold_fr(gamma, v, v2),
            fold_errors_fr(gamma, e, e2, ej))
