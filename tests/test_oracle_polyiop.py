"""Pins for the oracle's Poly-IOP quotient Q = R(f(x), f(omega x)) / (X^n - 1).

Checked against what fixes it independently of the oracle's own steps:
* f(omega x) against Horner at omega z;
* the assembled constraint polynomial against R evaluated on scalar
  operands (Horner of each f_k at z and omega z);
* schoolbook multiplication back, Q (X^n - 1) + rem = R(...);
* divisibility exactly when the witnesses satisfy R on H, for BooleanCheck,
  Sub Check (the shift goes to omega x, not omega^-1 x), i-thIsZero and a
  running-product constraint z(omega x) = z(x) f(x) of degree 2;
* the identity Q(z) (z^n - 1) = R(f(z), f(omega z)) with the operands
  evaluated barycentrically from the witness vectors (no inverse transform);
* BooleanCheck on the two-point domain {1, -1} by hand: Q = -f_1^2;
* the degree bound deg Q <= d (n - 1) - n.
"""
from oracle import field, polyiop as op
from oracle.ntt import barycentric_eval, horner, root_of_unity

R = field.R


def _schoolbook(a, b):
    out = [0] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] = (out[i + j] + x * y) % R
    return out


def _boolean(rng, n):
    return [rng.randrange(2) for _ in range(n)]


def _sub_check_witness(rng, n):
    g = [rng.randrange(R) for _ in range(n)]
    d = [(g[(i + 1) % n] - g[i]) % R for i in range(n)]   # d = g(omega x) - g(x) on H
    return [g, d]


def _running_product_witness(rng, n):
    # z_(i+1) = z_i f_i cyclically, so the product of all f_i is 1
    f = [rng.randrange(1, R) for _ in range(n - 1)]
    prod = 1
    for v in f:
        prod = prod * v % R
    f.append(pow(prod, -1, R))
    z = [rng.randrange(1, R)]
    for i in range(n - 1):
        z.append(z[-1] * f[i] % R)
    return [z, f]


# z(omega x) - z(x) f(x): N = 2, x_1 = z, x_2 = f, x_3 = z(omega x)
RUNNING_PRODUCT = [(1, [2]), (R - 1, [0, 1])]


def test_shift_is_evaluation_at_omega_z(rng):
    for n in (1, 2, 8, 32):
        c = [rng.randrange(R) for _ in range(n)]
        z = rng.randrange(R)
        assert horner(op.shifted(c), z) == horner(c, root_of_unity(n) * z % R)


def test_constraint_poly_matches_scalar_evaluation(rng):
    n = 16
    w = root_of_unity(n)
    for terms, N in ((op.BOOLEAN_CHECK, 1), (op.SUB_CHECK, 2), (op.ITH_IS_ZERO, 2), (RUNNING_PRODUCT, 2),
                     ([(5, [0, 0, 1]), (7, [3]), (11, [])], 2)):
        polys = [[rng.randrange(R) for _ in range(n)] for _ in range(N)]
        p = op.constraint_poly(polys, terms)
        for _ in range(3):
            z = rng.randrange(R)
            vals = [horner(f, z) for f in polys] + [horner(f, w * z % R) for f in polys]
            assert horner(p, z) == op.constraint_at(vals, terms)


def test_quotient_multiplies_back(rng):
    n = 8
    for terms, N in ((op.BOOLEAN_CHECK, 1), (RUNNING_PRODUCT, 2), ([(3, [0, 1, 1])], 2)):
        vecs = [[rng.randrange(R) for _ in range(n)] for _ in range(N)]
        q, rem, polys = op.polyiop_quotient(vecs, terms)
        p = op.constraint_poly(polys, terms)
        back = _schoolbook(q, [R - 1] + [0] * (n - 1) + [1])
        back = back + [0] * max(0, len(p) - len(back))
        for i, r in enumerate(rem):
            back[i] = (back[i] + r) % R
        assert back[:len(p)] == p and not any(back[len(p):])


def test_divisible_exactly_when_satisfied(rng):
    for n in (2, 4, 16, 64):
        # BooleanCheck
        v = _boolean(rng, n)
        q, rem, _ = op.polyiop_quotient([v], op.BOOLEAN_CHECK)
        assert not any(rem)
        bad = list(v)
        bad[n // 2] = 2
        assert any(op.polyiop_quotient([bad], op.BOOLEAN_CHECK)[1])
        # Sub Check: the shifted operand is g(omega x); d built for the
        # backward shift g(omega^-1 x) does not divide (for n > 2, where
        # omega^-1 differs from omega)
        g, d = _sub_check_witness(rng, n)
        q, rem, _ = op.polyiop_quotient([g, d], op.SUB_CHECK)
        assert not any(rem) and not any(q)
        if n > 2:
            back = [(g[(i - 1) % n] - g[i]) % R for i in range(n)]
            assert any(op.polyiop_quotient([g, back], op.SUB_CHECK)[1])
        # i-thIsZero: L_i times d with d_i = 0
        i0 = rng.randrange(n)
        L = [1 if j == i0 else 0 for j in range(n)]
        d = [rng.randrange(R) for _ in range(n)]
        d[i0] = 0
        assert not any(op.polyiop_quotient([L, d], op.ITH_IS_ZERO)[1])
        d[i0] = 1
        assert any(op.polyiop_quotient([L, d], op.ITH_IS_ZERO)[1])
        # running product z(omega x) = z(x) f(x), cyclic
        z, f = _running_product_witness(rng, n)
        assert not any(op.polyiop_quotient([z, f], RUNNING_PRODUCT)[1])
        f2 = list(f)
        f2[0] = (f2[0] + 1) % R
        assert any(op.polyiop_quotient([z, f2], RUNNING_PRODUCT)[1])


def test_identity_at_random_points_barycentric(rng):
    n = 32
    w = root_of_unity(n)
    for terms, vecs in ((op.BOOLEAN_CHECK, [_boolean(rng, n)]), (RUNNING_PRODUCT, _running_product_witness(rng, n))):
        q, rem, _ = op.polyiop_quotient(vecs, terms)
        assert not any(rem)
        for _ in range(3):
            z = rng.randrange(R)
            vals = [barycentric_eval(v, z) for v in vecs] + [barycentric_eval(v, w * z % R) for v in vecs]
            assert horner(q, z) * (pow(z, n, R) - 1) % R == op.constraint_at(vals, terms)


def test_boolean_check_two_point_domain_by_hand(rng):
    # H = {1, -1}: f = (a0 + a1)/2 + (a0 - a1)/2 X; f - f^2 divided by X^2 - 1
    # leaves Q = -f_1^2 (the X^2 coefficient), for booleans with no remainder
    half = pow(2, -1, R)
    for a0, a1 in ((0, 0), (0, 1), (1, 0), (1, 1)):
        f1 = (a0 - a1) * half % R
        q, rem, _ = op.polyiop_quotient([[a0, a1]], op.BOOLEAN_CHECK)
        assert q == [(-f1 * f1) % R, 0]
        assert rem == [0, 0]


def test_degree_bound(rng):
    n = 64
    q, rem, _ = op.polyiop_quotient([_boolean(rng, n)], op.BOOLEAN_CHECK)
    assert len(q) == n and q[n - 1] == 0          # d = 2: deg Q <= n - 2
    cubic = [(1, [0, 0, 0]), (R - 1, [0])]         # f^3 - f vanishes on {0, 1, -1} values
    v = [rng.choice((0, 1, R - 1)) for _ in range(n)]
    q3, rem3, _ = op.polyiop_quotient([v], cubic)
    assert not any(rem3)
    assert len(q3) == 2 * n and not any(q3[2 * n - 2:])   # deg Q <= 3 (n - 1) - n = 2n - 3
