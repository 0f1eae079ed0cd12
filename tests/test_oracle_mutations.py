"""Planted mistakes in the oracle (on the CPU) must be caught by its pins.

Each case patches one plausible slip into an oracle function -- a swapped
sign, a dropped special case, a transposed operand, an off-by-one index --
and re-runs the pin that is meant to catch it, expecting it to fail.
"""
import random

import pytest

from oracle import field, fold, g1, g2, kzg, msm, ntt, quotient, srs
from tests import test_oracle_g1 as tg
from tests import test_oracle_kzg as tk
from tests import test_oracle_quotient as tq
from tests import test_oracle_accum as ta
from tests import test_oracle_g2 as tg2
from tests import test_oracle_msm_fold as tm
from tests import test_oracle_ntt as tn

R = field.R


def _fails(fn, *args):
    with pytest.raises(AssertionError):
        fn(*args)


def test_swapped_butterfly_sign_is_caught(monkeypatch):
    def bad_fft(a, w):
        n = len(a)
        if n == 1:
            return [a[0] % R]
        even, odd = bad_fft(a[0::2], w * w % R), bad_fft(a[1::2], w * w % R)
        out, t, h = [0] * n, 1, n // 2
        for j in range(h):
            v = odd[j] * t % R
            out[j], out[j + h] = (even[j] - v) % R, (even[j] + v) % R
            t = t * w % R
        return out
    monkeypatch.setattr(ntt, "_fft", bad_fft)
    _fails(tn.test_fft_equals_dft_and_inverse, random.Random(1), 3)


def test_wrong_root_is_caught(monkeypatch):
    good = ntt.root_of_unity
    monkeypatch.setattr(ntt, "root_of_unity", lambda n: good(n) * good(n) % R)
    _fails(tn.test_root_of_unity_is_primitive, 5)


def test_dropped_coset_shift_is_caught(monkeypatch):
    good = ntt.coset_evals
    monkeypatch.setattr(ntt, "coset_evals", lambda c, lb, s=5: good(c, lb, 1))
    _fails(tn.test_coset_equals_interleaved_small_transforms, random.Random(2))


def test_missing_doubling_case_is_caught(monkeypatch):
    def bad_add(p1, p2):
        if p1 is None:
            return p2
        if p2 is None:
            return p1
        if p1[0] == p2[0]:
            return None
        lam = (p2[1] - p1[1]) * pow(p2[0] - p1[0], -1, field.P) % field.P
        x3 = (lam * lam - p1[0] - p2[0]) % field.P
        return (x3, (lam * (p1[0] - x3) - p1[1]) % field.P)
    monkeypatch.setattr(g1, "add", bad_add)
    _fails(tg.test_special_cases)


def test_fold_operands_transposed_is_caught(monkeypatch):
    monkeypatch.setattr(fold, "fold_pair",
                        lambda gam, a, b: [g1.add(x, g1.mul(gam % R, y)) for x, y in zip(a, b)])
    _fails(tm.test_extractor_identity, random.Random(3))


def test_srs_index_shift_is_caught(monkeypatch):
    monkeypatch.setattr(msm, "srs_msm_closed_form",
                        lambda tau, s: g1.gen_mul(sum(int(c) * pow(tau, i + 1, R) for i, c in enumerate(s))))
    _fails(tm.test_naive_msm_equals_closed_form_on_srs, random.Random(4))


def test_dropped_flat_coefficient_is_caught(monkeypatch):
    good = fold.flat_coefficients

    def bad(m, gam):
        s = good(m, gam)
        s[0] = 1
        return s
    monkeypatch.setattr(fold, "flat_coefficients", bad)
    _fails(tm.test_tree_equals_flat_on_points, random.Random(5), 5)


def test_barycentric_missing_scale_is_caught(monkeypatch):
    good = ntt.barycentric_eval
    monkeypatch.setattr(ntt, "barycentric_eval", lambda v, x: good(v, x) * len(v) % R)
    _fails(tn.test_barycentric_matches_interpolation, random.Random(6))


def test_srs_generator_off_by_one_is_caught(monkeypatch):
    monkeypatch.setattr(srs, "srs", lambda tau, n: [g1.gen_mul(pow(tau, i + 1, R)) for i in range(n)])
    _fails(tm.test_srs_points, random.Random(7))


def test_synthetic_division_sign_is_caught(monkeypatch):
    def bad(coeffs, x):
        f = [int(c) % R for c in coeffs]
        if not f:
            return [], 0
        q, carry = [0] * (len(f) - 1), f[-1]
        for i in range(len(f) - 2, -1, -1):
            q[i] = carry
            carry = (f[i] - x * carry) % R
        return q, carry
    monkeypatch.setattr(kzg, "divide_by_linear", bad)
    _fails(tk.test_division_multiplies_back, random.Random(8))


def test_quotient_index_shift_is_caught(monkeypatch):
    def bad(coeffs, x):
        f = [int(c) % R for c in coeffs]
        if not f:
            return [], 0
        q, carry = [0] * (len(f) - 1), f[-1]
        for i in range(len(f) - 2, -1, -1):
            carry = (f[i] + x * carry) % R
            q[i] = carry
        return q, carry
    monkeypatch.setattr(kzg, "divide_by_linear", bad)
    _fails(tk.test_hand_worked_example)


def test_batch_gamma_power_shift_is_caught(monkeypatch):
    good = kzg.batch_open_at

    def bad(polys, x, gamma):
        ys, h = good(polys, x, gamma)
        return ys, [c * gamma % R for c in h]  # gamma^(i+1) instead of gamma^i
    monkeypatch.setattr(kzg, "batch_open_at", bad)
    _fails(tk.test_batch_is_gamma_combination_of_single_quotients, random.Random(10))


def test_verifier_sign_slip_is_caught(monkeypatch):
    monkeypatch.setattr(kzg, "verify_with_trapdoor",
                        lambda tau, com, x, y, pi: g1.add(com, g1.gen_mul(y % R)) == g1.mul((tau - x) % R, pi))
    _fails(tk.test_verifier_equation_with_trapdoor, random.Random(11))


def test_vanishing_division_sign_is_caught(monkeypatch):
    def bad(p, n):
        work = [int(c) % R for c in p]
        if len(work) <= n:
            return [], work + [0] * (n - len(work))
        t = [0] * (len(work) - n)
        for i in range(len(work) - 1, n - 1, -1):
            c = work[i]
            t[i - n] = (t[i - n] + c) % R
            work[i - n] = (work[i - n] - c) % R
            work[i] = 0
        return t, work[:n]
    monkeypatch.setattr(quotient, "divide_by_vanishing", bad)
    _fails(tq.test_division_multiplies_back, random.Random(12))


def test_cyclic_product_is_caught(monkeypatch):
    def bad(f, h):
        size = max(len(f), len(h))
        F = ntt.fft(list(f) + [0] * (size - len(f)))
        H = ntt.fft(list(h) + [0] * (size - len(h)))
        return ntt.ifft([x * y % R for x, y in zip(F, H)]) + [0] * (len(f) + len(h) - 1 - size)
    monkeypatch.setattr(quotient, "poly_mul_fft", bad)
    _fails(tq.test_two_point_domain_by_hand, random.Random(13))


def test_error_fold_roles_swapped_is_caught(monkeypatch):
    good = fold.fold_errors_g1
    monkeypatch.setattr(fold, "fold_errors_g1", lambda gam, E, E2, Ej: good(gam, E2, E, Ej))
    _fails(ta.test_two_term_case, random.Random(14))


def test_fr_fold_operands_swapped_is_caught(monkeypatch):
    monkeypatch.setattr(fold, "fold_fr", lambda gam, v, v2: [(gam * b + a) % R for a, b in zip(v, v2)])
    _fails(ta.test_commitment_homomorphism, random.Random(15))


def test_error_power_off_by_one_is_caught(monkeypatch):
    def bad(gam, e, e2, ej):
        vecs = [e2] + list(ej) + [e]
        return [sum(pow(gam, j + (j > 0), R) * int(v[i]) for j, v in enumerate(vecs)) % R for i in range(len(e))]
    monkeypatch.setattr(fold, "fold_errors_fr", bad)
    _fails(ta.test_error_polynomial_extraction, random.Random(16))


def test_fq2_sign_of_u_squared_is_caught(monkeypatch):
    monkeypatch.setattr(g2, "f2_mul", lambda a, b: ((a[0] * b[0] + a[1] * b[1]) % field.P,
                                                    (a[0] * b[1] + a[1] * b[0]) % field.P))
    _fails(tg2.test_fq2_definition, random.Random(17))


def test_g2_doubling_slip_is_caught(monkeypatch):
    good = g2.double

    def bad(pt):
        r = good(pt)
        return None if r is None else (r[0], g2.f2_neg(r[1]))
    monkeypatch.setattr(g2, "double", bad)
    _fails(tg2.test_generator_order_r)


def _runs_at_variant(geo_extra=0, start_extra=0, replace=True, one_len_extra=0):
    """sum_runs_at with one planted slip (geometric length, start exponent,
    point added instead of replacing its run's value, or the x = 1 case)."""
    def f(runs, points, x):
        x %= R
        acc = 0
        for start, length, v in runs:
            if x == 1:
                g = (length + one_len_extra) % R
            else:
                g = (pow(x, length + geo_extra, R) - 1) * field.fr_inv(x - 1) % R
            acc = (acc + int(v) * pow(x, start + start_extra, R) % R * g) % R
        for i, v in points.items():
            base = 0
            if replace:
                for start, length, rv in runs:
                    if start <= i < start + length:
                        base = int(rv)
                        break
            acc = (acc + (int(v) - base) * pow(x, i, R)) % R
        return acc
    return f


@pytest.mark.parametrize("slip", [dict(geo_extra=1), dict(start_extra=1), dict(replace=False),
                                  dict(one_len_extra=-1)])
def test_run_structured_slips_are_caught(monkeypatch, slip):
    monkeypatch.setattr(ntt, "sum_runs_at", _runs_at_variant(**slip))
    _fails(tn.test_run_structured_outputs_match_dense_transforms, random.Random(3), 6)


def test_run_structured_missing_inverse_scale_is_caught(monkeypatch):
    def bad(runs, points, log_domain, k, inverse=False, shift=1):
        w = ntt.root_of_unity(1 << log_domain)
        base = pow(field.fr_inv(w), k, R) if inverse else shift * pow(w, k, R) % R
        return ntt.sum_runs_at(runs, points, base)
    monkeypatch.setattr(ntt, "ntt_runs_at", bad)
    _fails(tn.test_run_structured_outputs_match_dense_transforms, random.Random(4), 6)


def test_polyiop_backward_shift_is_caught(monkeypatch):
    from oracle import polyiop
    from tests import test_oracle_polyiop as tp

    def bad_shifted(coeffs):
        n = len(coeffs)
        w = field.fr_inv(ntt.root_of_unity(n))
        return [int(c) * pow(w, i, R) % R for i, c in enumerate(coeffs)]
    monkeypatch.setattr(polyiop, "shifted", bad_shifted)
    _fails(tp.test_divisible_exactly_when_satisfied, random.Random(11))


def test_polyiop_dropped_term_is_caught(monkeypatch):
    from oracle import polyiop
    from tests import test_oracle_polyiop as tp
    good = polyiop.constraint_poly
    monkeypatch.setattr(polyiop, "constraint_poly", lambda polys, terms: good(polys, terms[:-1]))
    _fails(tp.test_constraint_poly_matches_scalar_evaluation, random.Random(12))


def test_polyiop_quotient_cut_to_n_is_caught(monkeypatch):
    from oracle import polyiop
    from tests import test_oracle_polyiop as tp
    good = polyiop.polyiop_quotient

    def cut(vectors, terms):
        q, rem, polys = good(vectors, terms)
        return q[:len(vectors[0])], rem, polys
    monkeypatch.setattr(polyiop, "polyiop_quotient", cut)
    _fails(tp.test_degree_bound, random.Random(13))
