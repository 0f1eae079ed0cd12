"""Pins for the oracle's transforms over Fr (evaluations on H, Foldable basic blocks;
coset evaluation for the X^n - 1 quotients of Mul and the Poly-IOP)."""
import pytest

from oracle import field, ntt

R = field.R


def _vec(rng, n):
    return [rng.randrange(R) for _ in range(n)]


@pytest.mark.parametrize("logn", [0, 1, 2, 5, 10, 28])
def test_root_of_unity_is_primitive(logn):
    n = 1 << logn
    w = ntt.root_of_unity(n)
    assert pow(w, n, R) == 1
    if n > 1:
        assert pow(w, n // 2, R) == R - 1


def test_root_bad_sizes():
    for n in (0, 3, 6, 1 << 29):
        with pytest.raises(ValueError):
            ntt.root_of_unity(n)


@pytest.mark.parametrize("logn", [0, 1, 2, 3, 6, 10])
def test_fft_equals_dft_and_inverse(rng, logn):
    n = 1 << logn
    a = _vec(rng, n)
    A = ntt.dft(a)
    assert ntt.fft(a) == A
    assert ntt.idft(A) == a
    assert ntt.ifft(A) == a


def test_sum_over_domain_is_n_times_constant_term(rng):
    # Sum protocol: sum_{x in H} f(x) = n * f(0)
    for logn in (3, 8, 12):
        n = 1 << logn
        a = _vec(rng, n)
        assert sum(ntt.fft(a)) % R == n * a[0] % R


def test_delta_and_constant(rng):
    n = 64
    delta = [1] + [0] * (n - 1)
    assert ntt.fft(delta) == [1] * n
    c = rng.randrange(R)
    assert ntt.fft([c] + [0] * (n - 1)) == [c] * n
    assert ntt.fft([c] * n) == [n * c % R] + [0] * (n - 1)


def test_monomial_maps_to_powers():
    n = 32
    w = ntt.root_of_unity(n)
    for k in (1, 5, 31):
        e = [0] * n
        e[k] = 1
        assert ntt.fft(e) == [pow(w, k * j, R) for j in range(n)]


def test_convolution_theorem(rng):
    n = 32
    a, b = _vec(rng, n), _vec(rng, n)
    cyc = [0] * n
    for i in range(n):
        for j in range(n):
            cyc[(i + j) % n] = (cyc[(i + j) % n] + a[i] * b[j]) % R
    A, B = ntt.fft(a), ntt.fft(b)
    assert ntt.fft(cyc) == [x * y % R for x, y in zip(A, B)]


def test_fft_4096_roundtrip_and_samples(rng):
    n = 1 << 12
    a = _vec(rng, n)
    A = ntt.fft(a)
    assert ntt.ifft(A) == a
    w = ntt.root_of_unity(n)
    for j in (0, 1, 7, 2048, 4095):
        assert A[j] == ntt.horner(a, pow(w, j, R))


def test_coset_equals_interleaved_small_transforms(rng):
    # f(g w_4n^(4m + k)) = sum_i (a_i (g w_4n^k)^i) w_n^(mi): four size-n transforms
    n, logb, g = 16, 2, 5
    a = _vec(rng, n)
    E = ntt.coset_evals(a, logb, g)
    assert len(E) == 4 * n
    w4 = ntt.root_of_unity(4 * n)
    for k in range(4):
        base = g * pow(w4, k, R) % R
        sub = ntt.fft([a[i] * pow(base, i, R) % R for i in range(n)])
        assert E[k::4] == sub
    for j in (0, 3, 33, 63):
        assert E[j] == ntt.coset_eval_at(a, logb, j, g)


def test_coset_trivial_cases(rng):
    a = _vec(rng, 8)
    assert ntt.coset_evals(a, 0, 1) == ntt.fft(a)
    # the coset misses the domain: f(g w^j) never hits an element of H_4n when g = 5
    w = ntt.root_of_unity(32)
    H = {pow(w, j, R) for j in range(32)}
    assert all(5 * pow(w, j, R) % R not in H for j in range(32))


def test_barycentric_matches_interpolation(rng):
    for logn in (0, 1, 3, 6):
        n = 1 << logn
        v = _vec(rng, n)
        x = rng.randrange(R)
        assert ntt.barycentric_eval(v, x) == ntt.horner(ntt.ifft(v), x)


def test_lagrange_basis_pins(rng):
    from oracle import srs as osrs
    n = 16
    w = ntt.root_of_unity(n)
    tau = rng.randrange(R)
    lj = [osrs.lagrange_basis_at(tau, n, j) for j in range(n)]
    # partition of unity, and the basis reproduces every monomial X^k, k < n
    assert sum(lj) % R == 1
    for k in (1, 5, n - 1):
        assert sum(l * pow(w, j * k, R) for j, l in enumerate(lj)) % R == pow(tau, k, R)
    # l_j is the interpolant of the j-th unit vector (inverse transform, Horner)
    for j in (0, 3):
        e = [0] * n
        e[j] = 1
        assert lj[j] == ntt.horner(ntt.idft(e), tau)
    # tau on H: the basis is a unit vector
    assert [osrs.lagrange_basis_at(pow(w, 5, R), n, j) for j in range(n)] == [int(j == 5) for j in range(n)]


def _runs_vector(rng, n, nruns, npoints):
    """A random run-structured vector (with gaps) and its dense form."""
    cuts = sorted(rng.sample(range(1, n), min(2 * nruns, n - 1)))
    edges = [0] + cuts + [n]
    runs, dense = [], [0] * n
    for t in range(len(edges) - 1):
        if t % 3 == 2:  # a gap of zeros
            continue
        s, e = edges[t], edges[t + 1]
        v = rng.randrange(R)
        runs.append((s, e - s, v))
        dense[s:e] = [v] * (e - s)
    points = {}
    for i in rng.sample(range(n), min(npoints, n)):
        points[i] = rng.randrange(R)
        dense[i] = points[i]
    return runs, points, dense


@pytest.mark.parametrize("logn", [0, 1, 3, 6, 9])
def test_run_structured_outputs_match_dense_transforms(rng, logn):
    # the geometric-sum shortcut against the O(n^2) definitions
    n = 1 << logn
    runs, points, dense = _runs_vector(rng, n, 5, 4)
    A, a = ntt.dft(dense), ntt.idft(dense)
    for k in range(n):
        assert ntt.ntt_runs_at(runs, points, logn, k) == A[k]
        assert ntt.ntt_runs_at(runs, points, logn, k, inverse=True) == a[k]


@pytest.mark.parametrize("logn,lb", [(0, 2), (3, 1), (5, 2), (6, 3)])
def test_run_structured_coset_outputs(rng, logn, lb):
    n = 1 << logn
    runs, points, dense = _runs_vector(rng, n, 3, 3)
    E = ntt.coset_evals(dense, lb)
    for k in range(n << lb):
        assert ntt.ntt_runs_at(runs, points, logn + lb, k, shift=field.GENERATOR_FR) == E[k]


def test_run_structured_edge_cases(rng):
    # one run over everything: a constant vector transforms to n*c at 0 and 0 elsewhere
    c = rng.randrange(R)
    for k in range(16):
        assert ntt.ntt_runs_at([(0, 16, c)], {}, 4, k) == (16 * c % R if k == 0 else 0)
    # only points: a delta at i gives omega^(ik)
    w = ntt.root_of_unity(1 << 20)
    for k in (0, 1, 12345, (1 << 20) - 1):
        assert ntt.ntt_runs_at([], {777: 1}, 20, k) == pow(w, 777 * k, R)
    # a point inside a run replaces the run's value rather than adding to it
    assert ntt.sum_runs_at([(0, 4, 5)], {2: 5}, 3) == 5 * (1 + 3 + 9 + 27) % R
