"""Number-theoretic transforms over Fr (test oracle only).

Foldable basic blocks: a length-n vector is the evaluations of a polynomial f
on H = {omega^i : i in [n]} with omega^n = 1, element i being f(omega^i).
The forward transform takes coefficients a to evaluations A_j = f(omega^j) =
sum_i a_i omega^(ij); the inverse takes evaluations to coefficients,
a_i = n^(-1) sum_j A_j omega^(-ij).

Quotients by the vanishing polynomial X^n - 1 (Mul; Poly-IOP) need f outside H;
``coset_evals`` gives f on the coset g * H_(Bn) of a B-times larger domain.

Root of unity convention: omega_n = 5^((r-1)/n) (5 is a non-residue mod r).
"""
from .field import R, GENERATOR_FR, TWO_ADICITY, fr_inv


def root_of_unity(n: int) -> int:
    """A primitive n-th root of unity, n a power of two <= 2^28."""
    if n < 1 or n & (n - 1) or n > (1 << TWO_ADICITY):
        raise ValueError("n must be a power of two <= 2^28")
    return pow(GENERATOR_FR, (R - 1) // n, R)


def horner(coeffs, x: int) -> int:
    """f(x) = sum_i coeffs[i] x^i."""
    acc = 0
    for c in reversed(list(coeffs)):
        acc = (acc * x + int(c)) % R
    return acc


def dft(a):
    """O(n^2) definition: A_j = sum_i a_i omega^(ij)."""
    n = len(a)
    w = root_of_unity(n)
    out = []
    wj = 1
    for _ in range(n):
        out.append(horner(a, wj))
        wj = wj * w % R
    return out


def idft(A):
    """O(n^2) definition: a_i = n^(-1) sum_j A_j omega^(-ij)."""
    n = len(A)
    winv = fr_inv(root_of_unity(n))
    ninv = fr_inv(n)
    out = []
    wi = 1
    for _ in range(n):
        out.append(horner(A, wi) * ninv % R)
        wi = wi * winv % R
    return out


def _fft(a, w):
    n = len(a)
    if n == 1:
        return [a[0] % R]
    even = _fft(a[0::2], w * w % R)
    odd = _fft(a[1::2], w * w % R)
    out = [0] * n
    t = 1
    half = n // 2
    for j in range(half):
        u = even[j]
        v = odd[j] * t % R
        out[j] = (u + v) % R
        out[j + half] = (u - v) % R
        t = t * w % R
    return out


def fft(a):
    """Plain recursive radix-2 transform (same result as ``dft``)."""
    a = [int(x) % R for x in a]
    return _fft(a, root_of_unity(len(a)))


def ifft(A):
    """Inverse of ``fft`` (same result as ``idft``)."""
    n = len(A)
    out = _fft([int(x) % R for x in A], fr_inv(root_of_unity(n)))
    ninv = fr_inv(n)
    return [x * ninv % R for x in out]


def coset_evals(coeffs, log_blowup: int, shift: int = GENERATOR_FR):
    """E_j = f(shift * omega_(Bn)^j), j < Bn, B = 2^log_blowup: the transform of
    (a_i shift^i) zero-padded to length Bn."""
    n = len(coeffs)
    big = n << log_blowup
    scaled = []
    gi = 1
    for c in coeffs:
        scaled.append(int(c) * gi % R)
        gi = gi * shift % R
    scaled += [0] * (big - n)
    return fft(scaled)


def coset_eval_at(coeffs, log_blowup: int, j: int, shift: int = GENERATOR_FR) -> int:
    """One output of ``coset_evals`` by Horner: f(shift * omega_(Bn)^j)."""
    big = len(coeffs) << log_blowup
    x = shift * pow(root_of_unity(big), j, R) % R
    return horner(coeffs, x)


def barycentric_eval(evals, x: int) -> int:
    """f(x) straight from f's evaluations on H, for x not in H:
    f(x) = (x^n - 1)/n * sum_j v_j omega^j / (x - omega^j)."""
    n = len(evals)
    w = root_of_unity(n)
    acc = 0
    wj = 1
    for v in evals:
        acc = (acc + int(v) * wj * fr_inv(x - wj)) % R
        wj = wj * w % R
    return (pow(x, n, R) - 1) * fr_inv(n) % R * acc % R


def sum_runs_at(runs, points, x: int) -> int:
    """f(x) = sum_i v_i x^i for a vector given as constant runs plus single
    values: ``runs`` lists (start, length, value) over disjoint index ranges,
    ``points`` maps an index to the value that replaces its run's value there
    (indices outside every run hold 0 unless listed).  A run contributes
    value * x^start * (x^length - 1) / (x - 1), or value * length at x = 1
    (the geometric sum); each point then adds (v - run value) x^i.  This is the
    definition of one transform output (x = shift * omega^j, or omega^(-i) for
    the inverse) evaluated in O(#runs + #points) operations, which makes single
    outputs of transforms of up to 2^28 points checkable."""
    x %= R
    acc = 0
    for start, length, v in runs:
        if x == 1:
            g = length % R
        else:
            g = (pow(x, length, R) - 1) * fr_inv(x - 1) % R
        acc = (acc + int(v) * pow(x, start, R) % R * g) % R
    for i, v in points.items():
        base = 0
        for start, length, rv in runs:
            if start <= i < start + length:
                base = int(rv)
                break
        acc = (acc + (int(v) - base) * pow(x, i, R)) % R
    return acc


def ntt_runs_at(runs, points, log_domain: int, k: int, inverse: bool = False, shift: int = 1) -> int:
    """Output k of the forward (shift = 1), coset (shift = g) or inverse
    transform on the domain of N = 2^log_domain points of a run-structured
    vector (``sum_runs_at``; a coset input has fewer than N coefficients and is
    zero-padded): forward/coset sum_i v_i (g w^k)^i, inverse
    N^(-1) sum_i v_i w^(-ik), w = omega_N."""
    w = root_of_unity(1 << log_domain)
    if inverse:
        return sum_runs_at(runs, points, pow(fr_inv(w), k, R)) * fr_inv(1 << log_domain) % R
    return sum_runs_at(runs, points, shift * pow(w, k, R) % R)
