"""CPU oracle for the KZG commit / accumulation-fold hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously-correct
Python big-integer statement of what the GPU library computes.  Only the test
suite, the package smoke check and the CPU-baseline leg of the benchmark may
import it; the product path never does, and it shares no code with the HIP
kernels or their host library.

Modules and what they follow (section names refer to the ZKTorch paper,
"Compiling ML Inference to Zero-Knowledge Proofs via Parallel Proof
Accumulation"):

* ``field`` -- BN254 prime fields Fq (coordinates) and Fr (scalars); the paper
  fixes BN254 (Experimental Setup) and writes p for the group order
  (Preliminaries), which this code calls r.
* ``g1``    -- affine short-Weierstrass group G1, [x]_1 = xG (Preliminaries).
* ``g2``    -- G2 over Fq2 (the sextic twist), [x]_2 = x H, its MSM and SRS
  (commitments in G2 of MulScalar, Mul and MatMul).
* ``msm``   -- KZG commit com = [f(tau)]_1 = sum_i f_i [tau^i]_1 as a naive sum of
  scalar multiples, and its closed form (Polynomial Commitment).
* ``ntt``   -- evaluations on H = {omega^i} (Foldable basic blocks), O(n^2) DFT,
  plain recursive FFT, coset evaluation for the X^n - 1 quotients (Mul,
  Poly-IOP), barycentric commit-from-evaluations.
* ``fold``  -- the random linear combination gamma*v + v' of the accumulation
  prover (Parallel Accumulation, prover step 5) and its tree schedule, and
  the full step: E'' = E' + sum_j gamma^j E_j + gamma^d E, the Fr parts and
  the error vectors.
* ``transcript`` -- the challenge hash (the paper's random oracles, read as
  SHA-256 to the field).
* ``srs``   -- [tau^i]_1 for a known test trapdoor (Polynomial Commitment: srs).
* ``kzg``   -- opening y = f(x), q = (f - y)/(X - x), pi = [q(tau)]_1, and the
  batched opening at one point with challenge powers gamma^i (Polynomial
  Commitment: open, batching), plus the verifier equation with tau known.
* ``quotient`` -- the Mul block's quotient t = (f h - g) / (X^n - 1) from the
  witness vectors, by transform-based product and long division (Mul).
* ``polyiop`` -- the quotient Q of a Poly-IOP constraint,
  R(f_1(x), .., f_N(x), f_1(omega x), .., f_N(omega x)) = Q(x) (x^n - 1), for
  R given as a sum of monomial terms (Basic blocks based on a Poly-IOP:
  BooleanCheck, Sub Check, i-thIsZero).

Every function here is pinned by a CPU test against something other than
itself (closed forms, invariants, brute force); see ``tests/test_oracle_*``.
"""
