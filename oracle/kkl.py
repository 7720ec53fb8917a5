"""The KKLLL permanent estimator (Section 2.3, Algorithm KKLLL) in float64 (oracle).

TEST INFRASTRUCTURE ONLY.

Algorithm KKLLL, for a 0-1 matrix A: B_ij = 0 where A_ij = 0; elsewhere B_ij is one of the
three cube roots of unity w0 = 1, w1, w2, each with probability 1/3, independently; the
estimate is X_A = det(B) * conj(det(B)) = |det B|^2. Its expectation is per(A) (the theorem
stated after the algorithm). The paper applies it to the 0-1 pattern of each sub-matrix
(Section 3: the time for per(A) and for per(B), B the pattern of A, are almost equal) and
orders jobs by the approximate permanents (the improved Step 3 of Algorithm PH), using
about n^2 trials per matrix (the footnotes to the C100, C60 and dwt_66 timing tables).

Random draws: exponents u_ij in {0, 1, 2} come from a counter-based SplitMix64 generator
(Steele, Lea and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
the k-th output (k = 0, 1, ...) of the stream seeded with ``seed`` is
mix(seed + (k + 1) * 0x9E3779B97F4A7C15 mod 2^64), where
mix(z) = z3 with z1 = (z ^ z>>30) * 0xBF58476D1CE4E5B9, z2 = (z1 ^ z1>>27) * 0x94D049BB133111EB,
z3 = z2 ^ z2>>31 (all mod 2^64). The counter of entry (i, j) of trial t of job w is
k = (w << 36) | (t << 12) | (i << 6) | j  (so w < 2^28, t < 2^24, i, j < 64), and the
exponent is u = floor(3 * (x >> 32) / 2^32) for the output x.
"""
from __future__ import annotations

import math

import numpy as np

_M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, k: int) -> int:
    """k-th output (0-based) of the SplitMix64 stream seeded with ``seed``."""
    z = (seed + (k + 1) * GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def kkl_counter(job: int, trial: int, i: int, j: int) -> int:
    if not (0 <= job < 1 << 28 and 0 <= trial < 1 << 24 and 0 <= i < 64 and 0 <= j < 64):
        raise ValueError("counter field out of range")
    return (job << 36) | (trial << 12) | (i << 6) | j


def kkl_exponent(seed: int, job: int, trial: int, i: int, j: int) -> int:
    """Cube-root exponent u_ij in {0, 1, 2} of entry (i, j) for (job, trial)."""
    x = splitmix64(seed, kkl_counter(job, trial, i, j))
    return ((x >> 32) * 3) >> 32


def kkl_trial(A, u) -> float:
    """One KKLLL trial X = |det B|^2 (float64) with B_ij = w^{u_ij} on the nonzero pattern of A."""
    A = np.asarray(A)
    u = np.asarray(u)
    w = np.exp(2j * np.pi * u / 3.0)
    B = np.where(A != 0, w, 0.0).astype(np.complex128)
    d = np.linalg.det(B) if B.shape[0] else 1.0 + 0j
    return float((d * np.conj(d)).real)


def kkl_exponents(A, seed: int, job: int, trial: int) -> np.ndarray:
    n = np.asarray(A).shape[0]
    return np.array([[kkl_exponent(seed, job, trial, i, j) for j in range(n)] for i in range(n)],
                    dtype=np.int64)


def kkl_key(A, trials: int, seed: int, job: int) -> float:
    """log of the mean of ``trials`` KKLLL trials of the pattern of A (natural log; -inf if all 0)."""
    xs = [kkl_trial(A, kkl_exponents(A, seed, job, t)) for t in range(trials)]
    mean = sum(xs) / trials
    return math.log(mean) if mean > 0 else float("-inf")
