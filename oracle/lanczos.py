"""Skew-Lanczos process (paper Sec. 3.2, Fig. 2) and its start vector.

Start vector (reading: the paper leaves q_1 arbitrary): component i (0-based)
is the i-th output of the SplitMix64 generator (Steele, Lea, Flood 2014)
seeded with ``seed``: z = seed + (i+1)*0x9E3779B97F4A7C15 (mod 2^64), then
z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
z ^= z >> 31.  The top 53 bits give u in [0, 1) and q_i = 2u - 1.

Breakdown (reading): the process stops when alpha_1 == 0 or, for i >= 2, when
alpha_i <= 1e-14 * alpha_1; k_eff is the number of Lanczos vectors produced.
No reorthogonalisation (the paper reports it brings negligible benefit).
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)
DEFAULT_SEED = 0x2009069540
BREAKDOWN_REL = 1e-14


def splitmix64_raw(seed: int, n: int) -> np.ndarray:
    """SplitMix64 outputs 0..n-1 of the stream started at state ``seed``."""
    with np.errstate(over="ignore"):
        ctr = np.arange(1, n + 1, dtype=np.uint64) * GOLDEN
        z = ctr + np.uint64(seed & 0xFFFFFFFFFFFFFFFF)
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix64_uniform(seed: int, n: int) -> np.ndarray:
    """U[-1, 1) values: top 53 bits of each output, u = bits * 2^-53, 2u - 1."""
    z = splitmix64_raw(seed, n)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0


def start_vector(seed: int, n: int) -> np.ndarray:
    q = splitmix64_uniform(seed, n)
    return q / np.linalg.norm(q)


def skew_lanczos(J_apply, q1: np.ndarray, k: int):
    """k steps of Fig. 2 on a skew-symmetric operator.

    Returns (Q, alpha) with Q of shape (n, k_eff) and alpha of length k_eff-1,
    such that Q^T J Q = S_k with S_k[i, i+1] = alpha_i, S_k[i+1, i] = -alpha_i.
    """
    n = q1.size
    if k <= 0:
        return np.zeros((n, 0)), np.zeros(0)
    q = q1 / np.linalg.norm(q1)
    Q = [q]
    alpha = []
    if k == 1:
        return np.stack(Q, axis=1), np.zeros(0)
    z = J_apply(Q[0])
    a1 = np.linalg.norm(z)
    if a1 == 0.0:
        return np.stack(Q, axis=1), np.zeros(0)
    alpha.append(a1)
    Q.append(-z / a1)
    for i in range(2, k):                    # paper's i = 2 .. k-1 (1-based)
        z = J_apply(Q[i - 1]) - alpha[i - 2] * Q[i - 2]
        ai = np.linalg.norm(z)
        if ai <= BREAKDOWN_REL * a1:
            break
        alpha.append(ai)
        Q.append(-z / ai)
    return np.stack(Q, axis=1), np.asarray(alpha)


def skew_tridiagonal(alpha: np.ndarray) -> np.ndarray:
    """Dense S_k from alpha (superdiagonal +alpha, subdiagonal -alpha)."""
    k = alpha.size + 1
    S = np.zeros((k, k))
    for i, a in enumerate(alpha):
        S[i, i + 1] = a
        S[i + 1, i] = -a
    return S
