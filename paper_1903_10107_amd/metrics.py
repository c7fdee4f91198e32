"""Reconciliation metrics: frame error rate with a Wilson interval, efficiency
f = (1 - R_eff) / h(QBER) and corrected-key throughput.

The paper reports throughput in Mbps and efficiency f (abstract, Table 2) but
defines neither; the readings here are: corrected-key bits are the key bits of
frames whose decoded word equals Alice's (uncorrectable keys are discarded,
Sec. 1); R_eff = (k - s) / (n - p - s) for a rate-adaptive frame with p
punctured and s shortened positions of a mother code of design rate k / n.
"""
from __future__ import annotations

import math

import numpy as np


def wilson_interval(failures: int, trials: int, z: float = 1.96) -> tuple[float, float]:
    if trials <= 0:
        return (0.0, 1.0)
    p = failures / trials
    den = 1 + z * z / trials
    centre = (p + z * z / (2 * trials)) / den
    half = z * math.sqrt(p * (1 - p) / trials + z * z / (4 * trials * trials)) / den
    return (max(0.0, centre - half), min(1.0, centre + half))


def binary_entropy(q: float) -> float:
    if q <= 0.0 or q >= 1.0:
        return 0.0
    return -q * math.log2(q) - (1 - q) * math.log2(1 - q)


def effective_rate(n: int, m: int, n_punct, n_short):
    k = n - m
    return (k - np.asarray(n_short, dtype=np.float64)) / (n - np.asarray(n_punct, dtype=np.float64)
                                                          - np.asarray(n_short, dtype=np.float64))


def efficiency(n: int, m: int, n_punct, n_short, qber) -> np.ndarray:
    """f = (1 - R_eff) / h(q), per frame."""
    r = effective_rate(n, m, n_punct, n_short)
    h = np.vectorize(binary_entropy)(np.asarray(qber, dtype=np.float64))
    return (1.0 - r) / h


def frame_outcomes(x: np.ndarray, bits_unpacked: np.ndarray, conv: np.ndarray):
    """(correct, undetected): correct = converged and equal to x; undetected =
    converged to a different word satisfying the syndrome."""
    equal = (bits_unpacked == x).all(axis=1)
    conv = np.asarray(conv).astype(bool)
    return conv & equal, conv & ~equal
