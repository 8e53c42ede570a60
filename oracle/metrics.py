"""Error and statistics helpers used to compare amplitudes.

Element-wise relative error is ill-conditioned for Porter-Thomas distributed
amplitudes (a few per cent of them sit far below the mean), so comparisons use
the norm-wise relative error over a whole batch.
"""
from __future__ import annotations

import numpy as np


def rel_err(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2 over the whole batch (||a - ref|| if ref is all zero)."""
    a = np.asarray(a, dtype=np.complex128).reshape(-1)
    ref = np.asarray(ref, dtype=np.complex128).reshape(-1)
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / den) if den > 0 else float(np.linalg.norm(a - ref))


def porter_thomas(amps: np.ndarray, n_qubits: int):
    """For p = |a|^2 of uniformly drawn bitstrings, N p ~ Exp(1) for deep random
    circuits (N = 2^n_qubits): returns (mean of N p, mean of (N p)^2, Kolmogorov-Smirnov
    distance between the empirical distribution of N p and 1 - e^-x)."""
    p = np.abs(np.asarray(amps).reshape(-1)) ** 2 * (2.0 ** n_qubits)
    xs = np.sort(p)
    m = len(xs)
    cdf = 1.0 - np.exp(-xs)
    ks = max(np.max(np.arange(1, m + 1) / m - cdf), np.max(cdf - np.arange(0, m) / m))
    return float(np.mean(p)), float(np.mean(p ** 2)), float(ks)
