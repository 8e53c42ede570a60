"""Consumers of the amplitudes: frugal rejection sampling and cross-entropy benchmarking.

Host-side (numpy) post-processing of the complex128 amplitudes that qf_amplitudes returns; the
contraction itself stays in the HIP library.

Frugal rejection sampling (paper Sec. III-B): each pass contracts one random prefix x1 with k
open qubits, which yields the probabilities p(x1 x2) of all 2^k completions x2 at the cost of
about one amplitude.  A candidate drawn uniformly from that batch is accepted with probability
min(1, N p / M) (N = 2^n, M a bound on N p that Porter-Thomas statistics exceed rarely); the
first accepted candidate is the pass's sample, and the next pass starts from a new prefix.

Cross-entropy benchmarking (paper Sec. I-A, Fig. 1): for samples S of an n-qubit circuit,
    linear XEB  = N * mean_{x in S} p(x) - 1       (1 for ideal samples, 0 for uniform ones)
    log XEB     = log N + gamma + mean_{x in S} log p(x)   (gamma = Euler's constant)
The figure's running product of probabilities underflows for any useful sample size, so the
cross entropy is accumulated as a sum of logarithms.
"""
from __future__ import annotations

from typing import Optional, Sequence, Tuple

import numpy as np

EULER_GAMMA = 0.5772156649015329


def complete(prefix: np.ndarray, open_qubits: Sequence[int], j: int) -> np.ndarray:
    """Bitstring of completion j of a prefix (first open qubit = most significant bit of j)."""
    x = np.array(prefix, dtype=np.uint8, copy=True)
    k = len(open_qubits)
    for t, q in enumerate(open_qubits):
        x[q] = (j >> (k - 1 - t)) & 1
    return x


def frugal_rejection_sample(amps: np.ndarray, prefixes: np.ndarray, open_qubits: Sequence[int],
                            n_qubits: int, M: float = 10.0, rng: Optional[np.random.Generator] = None,
                            tries_per_pass: Optional[int] = None) -> Tuple[np.ndarray, np.ndarray]:
    """One sample per pass (row of `amps`, shape (passes, 2^k)).  Returns (samples, accepted):
    samples[i] is the accepted bitstring of pass i (undefined where accepted[i] is False)."""
    rng = np.random.default_rng() if rng is None else rng
    amps = np.asarray(amps)
    passes, width = amps.shape
    N = 2.0 ** n_qubits
    tries = width if tries_per_pass is None else tries_per_pass
    samples = np.zeros((passes, n_qubits), dtype=np.uint8)
    accepted = np.zeros(passes, dtype=bool)
    for i in range(passes):
        p = np.abs(amps[i]) ** 2
        for j in rng.permutation(width)[:tries]:
            j = int(j)
            if rng.random() < min(1.0, N * p[j] / M):
                samples[i] = complete(prefixes[i], open_qubits, j)
                accepted[i] = True
                break
    return samples, accepted


def xeb_linear(probs: np.ndarray, n_qubits: int) -> float:
    return float(2.0 ** n_qubits * np.mean(probs) - 1.0)


def xeb_log(probs: np.ndarray, n_qubits: int) -> float:
    probs = np.asarray(probs, dtype=np.float64)
    return float(n_qubits * np.log(2.0) + EULER_GAMMA + np.mean(np.log(probs)))
