"""Seeded output bitstrings (input data only).

Bitstrings are uniform random, one byte (0 or 1) per qubit, row-major qubit
order: bits[b, q] is the value of qubit q in bitstring b.  This mirrors drawing
a fresh random prefix x1 per pass in the fast-sampling scheme (paper Sec. III-B).
"""
from __future__ import annotations

import numpy as np


def random_bitstrings(n_batch: int, n_qubits: int, seed: int = 1) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=(n_batch, n_qubits), dtype=np.uint8)


def all_bitstrings(n_qubits: int) -> np.ndarray:
    """All 2^n bitstrings, index i -> bits with qubit 0 as the most significant bit."""
    idx = np.arange(2 ** n_qubits, dtype=np.int64)
    shifts = np.arange(n_qubits - 1, -1, -1, dtype=np.int64)
    return ((idx[:, None] >> shifts[None, :]) & 1).astype(np.uint8)
