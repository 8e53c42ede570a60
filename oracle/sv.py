"""Direct state-vector evolution in complex128 (paper Sec. II, first class).

This is the plain definition of what the tensor-network method computes:
a(x) = <x| U |0...0>, U the product of the circuit's gates in cycle order.
Index convention: qubit 0 is the most significant bit, index(x) = sum_q x_q 2^(n-1-q).
Feasible for n up to about 28 on a host.
"""
from __future__ import annotations

import numpy as np

from .parse import OracleCircuit, read_circuit


def _apply_1q(psi: np.ndarray, n: int, q: int, g: np.ndarray) -> np.ndarray:
    v = psi.reshape(2 ** q, 2, 2 ** (n - q - 1))
    return np.einsum("ij,ajb->aib", g, v).reshape(-1)


def _diag_factor(n: int, q0: int, q1: int, g: np.ndarray) -> np.ndarray:
    """Broadcastable array with g[2*b_q0 + b_q1] along axes q0, q1 of a (2,)*n view."""
    shape = [1] * n
    shape[q0] = 2
    shape[q1] = 2
    return g.reshape(2, 2).reshape(shape)


def _apply_diag(psi: np.ndarray, n: int, q0: int, q1: int, g: np.ndarray) -> np.ndarray:
    v = psi.reshape((2,) * n) * _diag_factor(n, q0, q1, g)
    return v.reshape(-1)


def apply_op(psi: np.ndarray, n: int, qubits, value) -> np.ndarray:
    if len(qubits) == 1:
        return _apply_1q(psi, n, qubits[0], value)
    return _apply_diag(psi, n, qubits[0], qubits[1], value)


def final_state(circ) -> np.ndarray:
    if isinstance(circ, str):
        circ = read_circuit(circ)
    n = circ.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    for (_, _, qs), val in zip(circ.ops, circ.values):
        psi = apply_op(psi, n, qs, val)
    return psi


def bit_index(bits: np.ndarray) -> np.ndarray:
    bits = np.asarray(bits, dtype=np.int64)
    n = bits.shape[-1]
    w = 2 ** np.arange(n - 1, -1, -1, dtype=np.int64)
    return bits @ w


def amplitudes(circ, bits: np.ndarray) -> np.ndarray:
    """Amplitudes <x_b| U |0> for each row x_b of `bits` (uint8 0/1)."""
    psi = final_state(circ)
    return psi[bit_index(bits)]


def open_amplitudes(circ, bits: np.ndarray, open_qubits) -> np.ndarray:
    """For each prefix row of `bits`, all 2^k completions over `open_qubits`
    (first open qubit most significant), shape (B, 2^k).  Bits of open qubits
    in `bits` are ignored."""
    psi = final_state(circ)
    bits = np.array(bits, dtype=np.int64, copy=True)
    k = len(open_qubits)
    out = np.empty((bits.shape[0], 2 ** k), dtype=np.complex128)
    for j in range(2 ** k):
        for t, q in enumerate(open_qubits):
            bits[:, q] = (j >> (k - 1 - t)) & 1
        out[:, j] = psi[bit_index(bits)]
    return out


def sliced_state(circ, cuts, s: int) -> np.ndarray:
    """Final state of one path (slice s) of the sliced sum (paper Sec. III-A and III-C), by direct
    evolution: every cut instance of a diagonal two-qubit gate D on (q0, q1) is replaced by the
    term of its rank-2 split D = sum_k |k><k|_q0 (x) diag(D[2k], D[2k+1])_q1 that the slice fixes.
    Cut conventions: bond bit j of an edge is the j-th gate on it in cycle order; slice ids
    concatenate the cuts' values, first cut most significant, bit bit_lo most significant inside
    a cut.  Summed over all slices this is final_state(circ) exactly."""
    if isinstance(circ, str):
        circ = read_circuit(circ)
    total = sum(int(c[3]) for c in cuts)
    fixed = {}
    off = total
    for q0, q1, lo, nb in cuts:
        off -= nb
        v = (s >> off) & ((1 << nb) - 1)
        for i in range(nb):
            fixed[(min(q0, q1), max(q0, q1), lo + i)] = (v >> (nb - 1 - i)) & 1
    n = circ.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    seen = {}
    for (_, _, qs), val in zip(circ.ops, circ.values):
        if len(qs) == 2:
            edge = (min(qs), max(qs))
            j = seen.get(edge, 0)
            seen[edge] = j + 1
            if edge + (j,) in fixed:
                k = fixed[edge + (j,)]
                # the projector sits on the lower-numbered qubit of the edge
                term = np.zeros(4, dtype=np.complex128)
                if qs[0] == edge[0]:
                    term[2 * k: 2 * k + 2] = val[2 * k: 2 * k + 2]
                else:
                    term[[k, 2 + k]] = val[[k, 2 + k]]
                val = term
        psi = apply_op(psi, n, qs, val)
    return psi
