"""Gradients of amplitudes with respect to gate entries (adjoint state vector).

Convention (PyTorch's for complex leaves): for a real loss L and a complex gate
entry G, grad = dL/dRe(G) + i dL/dIm(G).  Given the cotangent c_b of each
amplitude a_b (for L = sum_b |a_b|^2, c_b = 2 a_b), the amplitudes are linear
in each gate entry, so
    grad_G = sum_b c_b * conj(d a_b / d G).
Adjoint form: with psi_t = U_{<t}|0> (state before gate t) and
chi_t = U_{>t}^dagger sum_b c_b |x_b> (cotangent pulled back to just after
gate t),
    one-qubit G on q:   grad[i, j] = sum_rest chi_t[i, rest] conj(psi_t[j, rest])
    diagonal D on q0,q1: grad[k]   = sum_{idx in class k} chi_t[idx] conj(psi_t[idx])
Pinned in the tests by central finite differences, which are exact here
because L_c(G) = sum_b Re(conj(c_b) a_b(G)) is linear in every entry.
Gradients are not part of the paper; the amplitudes they differentiate are those
of the circuit's tensor network (paper Sec. II).
"""
from __future__ import annotations

import numpy as np

from . import sv
from .parse import OracleCircuit, read_circuit


def adjoint_gradient(circ, bits: np.ndarray, cot: np.ndarray):
    """Per-op gradients: 2x2 arrays for one-qubit gates, 4-vectors for diagonal
    two-qubit gates."""
    if isinstance(circ, str):
        circ = read_circuit(circ)
    n = circ.n
    psi = np.zeros(2 ** n, dtype=np.complex128)
    psi[0] = 1.0
    before = []
    for (_, _, qs), val in zip(circ.ops, circ.values):
        before.append(psi)
        psi = sv.apply_op(psi, n, qs, val)
    chi = np.zeros(2 ** n, dtype=np.complex128)
    np.add.at(chi, sv.bit_index(bits), np.asarray(cot, dtype=np.complex128))
    grads = [None] * len(circ.ops)
    for t in range(len(circ.ops) - 1, -1, -1):
        (_, _, qs), val = circ.ops[t], circ.values[t]
        p = before[t]
        if len(qs) == 1:
            q = qs[0]
            cv = chi.reshape(2 ** q, 2, -1)
            pv = p.reshape(2 ** q, 2, -1)
            grads[t] = np.einsum("aib,ajb->ij", cv, pv.conj())
            adj = val.conj().T
        else:
            q0, q1 = qs
            prod = (chi * p.conj()).reshape((2,) * n)
            axes = tuple(a for a in range(n) if a not in (q0, q1))
            grads[t] = prod.sum(axis=axes).reshape(4)
            adj = val.conj()
        chi = sv.apply_op(chi, n, qs, adj)
    return grads


def loss_linear(circ: OracleCircuit, bits: np.ndarray, cot: np.ndarray) -> float:
    a = sv.amplitudes(circ, bits)
    return float(np.sum((np.conj(cot) * a).real))


def fd_gradient(circ, bits: np.ndarray, cot: np.ndarray, op_index: int, h: float = 0.25) -> np.ndarray:
    """Central differences of L_c = sum_b Re(conj(c_b) a_b) for every entry of one op."""
    if isinstance(circ, str):
        circ = read_circuit(circ)
    base = [np.array(v, dtype=np.complex128) for v in circ.values]
    shape = base[op_index].shape
    g = np.zeros(shape, dtype=np.complex128)
    for idx in np.ndindex(*shape):
        parts = []
        for step in (h, 1j * h):
            vals_p = [v.copy() for v in base]
            vals_m = [v.copy() for v in base]
            vals_p[op_index][idx] += step
            vals_m[op_index][idx] -= step
            lp = loss_linear(circ.with_values(vals_p), bits, cot)
            lm = loss_linear(circ.with_values(vals_m), bits, cot)
            parts.append((lp - lm) / (2 * h))
        g[idx] = parts[0] + 1j * parts[1]
    return g


def fd_norm_loss_tn(circ, bits: np.ndarray, plan: dict, op_index: int, entry: int, h: float = 1e-2) -> complex:
    """Gradient of L = sum over bitstrings b and completions j of |a_bj|^2 with respect to one
    entry of one gate (entry: flat index into the 2x2 matrix, or into the 4 diagonal entries),
    as central finite differences of L evaluated by the tensor-network route (tn.amplitudes with
    `plan`), for circuits beyond the state vector's reach.  Returns dL/dRe + i dL/dIm.
    Every amplitude is linear in each gate entry, so L is a quadratic polynomial of it and the
    central difference carries no truncation error for any h (only rounding)."""
    from . import tn
    if isinstance(circ, str):
        circ = read_circuit(circ)
    base = [np.array(v, dtype=np.complex128) for v in circ.values]
    shape = base[op_index].shape
    idx = np.unravel_index(entry, shape)
    parts = []
    for step in (h, 1j * h):
        losses = []
        for sign in (1.0, -1.0):
            vals = [v.copy() for v in base]
            vals[op_index][idx] += sign * step
            a = tn.amplitudes(circ.with_values(vals), bits, plan)
            losses.append(float(np.sum(np.abs(a) ** 2)))
        parts.append((losses[0] - losses[1]) / (2 * h))
    return complex(parts[0], parts[1])
