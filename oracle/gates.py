"""Gate matrices of the random-circuit gate set, complex128 (oracle's own table).

The paper names the gate set (H, CZ, T, sqrt(X), sqrt(Y); Sec. III and its RQC
references) but prints no matrices.  Conventions fixed here:
    H      = (1/sqrt 2) [[1, 1], [1, -1]]
    T      = diag(1, exp(i pi/4));  S = T^2 = diag(1, i)
    sqrt X = principal square root of X = (1/2) [[1+i, 1-i], [1-i, 1+i]]
    sqrt Y = principal square root of Y = (1+i)/2 [[1, -1], [1, 1]]
    CZ     = diag(1, 1, 1, -1) on (q0, q1), index 2*b_q0 + b_q1
    id2    = diag(1, 1, 1, 1)   (two-qubit identity, same bond structure as CZ)
A 'dg' suffix means the adjoint.  The CPU tests pin the table by algebra:
H^2 = I, T^2 = S, T^8 = I, sqrt(X)^2 = X, sqrt(Y)^2 = Y, unitarity.
"""
from __future__ import annotations

import numpy as np

_s2 = 1.0 / np.sqrt(2.0)

ONE_QUBIT = {
    "h": np.array([[_s2, _s2], [_s2, -_s2]], dtype=np.complex128),
    "t": np.array([[1, 0], [0, np.exp(1j * np.pi / 4)]], dtype=np.complex128),
    "s": np.array([[1, 0], [0, 1j]], dtype=np.complex128),
    "x_1_2": 0.5 * np.array([[1 + 1j, 1 - 1j], [1 - 1j, 1 + 1j]], dtype=np.complex128),
    "y_1_2": 0.5 * np.array([[1 + 1j, -1 - 1j], [1 + 1j, 1 + 1j]], dtype=np.complex128),
    "x": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "id": np.eye(2, dtype=np.complex128),
}

# diagonal two-qubit gates: the 4 diagonal entries, index 2*b_q0 + b_q1
TWO_QUBIT_DIAG = {
    "cz": np.array([1, 1, 1, -1], dtype=np.complex128),
    "id2": np.array([1, 1, 1, 1], dtype=np.complex128),
}


def one_qubit(name: str) -> np.ndarray:
    if name.endswith("dg"):
        return ONE_QUBIT[name[:-2]].conj().T.copy()
    return ONE_QUBIT[name].copy()


def two_qubit_diag(name: str) -> np.ndarray:
    if name.endswith("dg"):
        return TWO_QUBIT_DIAG[name[:-2]].conj().copy()
    return TWO_QUBIT_DIAG[name].copy()


def is_two_qubit(name: str) -> bool:
    base = name[:-2] if name.endswith("dg") else name
    return base in TWO_QUBIT_DIAG
