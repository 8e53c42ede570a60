"""Gate values for the library's qf_op records (the binding's own table).

Conventions: H = (1/sqrt 2)[[1, 1], [1, -1]], T = diag(1, e^{i pi/4}), S = diag(1, i),
sqrt(X) = (1/2)[[1+i, 1-i], [1-i, 1+i]], sqrt(Y) = ((1+i)/2)[[1, -1], [1, 1]] (principal
roots), CZ = diag(1, 1, 1, -1) indexed 2*b_q0 + b_q1, id2 = diag(1, 1, 1, 1).  A 'dg'
suffix is the adjoint.
"""
from __future__ import annotations

import math

import numpy as np

_h = 1.0 / math.sqrt(2.0)
_w = complex(math.cos(math.pi / 4), math.sin(math.pi / 4))

_ONE = {
    "h": [[_h, _h], [_h, -_h]],
    "t": [[1, 0], [0, _w]],
    "s": [[1, 0], [0, 1j]],
    "x_1_2": [[0.5 + 0.5j, 0.5 - 0.5j], [0.5 - 0.5j, 0.5 + 0.5j]],
    "y_1_2": [[0.5 + 0.5j, -0.5 - 0.5j], [0.5 + 0.5j, 0.5 + 0.5j]],
    "x": [[0, 1], [1, 0]],
    "id": [[1, 0], [0, 1]],
}
_TWO = {"cz": [1, 1, 1, -1], "id2": [1, 1, 1, 1]}


def gate_entries(name: str) -> np.ndarray:
    """4 complex entries: a row-major 2x2 matrix, or the 4 diagonal entries of a 2-qubit gate."""
    adj = name.endswith("dg")
    base = name[:-2] if adj else name
    if base in _ONE:
        m = np.array(_ONE[base], dtype=np.complex128)
        if adj:
            m = m.conj().T
        return m.reshape(4)
    if base in _TWO:
        d = np.array(_TWO[base], dtype=np.complex128)
        return d.conj() if adj else d
    raise KeyError(f"unknown gate {name}")


def is_two_qubit(name: str) -> bool:
    base = name[:-2] if name.endswith("dg") else name
    return base in _TWO
