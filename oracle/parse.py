"""The oracle's own reader for circuit text and plan dictionaries.

Circuit text: an optional '# grid rows cols [r:c ...]' comment, the qubit count,
then one gate per line: '<cycle> <name> <q0> [<q1>]'.  Gates are returned in
(cycle, line) order; gates in one cycle act on disjoint qubits.
"""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

from . import gates


class OracleCircuit:
    def __init__(self, n: int, ops: List[Tuple[int, str, Tuple[int, ...]]], rows=None, cols=None, removed=()):
        self.n = n
        self.ops = ops  # (cycle, name, qubits)
        self.rows, self.cols, self.removed = rows, cols, tuple(removed)
        self.values = []  # per op: 2x2 matrix or 4 diagonal entries
        for _, name, qs in ops:
            if len(qs) == 1:
                self.values.append(gates.one_qubit(name))
            else:
                if not gates.is_two_qubit(name):
                    raise ValueError(f"unknown two-qubit gate {name}")
                self.values.append(gates.two_qubit_diag(name))

    def with_values(self, values) -> "OracleCircuit":
        c = OracleCircuit.__new__(OracleCircuit)
        c.n, c.ops, c.rows, c.cols, c.removed = self.n, self.ops, self.rows, self.cols, self.removed
        c.values = [np.array(v, dtype=np.complex128) for v in values]
        return c


def read_circuit(text: str) -> OracleCircuit:
    n = None
    rows = cols = None
    removed = []
    ops = []
    for raw in text.splitlines():
        s = raw.strip()
        if not s:
            continue
        if s.startswith("#"):
            f = s[1:].split()
            if f and f[0] == "grid":
                rows, cols = int(f[1]), int(f[2])
                removed = [tuple(int(v) for v in p.split(":")) for p in f[3:]]
            continue
        if n is None:
            n = int(s)
            continue
        f = s.split()
        cyc, name, qs = int(f[0]), f[1], tuple(int(v) for v in f[2:])
        if len(qs) == 2 and not qs[0] < qs[1]:
            raise ValueError("two-qubit gate needs q0 < q1")
        for q in qs:
            if not 0 <= q < n:
                raise ValueError("qubit out of range")
        ops.append((cyc, name, qs))
    order = sorted(range(len(ops)), key=lambda i: (ops[i][0], i))
    return OracleCircuit(n, [ops[i] for i in order], rows, cols, removed)


def check_plan(n: int, plan: dict) -> None:
    """Every leaf and intermediate used exactly once; the last result is the root."""
    steps = plan["steps"]
    used = set()
    for i, (a, b) in enumerate(steps):
        for x in (a, b):
            if not (0 <= x < n + i):
                raise ValueError(f"step {i} uses node {x} before it exists")
            if x in used:
                raise ValueError(f"node {x} used twice")
            used.add(x)
    if len(used) != n + len(steps) - 1:
        raise ValueError("plan does not contract every node")
