"""Seeded random-quantum-circuit generator for planar grids (input data only).

This module draws the *structure* of a random circuit: which gate acts on which
qubit at which cycle.  It contains none of the simulation arithmetic: gates are
named, not given as matrices, so the product path and the oracle each map names
to matrices with their own tables.

Circuit class (paper Sec. III, RQC prescription; Sec. V, depth written 1+d+1):
qubits on a rows x cols grid (optionally with sites removed), CZ gates only
between nearest neighbours, an H layer on every qubit at cycle 0, d cycles of CZ
layers interleaved with single-qubit gates from {T, sqrt(X), sqrt(Y)}, and a
final H layer at cycle d+1.  The exact placement rules are not printed in the
paper; the reading used here is:

* Eight CZ patterns.  Horizontal edge (r,c)-(r,c+1) belongs to class
  h = (c + 2*(r mod 2)) mod 4; vertical edge (r,c)-(r+1,c) to class
  v = (r + 2*(c mod 2)) mod 4.  Cycle t (1-based) uses pattern
  P[(t-1) mod 8] with P = [H0, V0, H2, V2, H1, V1, H3, V3].  Every edge
  therefore carries exactly one CZ per 8 cycles, so after time-first
  contraction each grid bond has dimension 2^(d/8).
* Single-qubit gates.  At cycle t >= 2 a qubit that is idle in cycle t's CZ
  pattern but was busy at cycle t-1 gets one gate: its first is T, later ones
  are drawn uniformly from {T, sqrt(X), sqrt(Y)} minus its previous gate.
  Draws use numpy's default_rng(seed) in (cycle, qubit) order.

Text format (one op per line after a header):
    # grid <rows> <cols> [<r>:<c> ...]      removed sites, if any
    <n_qubits>
    <cycle> <name> <q0> [<q1>]
with names h, t, x_1_2, y_1_2, cz.  Qubits are numbered row-major over present
sites; in a cz line q0 < q1.
"""
from __future__ import annotations

import dataclasses
from typing import List, Sequence, Tuple

import numpy as np

GATE_NAMES_1Q = ("t", "x_1_2", "y_1_2")
PATTERN_ORDER = (("h", 0), ("v", 0), ("h", 2), ("v", 2), ("h", 1), ("v", 1), ("h", 3), ("v", 3))


@dataclasses.dataclass(frozen=True)
class Op:
    cycle: int
    name: str
    qubits: Tuple[int, ...]


@dataclasses.dataclass
class Circuit:
    rows: int
    cols: int
    removed: Tuple[Tuple[int, int], ...]
    ops: List[Op]

    @property
    def sites(self) -> List[Tuple[int, int]]:
        rem = set(self.removed)
        return [(r, c) for r in range(self.rows) for c in range(self.cols) if (r, c) not in rem]

    @property
    def n_qubits(self) -> int:
        return len(self.sites)

    def qubit_of(self) -> dict:
        return {rc: i for i, rc in enumerate(self.sites)}

    @property
    def present_mask(self) -> np.ndarray:
        m = np.ones((self.rows, self.cols), dtype=np.uint8)
        for r, c in self.removed:
            m[r, c] = 0
        return m.reshape(-1)

    def to_text(self) -> str:
        rem = " ".join(f"{r}:{c}" for r, c in self.removed)
        lines = [f"# grid {self.rows} {self.cols} {rem}".rstrip(), str(self.n_qubits)]
        for op in self.ops:
            lines.append(" ".join([str(op.cycle), op.name] + [str(q) for q in op.qubits]))
        return "\n".join(lines) + "\n"

    def edges(self) -> List[Tuple[int, int]]:
        """Grid edges (q0 < q1) carrying at least one two-qubit gate, sorted."""
        return sorted({op.qubits for op in self.ops if len(op.qubits) == 2})


def circuit_from_text(text: str) -> Circuit:
    rows = cols = None
    removed: List[Tuple[int, int]] = []
    ops: List[Op] = []
    n = None
    for raw in text.splitlines():
        line = raw.strip()
        if not line:
            continue
        if line.startswith("#"):
            parts = line[1:].split()
            if parts and parts[0] == "grid":
                rows, cols = int(parts[1]), int(parts[2])
                removed = [tuple(int(v) for v in p.split(":")) for p in parts[3:]]
            continue
        if n is None:
            n = int(line)
            continue
        parts = line.split()
        ops.append(Op(int(parts[0]), parts[1], tuple(int(q) for q in parts[2:])))
    circ = Circuit(rows, cols, tuple(removed), ops)
    assert circ.n_qubits == n
    return circ


def edge_class(r0: int, c0: int, r1: int, c1: int) -> Tuple[str, int]:
    if r0 == r1:
        c = min(c0, c1)
        return "h", (c + 2 * (r0 % 2)) % 4
    r = min(r0, r1)
    return "v", (r + 2 * (c0 % 2)) % 4


def grid_edges(rows: int, cols: int, removed: Sequence[Tuple[int, int]] = ()) -> List[Tuple[Tuple[int, int], Tuple[int, int]]]:
    rem = set(removed)
    out = []
    for r in range(rows):
        for c in range(cols):
            if (r, c) in rem:
                continue
            if c + 1 < cols and (r, c + 1) not in rem:
                out.append(((r, c), (r, c + 1)))
            if r + 1 < rows and (r + 1, c) not in rem:
                out.append(((r, c), (r + 1, c)))
    return out


def generate(rows: int, cols: int, depth: int, seed: int = 0,
             removed: Sequence[Tuple[int, int]] = ()) -> Circuit:
    """Random circuit of depth 1+depth+1 on a rows x cols grid (minus `removed`)."""
    rng = np.random.default_rng(seed)
    removed = tuple(sorted(tuple(x) for x in removed))
    circ = Circuit(rows, cols, removed, [])
    qid = circ.qubit_of()
    n = circ.n_qubits
    edges = grid_edges(rows, cols, removed)
    ops: List[Op] = [Op(0, "h", (q,)) for q in range(n)]
    busy_prev = set()
    last_gate = [None] * n
    for t in range(1, depth + 1):
        kind, cls = PATTERN_ORDER[(t - 1) % 8]
        cz = []
        for (a, b) in edges:
            k, cl = edge_class(a[0], a[1], b[0], b[1])
            if k == kind and cl == cls:
                q0, q1 = sorted((qid[a], qid[b]))
                cz.append((q0, q1))
        busy = {q for e in cz for q in e}
        if t >= 2:
            for q in range(n):
                if q in busy_prev and q not in busy:
                    if last_gate[q] is None:
                        name = "t"
                    else:
                        choices = [g for g in GATE_NAMES_1Q if g != last_gate[q]]
                        name = choices[int(rng.integers(0, len(choices)))]
                    last_gate[q] = name
                    ops.append(Op(t, name, (q,)))
        for e in sorted(cz):
            ops.append(Op(t, "cz", e))
        busy_prev = busy
    ops.extend(Op(depth + 1, "h", (q,)) for q in range(n))
    circ.ops = ops
    return circ


def identity_cz(circ: Circuit) -> Circuit:
    """Same structure with every CZ renamed to the two-qubit identity 'id2'.

    Used for the product-state special case: the bond structure (and therefore
    every tensor shape) is unchanged, while the amplitude factorises over qubits.
    """
    ops = [Op(op.cycle, "id2" if op.name == "cz" else op.name, op.qubits) for op in circ.ops]
    return Circuit(circ.rows, circ.cols, circ.removed, ops)


def clifford_substitute(circ: Circuit) -> Circuit:
    """Replace every T by S ('s'): the circuit becomes Clifford."""
    ops = [Op(op.cycle, "s" if op.name == "t" else op.name, op.qubits) for op in circ.ops]
    return Circuit(circ.rows, circ.cols, circ.removed, ops)


INVERSE_NAME = {"h": "h", "t": "tdg", "x_1_2": "x_1_2dg", "y_1_2": "y_1_2dg", "cz": "cz",
                "s": "sdg", "id2": "id2"}


def mirror(circ: Circuit, depth: int, seed: int = 0) -> Circuit:
    """V^dagger V with V the circuit of `depth` CZ cycles (no final H layer).

    The result has 1 + 2*depth + 1 cycles, its unitary is the identity, so the
    amplitude of |0...0> is 1 and every other amplitude is 0.  Gate names of the
    second half carry a 'dg' suffix (adjoint).
    """
    base = generate(circ.rows, circ.cols, depth, seed, circ.removed)
    fwd = [op for op in base.ops if op.cycle <= depth]
    back = []
    for op in reversed(fwd):
        back.append(Op(2 * depth + 1 - op.cycle, INVERSE_NAME[op.name], op.qubits))
    back.sort(key=lambda o: o.cycle)
    return Circuit(circ.rows, circ.cols, circ.removed, fwd + back)
