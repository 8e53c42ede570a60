"""Contraction plans for the time-first 2D grid network (input data only).

A plan says *in which order* the per-qubit world-line tensors are contracted,
which grid bonds are cut (sliced), and which output qubits stay open.  It holds
no arithmetic of the method; both the product path and the oracle receive the
same plan and must give the same amplitudes for any valid plan (the amplitude
is plan-invariant in exact arithmetic).

Plan dictionary:
    steps : list of [lhs, rhs] node ids in execution order.  Ids 0..n-1 are the
            qubits' world-line tensors (row-major qubit ids); id n+i is the
            result of step i.  Every node except the last result is consumed
            exactly once.
    cuts  : list of [q0, q1, bit_lo, nbits]: on grid edge (q0 < q1), the bond
            bits bit_lo .. bit_lo+nbits-1 (bond bit j belongs to the j-th two-qubit
            gate on that edge in time order) are fixed per slice.  The slice id
            concatenates the cut values, first listed cut most significant, and
            within a cut bond bit bit_lo is the most significant.
    open  : qubit ids whose output leg stays open; the root tensor enumerates
            all 2^k completions, the first listed open qubit most significant.

Orders follow the paper's recipe (Sec. III-A, Fig. 3 caption; Sec. III-D):
build a few large regions, contract them with each other in a handful of
large, high-arithmetic-intensity contractions, then absorb the remaining cells
one at a time; keep cut bonds on the region boundary.
"""
from __future__ import annotations

from collections import Counter
from typing import Dict, Iterable, List, Sequence, Tuple

from .circuits import Circuit


class PlanBuilder:
    """Tracks open bond bits of each node so orders can be chosen by size."""

    def __init__(self, circ: Circuit, cuts: Sequence[Sequence[int]] = (), open_qubits: Sequence[int] = ()):
        self.circ = circ
        self.n = circ.n_qubits
        self.qid = circ.qubit_of()
        self.site = {v: k for k, v in self.qid.items()}
        cnt = Counter(op.qubits for op in circ.ops if len(op.qubits) == 2)
        cut_bits = Counter()
        for q0, q1, lo, nb in cuts:
            cut_bits[(min(q0, q1), max(q0, q1))] += nb
        self.edge_bits = {e: c - cut_bits.get(e, 0) for e, c in cnt.items()}
        self.cuts = [list(c) for c in cuts]
        self.open = list(open_qubits)
        self.members: Dict[int, frozenset] = {q: frozenset([q]) for q in range(self.n)}
        self.steps: List[List[int]] = []
        self.alive = set(range(self.n))

    def bits_of(self, members: Iterable[int]) -> int:
        s = set(members)
        b = sum(1 for q in s if q in self.open)
        for (q0, q1), nb in self.edge_bits.items():
            if (q0 in s) != (q1 in s):
                b += nb
        return b

    def contract(self, a: int, b: int) -> int:
        assert a in self.alive and b in self.alive and a != b
        nid = self.n + len(self.steps)
        self.steps.append([a, b])
        self.members[nid] = self.members[a] | self.members[b]
        self.alive -= {a, b}
        self.alive.add(nid)
        return nid

    def node_of_site(self, r: int, c: int) -> int:
        return self.qid[(r, c)]

    def chain(self, sites: Sequence[Tuple[int, int]]) -> int:
        """Absorb the listed sites one after another into a running tensor."""
        cur = self.node_of_site(*sites[0])
        for rc in sites[1:]:
            cur = self.contract(cur, self.node_of_site(*rc))
        return cur

    def greedy_region(self, region: Sequence[Tuple[int, int]], start: Tuple[int, int],
                      last: Sequence[Tuple[int, int]] = (), into: int = None) -> int:
        """Grow from `start` (or from node `into`), each time absorbing the adjacent
        cell of `region` that gives the smallest result; cells in `last` go last."""
        remaining = [rc for rc in region if rc != start or into is not None]
        if into is None:
            cur = self.node_of_site(*start)
            cur_sites = {start}
        else:
            cur = into
            cur_sites = {self.site[q] for q in self.members[into]}
        last = set(last)
        while remaining:
            def adjacent(rc):
                r, c = rc
                return any((r + dr, c + dc) in cur_sites for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1)))
            cands = [rc for rc in remaining if adjacent(rc)] or list(remaining)
            pref = [rc for rc in cands if rc not in last] or cands
            def score(rc):
                mem = self.members[cur] | {self.node_of_site(*rc)}
                return (self.bits_of(mem), rc)
            best = min(pref, key=score)
            cur = self.contract(cur, self.node_of_site(*best))
            cur_sites.add(best)
            remaining.remove(best)
        return cur

    def plan(self) -> dict:
        assert len(self.alive) == 1, f"plan leaves {len(self.alive)} nodes"
        return {"steps": [list(s) for s in self.steps], "cuts": [list(c) for c in self.cuts],
                "open": list(self.open)}

    def sizes(self) -> List[int]:
        """Bits of every step result, in step order."""
        return [self.bits_of(self.members[self.n + i]) for i in range(len(self.steps))]


def snake_order(rows: int, cols: int, removed: Sequence[Tuple[int, int]] = ()) -> List[Tuple[int, int]]:
    rem = set(removed)
    out = []
    for r in range(rows):
        cs = range(cols) if r % 2 == 0 else range(cols - 1, -1, -1)
        out.extend((r, c) for c in cs if (r, c) not in rem)
    return out


def sweep_plan(circ: Circuit, open_qubits: Sequence[int] = (), cuts: Sequence[Sequence[int]] = (),
               by: str = "row") -> dict:
    """Row-major (or column-major) sweep: absorb every cell into one running tensor."""
    pb = PlanBuilder(circ, cuts, open_qubits)
    if by == "row":
        sites = [(r, c) for r in range(circ.rows) for c in range(circ.cols)]
    else:
        sites = [(r, c) for c in range(circ.cols) for r in range(circ.rows)]
    rem = set(circ.removed)
    pb.chain([s for s in sites if s not in rem])
    return pb.plan()


def region_plan(circ: Circuit, split_row: int, split_col: int, cuts: Sequence[Sequence[int]] = (),
                open_sites: Sequence[Tuple[int, int]] = ()) -> Tuple[dict, PlanBuilder]:
    """Regions A (top-left), B (top-right), D (bottom-left), C (bottom-right).

    A, B and D are grown greedily from their outer corners; then A x B, then
    (AB) x D; the C cells are absorbed one at a time, open cells last.
    """
    R, Cc = circ.rows, circ.cols
    qid = circ.qubit_of()
    open_q = [qid[s] for s in open_sites]
    pb = PlanBuilder(circ, cuts, open_q)
    A = [(r, c) for r in range(split_row) for c in range(split_col)]
    B = [(r, c) for r in range(split_row) for c in range(split_col, Cc)]
    D = [(r, c) for r in range(split_row, R) for c in range(split_col)]
    C = [(r, c) for r in range(split_row, R) for c in range(split_col, Cc)]
    a = pb.greedy_region(A, (0, 0))
    b = pb.greedy_region(B, (0, Cc - 1))
    ab = pb.contract(a, b)
    d = pb.greedy_region(D, (R - 1, 0))
    abd = pb.contract(ab, d)
    pb.greedy_region(C, None, last=open_sites, into=abd)
    return pb.plan(), pb


# --- structural zeros of slices ------------------------------------------------
#
# Fixing a cut bond bit fixes, on the bond's lower-numbered qubit q0, a projection onto |k> at
# that gate's time (a diagonal gate is split as sum_k |k><k|_q0 (x) diag(.)_q1).  Two rules make
# a slice vanish identically, read off the gate names alone:
#   * only diagonal gates act on q0 between two consecutive projections of the same cut bond:
#     the two bits must agree;
#   * after the bond's last projection q0 sees only diagonal gates, then sqrt(Y) immediately
#     followed by the final H: H sqrt(Y) maps |k> to a multiple of |k>, so the last bit must
#     equal q0's output bit.  (A diagonal gate between sqrt(Y) and H would change that: a CZ
#     factor there flips the sign of |1> depending on another bond, a T rotates it.)
# A fidelity-f pass (a fraction of the paths) should compute paths that are not forced to zero.

DIAGONAL_GATES = {"t", "s", "tdg", "sdg", "cz", "id2"}


def _cut_rules(circ: Circuit, q0: int, q1: int):
    """(ties, tail) for a cut bond: ties = pairs (j, j+1) of bond bits that must agree;
    tail = True if the last bond bit must equal q0's output bit."""
    ops = [op for op in circ.ops if q0 in op.qubits]
    idx = [i for i, op in enumerate(ops) if op.qubits == (q0, q1)]
    ties = []
    for j, (a, b) in enumerate(zip(idx, idx[1:])):
        if all(op.name in DIAGONAL_GATES for op in ops[a + 1:b]):
            ties.append((j, j + 1))
    tail = False
    if idx:
        rest = [op.name for op in ops[idx[-1] + 1:]]
        nondiag = [i for i, name in enumerate(rest) if name not in DIAGONAL_GATES]
        tail = (len(nondiag) == 2 and rest[nondiag[0]] == "y_1_2" and rest[nondiag[1]] == "h"
                and nondiag[1] == nondiag[0] + 1)
    return ties, tail


def slice_vanishes(circ: Circuit, plan: dict, bits_row, s: int) -> bool:
    """True if the rules above force slice s of `plan` to contribute zero for this prefix."""
    cuts = plan.get("cuts", [])
    total = sum(c[3] for c in cuts)
    off = total
    for q0, q1, lo, nb in cuts:
        off -= nb
        v = (s >> off) & ((1 << nb) - 1)
        bit = {lo + i: (v >> (nb - 1 - i)) & 1 for i in range(nb)}
        ties, tail = _cut_rules(circ, q0, q1)
        for a, b in ties:
            if a in bit and b in bit and bit[a] != bit[b]:
                return True
        n_bond = sum(1 for op in circ.ops if op.qubits == (q0, q1))
        if tail and (n_bond - 1) in bit and q0 not in plan.get("open", []) and bit[n_bond - 1] != int(bits_row[q0]):
            return True
    return False


def nonvanishing_slices(circ: Circuit, plan: dict, bits_row, count: int, start: int = 0):
    """The first `count` slices at or after `start` not forced to zero (slice_vanishes)."""
    n_slices = 1 << sum(c[3] for c in plan.get("cuts", []))
    out = []
    for s in range(start, n_slices):
        if not slice_vanishes(circ, plan, bits_row, s):
            out.append(s)
            if len(out) == count:
                break
    return out


# --- the benchmark workloads -------------------------------------------------

C4_OPEN_SITES = ((5, 4), (5, 5), (5, 6), (6, 4), (6, 5), (6, 6))


def plan_7x7(circ: Circuit, depth: int) -> Tuple[dict, PlanBuilder]:
    """7x7 grid: regions split after row 3 and column 3 (paper Fig. 3 layout).

    depth 32 (bond 16): one whole cut on (6,2)-(6,3) -> 16 slices.
    depth 40 (bond 32): whole cuts on (2,6)-(3,6) and (6,2)-(6,3) -> 1024 slices.
    These corner bonds keep the largest tensor at 2^30 (2^28); a cut further inside the
    boundary leaves a hole that grows the region-C frontier to 2^35.  Six output qubits in the
    bottom-right corner stay open (64 amplitudes per pass).
    """
    qid = circ.qubit_of()
    nb = depth // 8
    cut_b = [min(qid[(2, 6)], qid[(3, 6)]), max(qid[(2, 6)], qid[(3, 6)]), 0, nb]
    cut_d = [min(qid[(6, 2)], qid[(6, 3)]), max(qid[(6, 2)], qid[(6, 3)]), 0, nb]
    cuts = [cut_d] if depth <= 32 else [cut_b, cut_d]
    return region_plan(circ, 3, 3, cuts, C4_OPEN_SITES)


# 8x9 grid with corners (0,0) and (7,8) removed: 70 qubits.
C5_REMOVED = ((0, 0), (7, 8))


def plan_8x9(circ: Circuit, depth: int = 24) -> Tuple[dict, PlanBuilder]:
    """Two halves (columns 0-4 and 5-8) joined in one last contraction; 8 cut bits on the boundary
    between them -> 256 slices: the whole bonds (0,4)-(0,5) and (1,4)-(1,5) and the two leading
    bits of (2,4)-(2,5) (a partial cut, paper Sec. III-A: slice sizes may be chosen adaptively).
    Each half is grown greedily from its removed corner without the three cells that carry the
    cut bonds; those three cells are contracted into a strip and absorbed last.  Everything but
    the strips and the three joining contractions is the same for every slice (Sec. III-A: the
    slices share all tensors that no cut touches).  Peak tensor 2^27."""
    qid = circ.qubit_of()
    nb = depth // 8
    cuts = []
    for r, bits in ((0, nb), (1, nb), (2, 2)):
        a, b = qid[(r, 4)], qid[(r, 5)]
        cuts.append([min(a, b), max(a, b), 0, bits])
    pb = PlanBuilder(circ, cuts, [])
    lstrip = [(0, 4), (1, 4), (2, 4)]
    rstrip = [(0, 5), (1, 5), (2, 5)]
    left = [(r, c) for c in range(5) for r in range(circ.rows) if (r, c) in qid and (r, c) not in lstrip]
    right = [(r, c) for c in range(circ.cols - 1, 4, -1) for r in range(circ.rows)
             if (r, c) in qid and (r, c) not in rstrip]
    left_rest = pb.greedy_region(left, (1, 0))
    right_rest = pb.greedy_region(right, (6, 8))
    L = pb.contract(left_rest, pb.chain(lstrip))
    R = pb.contract(right_rest, pb.chain(rstrip))
    pb.contract(L, R)
    return pb.plan(), pb


C11_OPEN_SITES = ((10, 8), (10, 9), (10, 10))


def plan_11x11(circ: Circuit) -> Tuple[dict, PlanBuilder]:
    """11x11 grid, depth (1+24+1), bond 8: regions split after row 5 and column 5, whole cuts
    on the corner bonds (4,10)-(5,10) and (10,4)-(10,5): 64 slices (one path per amplitude is
    the paper's fidelity 1/64), peak tensor 2^30.  Three output qubits in the bottom-right
    corner stay open (8 amplitudes per pass)."""
    qid = circ.qubit_of()
    cuts = []
    for a, b in (((4, 10), (5, 10)), ((10, 4), (10, 5))):
        q0, q1 = sorted((qid[a], qid[b]))
        cuts.append([q0, q1, 0, 3])
    return region_plan(circ, 5, 5, cuts, C11_OPEN_SITES)
