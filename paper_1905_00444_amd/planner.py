"""Automatic choice of cuts and contraction order for grid circuits (paper Sec. III-D).

Finding the best cuts and order is NP-hard in general; for planar grids the paper splits the
circuit into pieces with a small shared boundary, cuts bonds on that boundary, and favours orders
whose work sits in a handful of big contractions with many flops per byte moved.  This module searches that
family and ranks candidates by a time model, not by flop count alone:

* Orders.  Quadrant splits at (row r0, column c0): regions A (top-left), B (top-right), D
  (bottom-left), C (bottom-right); A, B and D are grown cell by cell from their outer corners,
  each time absorbing the adjacent cell that gives the smallest tensor; then A x B, (AB) x D, and
  the cells of C one by one (open output qubits last).  Half splits (left/right, top/bottom)
  grow each half from its outer corner and contract the two.  Plain row and column sweeps are
  included for small grids.
* Cuts.  Up to `max_cuts` bonds crossing region boundaries, each cut over its leading 1..all bond
  bits; the cut listed first is the most significant part of the slice id, and both orders of
  two cuts are tried (subtrees that depend only on the leading cut are reused across slices).
* Time model.  Per step: GEMM time max(8 M N K / rate, bytes / bandwidth) plus the operand
  permutes and a per-launch overhead; a step runs once per change of the cut values it depends
  on (the library's reuse rule), so the total over all slices of one prefix is
  sum_steps runs * time.  Rates default to figures measured on MI355X and can be replaced by the
  per-shape microseconds of a qf_autotune cache file.
* Constraint.  Every tensor (operands and results) has at most `max_bits` bits.

The result is a plan dictionary for Plan / qf_plan_create ({"steps", "cuts", "open"}), with the
model's peak size, flops and time.
"""
from __future__ import annotations

import itertools
import json
from collections import Counter
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from .api import read_circuit_text

Site = Tuple[int, int]


# ---------------------------------------------------------------------------------------------
class GridNetwork:
    """Qubits (row-major over present sites), bonds (edge -> bond bits = two-qubit gates on it)."""

    def __init__(self, text: str):
        rows, cols, removed, n, ops = read_circuit_text(text)
        self.rows, self.cols = rows, cols
        rem = {tuple(x) for x in removed}
        self.sites: List[Site] = [(r, c) for r in range(rows) for c in range(cols) if (r, c) not in rem]
        if len(self.sites) != n:
            raise ValueError("qubit count does not match the grid")
        self.n = n
        self.qid: Dict[Site, int] = {s: i for i, s in enumerate(self.sites)}
        bonds = Counter()
        for _, _, qs in ops:
            if len(qs) == 2:
                a, b = min(qs), max(qs)
                (ra, ca), (rb, cb) = self.sites[a], self.sites[b]
                if abs(ra - rb) + abs(ca - cb) != 1:
                    raise ValueError(f"two-qubit gate on non-neighbours {a}, {b}")
                bonds[(a, b)] += 1
        self.edges: List[Tuple[int, int]] = sorted(bonds)
        self.bond_bits = np.array([bonds[e] for e in self.edges], dtype=np.int64)
        self.e0 = np.array([e[0] for e in self.edges], dtype=np.int64)
        self.e1 = np.array([e[1] for e in self.edges], dtype=np.int64)
        self.edge_index = {e: i for i, e in enumerate(self.edges)}


def _bits(net: GridNetwork, mem: np.ndarray, w: np.ndarray, open_mask: np.ndarray) -> int:
    cross = mem[net.e0] != mem[net.e1]
    return int(cross @ w + np.count_nonzero(mem & open_mask))


class _Order:
    """Builds a step list while tracking members (boolean masks over qubits)."""

    def __init__(self, net: GridNetwork, w: np.ndarray, open_mask: np.ndarray):
        self.net, self.w, self.open_mask = net, w, open_mask
        self.mem: Dict[int, np.ndarray] = {}
        for q in range(net.n):
            m = np.zeros(net.n, dtype=bool)
            m[q] = True
            self.mem[q] = m
        self.steps: List[Tuple[int, int]] = []

    def contract(self, a: int, b: int) -> int:
        nid = self.net.n + len(self.steps)
        self.steps.append((a, b))
        self.mem[nid] = self.mem[a] | self.mem[b]
        return nid

    def grow(self, cells: Sequence[Site], start: Optional[Site] = None, into: Optional[int] = None) -> int:
        """Absorb `cells` one at a time into the node `into` (or starting from cell `start`),
        always the adjacent cell that gives the smallest tensor; open cells go last."""
        net = self.net
        todo = list(cells)
        if into is None:
            todo.remove(start)
            cur = net.qid[start]
        else:
            cur = into
        have = {net.sites[q] for q in np.flatnonzero(self.mem[cur])}
        while todo:
            adj = [s for s in todo if any((s[0] + dr, s[1] + dc) in have
                                          for dr, dc in ((1, 0), (-1, 0), (0, 1), (0, -1)))] or todo
            closed = [s for s in adj if not self.open_mask[net.qid[s]]] or adj
            best = min(closed, key=lambda s: (_bits(net, self.mem[cur] | self.mem[net.qid[s]], self.w,
                                                    self.open_mask), s))
            cur = self.contract(cur, net.qid[best])
            have.add(best)
            todo.remove(best)
        return cur


# ---------------------------------------------------------------------------------------------
@dataclass
class CostModel:
    """Time of one contraction step on one GPU (seconds)."""
    precision: str = "bf16x3"
    # large-GEMM rates and permute bandwidth measured on one MI355X (complex flop/s, bytes/s)
    gemm_rate: Dict[str, float] = field(default_factory=lambda: {"fp32": 137e12, "bf16x3": 520e12,
                                                                 "fp16": 750e12})
    bandwidth: float = 5.3e12       # bytes/s reached by the permutes
    launch: float = 4e-6            # seconds per kernel launch
    batch: int = 1                  # chains per launch
    measured: Dict[Tuple[int, int, int], float] = field(default_factory=dict)  # (M, N, K) bits -> s

    @classmethod
    def from_autotune(cls, path: str, precision: str = "bf16x3", batch: int = 1, **kw) -> "CostModel":
        """Take per-shape GEMM times (the chosen variant's microseconds) from a qf_autotune file."""
        from .api import PRECISIONS
        doc = json.load(open(path))
        m = {}
        for e in doc.get("entries", []):
            if e["precision"] != PRECISIONS[precision] or e["batch"] != batch:
                continue
            us = e.get("us", {}).get(e["variant"])
            if us:
                key = tuple(int(x).bit_length() - 1 for x in (e["M"], e["N"], e["K"]))
                m[key] = us * 1e-6
        return cls(precision=precision, batch=batch, measured=m, **kw)

    def steps_seconds(self, m: np.ndarray, n: np.ndarray, k: np.ndarray) -> np.ndarray:
        """step_seconds elementwise over arrays of step shapes (bits of M, N, K)."""
        G = self.batch
        f = np.power(2.0, m + n + k)
        mk, nk, mn = np.power(2.0, m + k), np.power(2.0, n + k), np.power(2.0, m + n)
        t = np.maximum(8.0 * G * f / self.gemm_rate[self.precision], 8.0 * G * (mk + nk + mn) / self.bandwidth)
        t = t + self.launch
        for (a, b, c), v in self.measured.items():
            t = np.where((m == a) & (n == b) & (k == c), v, t)
        return t + 16.0 * G * (mk + nk) / self.bandwidth + 2 * self.launch

    def step_seconds(self, m: int, n: int, k: int) -> float:
        G = self.batch
        flops = 8.0 * 2.0 ** (m + n + k) * G
        t = self.measured.get((m, n, k))
        if t is None:
            io = 8.0 * G * (2.0 ** (m + k) + 2.0 ** (n + k) + 2.0 ** (m + n))
            t = max(flops / self.gemm_rate[self.precision], io / self.bandwidth) + self.launch
        permute = 8.0 * G * 2.0 * (2.0 ** (m + k) + 2.0 ** (n + k)) / self.bandwidth + 2 * self.launch
        return t + permute


@dataclass
class PlanChoice:
    plan: dict
    description: str
    peak_bits: int
    n_slices: int
    flops: float          # executed flops over all slices of one prefix (with reuse)
    seconds: float        # model time over all slices of one prefix

    def __repr__(self) -> str:
        return (f"PlanChoice({self.description}: peak 2^{self.peak_bits}, {self.n_slices} slices, "
                f"{self.flops:.3e} flop, {self.seconds:.3g} s per prefix)")


class _Evaluator:
    """Vectorised evaluation of one order under many cut choices."""

    def __init__(self, net: GridNetwork, steps: Sequence[Tuple[int, int]], open_mask: np.ndarray):
        n = net.n
        mem = [None] * (n + len(steps))
        for q in range(n):
            m = np.zeros(n, dtype=bool)
            m[q] = True
            mem[q] = m
        ca, cb, cr, sk, oa, ob, orr, rm = [], [], [], [], [], [], [], []
        for i, (a, b) in enumerate(steps):
            ma, mb = mem[a], mem[b]
            mr = ma | mb
            mem[n + i] = mr
            ca.append(ma[net.e0] != ma[net.e1])
            cb.append(mb[net.e0] != mb[net.e1])
            cr.append(mr[net.e0] != mr[net.e1])
            sk.append((ma[net.e0] & mb[net.e1]) | (ma[net.e1] & mb[net.e0]))
            oa.append(np.count_nonzero(ma & open_mask))
            ob.append(np.count_nonzero(mb & open_mask))
            orr.append(np.count_nonzero(mr & open_mask))
            rm.append(mr)
        self.net = net
        self.steps = list(steps)
        self.ca, self.cb, self.cr, self.sk = (np.array(x, dtype=np.int64) for x in (ca, cb, cr, sk))
        self.oa, self.ob, self.orr = (np.array(x, dtype=np.int64) for x in (oa, ob, orr))
        self.rmem = np.array(rm, dtype=bool)
        # leaves: bits of every world-line with its output bit fixed or open
        self.leaf_cross = np.zeros((n, len(net.edges)), dtype=np.int64)
        for j, (a, b) in enumerate(net.edges):
            self.leaf_cross[a, j] = self.leaf_cross[b, j] = 1
        self.leaf_open = open_mask.astype(np.int64)

    def evaluate_many(self, sets: Sequence[Sequence[Tuple[int, int]]], model: CostModel, max_bits: int):
        """Every cut choice at once.  sets: tuples of (edge index, cut bits), first = most
        significant part of the slice id.  Returns (index, peak, slices, flops, seconds) of the
        choices whose tensors all fit in 2^max_bits."""
        net = self.net
        ns = len(sets)
        if ns == 0:
            return []
        kmax = max(1, max(len(c) for c in sets))
        E = np.zeros((ns, kmax), dtype=np.int64)
        NB = np.zeros((ns, kmax), dtype=np.int64)
        for i, cs in enumerate(sets):
            for j, (e, nb) in enumerate(cs):
                E[i, j], NB[i, j] = e, nb
        W = np.tile(net.bond_bits.astype(np.float64), (ns, 1))
        np.subtract.at(W, (np.repeat(np.arange(ns), kmax), E.reshape(-1)), NB.reshape(-1))
        ba = W @ self.ca.T + self.oa
        bb = W @ self.cb.T + self.ob
        br = W @ self.cr.T + self.orr
        kk = W @ self.sk.T
        leaf = W @ self.leaf_cross.T + self.leaf_open
        peak = np.maximum.reduce([ba.max(1), bb.max(1), br.max(1), leaf.max(1)])
        ok = np.flatnonzero(peak <= max_bits)
        if ok.size == 0:
            return []
        E, NB, ba, bb, kk = E[ok], NB[ok], ba[ok], bb[ok], kk[ok]
        total = NB.sum(1)
        # offset of each cut inside the slice id (from the least significant end)
        off = total[:, None] - np.cumsum(NB, axis=1)
        rm = self.rmem.T.astype(bool)                       # qubit x step
        dep = rm[net.e0[E]] | rm[net.e1[E]]                # set x cut x step
        dep &= (NB > 0)[:, :, None]
        low = np.where(dep, off[:, :, None], 10 ** 6).min(axis=1)  # set x step
        runs = np.where(low < 10 ** 6, np.power(2.0, total[:, None] - np.minimum(low, total[:, None])), 1.0)
        m, n = ba - kk, bb - kk
        flops = (runs * 8.0 * np.power(2.0, m + n + kk)).sum(1)
        secs = (runs * model.steps_seconds(m, n, kk)).sum(1)
        return [(int(ok[i]), int(peak[ok[i]]), int(1 << int(total[i])), float(flops[i]), float(secs[i]))
                for i in range(ok.size)]

    def evaluate(self, cuts: Sequence[Tuple[int, int]], model: CostModel):
        """(peak, slices, flops, seconds) of one cut choice (no size limit)."""
        _, peak, S, flops, secs = self.evaluate_many([tuple(cuts)], model, 10 ** 9)[0]
        return peak, S, flops, secs


# ---------------------------------------------------------------------------------------------
def _quadrant_order(net: GridNetwork, r0: int, c0: int, w: np.ndarray, open_mask: np.ndarray):
    R, C = net.rows, net.cols
    have = set(net.sites)
    reg = lambda rs, cs: [(r, c) for r in rs for c in cs if (r, c) in have]
    A, B = reg(range(r0), range(c0)), reg(range(r0), range(c0, C))
    D, Cq = reg(range(r0, R), range(c0)), reg(range(r0, R), range(c0, C))
    if not (A and B and D and Cq):
        return None
    o = _Order(net, w, open_mask)
    corner = lambda cells, key: min(cells, key=key)
    a = o.grow(A, start=corner(A, lambda s: (s[0] + s[1], s)))
    b = o.grow(B, start=corner(B, lambda s: (s[0] - s[1], s)))
    d = o.grow(D, start=corner(D, lambda s: (s[1] - s[0], s)))
    ab = o.contract(a, b)
    abd = o.contract(ab, d)
    o.grow(Cq, into=abd)
    return o.steps, (A, B, D, Cq)


def _half_order(net: GridNetwork, split: int, vertical: bool, w: np.ndarray, open_mask: np.ndarray):
    have = set(net.sites)
    if vertical:
        P = [s for s in net.sites if s[1] < split]
        Q = [s for s in net.sites if s[1] >= split]
        sp = min(P, key=lambda s: (s[1] + s[0], s))
        sq = min(Q, key=lambda s: (s[0] - s[1], s))
    else:
        P = [s for s in net.sites if s[0] < split]
        Q = [s for s in net.sites if s[0] >= split]
        sp = min(P, key=lambda s: (s[0] + s[1], s))
        sq = min(Q, key=lambda s: (s[1] - s[0], s))
    if not P or not Q or not (set(P) | set(Q)) <= have:
        return None
    o = _Order(net, w, open_mask)
    p = o.grow(P, start=sp)
    q = o.grow(Q, start=sq)
    o.contract(p, q)
    return o.steps, (P, Q)


def _sweep_order(net: GridNetwork, by_row: bool, open_mask: np.ndarray):
    sites = sorted(net.sites, key=(lambda s: s) if by_row else (lambda s: (s[1], s[0])))
    closed = [s for s in sites if not open_mask[net.qid[s]]]
    opened = [s for s in sites if open_mask[net.qid[s]]]
    seq = closed + opened
    o = _Order(net, net.bond_bits, open_mask)
    cur = net.qid[seq[0]]
    for s in seq[1:]:
        cur = o.contract(cur, net.qid[s])
    return o.steps


def _boundary_edges(net: GridNetwork, regions) -> List[int]:
    where = {}
    for i, reg in enumerate(regions):
        for s in reg:
            where[net.qid[s]] = i
    return [j for j, (a, b) in enumerate(net.edges) if where[a] != where[b]]


def _cut_sets(cands: Sequence[int], net: GridNetwork, max_cuts: int, max_cut_bits: int):
    yield ()
    for k in range(1, max_cuts + 1):
        for es in itertools.combinations(cands, k):
            ranges = [range(1, int(net.bond_bits[e]) + 1) for e in es]
            for nbs in itertools.product(*ranges):
                if sum(nbs) > max_cut_bits:
                    continue
                for perm in (itertools.permutations(range(k)) if k > 1 else [(0,)]):
                    yield tuple((es[i], nbs[i]) for i in perm)


def search(text: str, max_bits: int = 30, open_sites: Sequence[Site] = (), precision: str = "bf16x3",
           max_cuts: int = 2, max_cut_bits: int = 12, model: Optional[CostModel] = None,
           top: int = 1):
    """Best plan(s) for the circuit under the tensor-size limit, ranked by the time model over all
    slices of one prefix.  Returns a PlanChoice, or a list of the `top` best if top > 1."""
    net = GridNetwork(text)
    model = model or CostModel(precision=precision)
    open_q = [net.qid[tuple(s)] for s in open_sites]
    open_mask = np.zeros(net.n, dtype=bool)
    open_mask[open_q] = True
    cands = []  # (seconds, choice)

    def consider(steps, regions, desc):
        ev = _Evaluator(net, steps, open_mask)
        bedges = _boundary_edges(net, regions) if regions else []
        sets = list(_cut_sets(bedges, net, max_cuts, max_cut_bits))
        for i, peak, S, flops, secs in ev.evaluate_many(sets, model, max_bits):
            cs = sets[i]
            cuts = [[int(net.e0[e]), int(net.e1[e]), 0, int(nb)] for e, nb in cs]
            plan = {"steps": [list(s) for s in steps], "cuts": cuts, "open": list(open_q)}
            cands.append((secs, PlanChoice(plan, desc + (f", cuts {[(net.sites[c[0]], net.sites[c[1]], c[3]) for c in cuts]}" if cuts else ""),
                                           peak, S, flops, secs)))

    for by_row in (True, False):
        consider(_sweep_order(net, by_row, open_mask), None, "row sweep" if by_row else "column sweep")
    for r0 in range(1, net.rows):
        for c0 in range(1, net.cols):
            got = _quadrant_order(net, r0, c0, net.bond_bits, open_mask)
            if got:
                consider(got[0], got[1], f"quadrants at ({r0}, {c0})")
    for split in range(1, net.cols):
        got = _half_order(net, split, True, net.bond_bits, open_mask)
        if got:
            consider(got[0], got[1], f"left/right halves at column {split}")
    for split in range(1, net.rows):
        got = _half_order(net, split, False, net.bond_bits, open_mask)
        if got:
            consider(got[0], got[1], f"top/bottom halves at row {split}")
    if not cands:
        raise ValueError(f"no plan within 2^{max_bits} found (raise max_bits, max_cuts or max_cut_bits)")
    cands.sort(key=lambda t: (t[0], t[1].n_slices))
    best = [c for _, c in cands[:top]]
    return best[0] if top == 1 else best


def evaluate(text: str, plan: dict, precision: str = "bf16x3", model: Optional[CostModel] = None):
    """The time model's figures (peak bits, slices, flops, seconds per prefix) for a given plan."""
    net = GridNetwork(text)
    model = model or CostModel(precision=precision)
    open_mask = np.zeros(net.n, dtype=bool)
    open_mask[list(plan.get("open", []))] = True
    ev = _Evaluator(net, [tuple(s) for s in plan["steps"]], open_mask)
    cs = []
    for q0, q1, lo, nb in plan.get("cuts", []):
        cs.append((net.edge_index[(min(q0, q1), max(q0, q1))], int(nb)))
    peak, S, flops, secs = ev.evaluate(cs, model)
    return PlanChoice(plan, "given plan", peak, S, flops, secs)
