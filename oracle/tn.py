"""Tensor-network route to the same amplitudes, complex128, numpy only.

Follows the method in its own order:
  1. Circuit as a tensor network (paper Sec. II, tensor-network class): each
     gate is a small tensor; the input |0> and the output bits are rank-1
     projectors.  A diagonal two-qubit gate D on (q0 < q1) is split exactly as
     D = sum_k |k><k|_q0 (x) diag(D[2k], D[2k+1])_q1, which leaves one bond bit
     of dimension 2 per two-qubit gate between the two qubits (paper Fig. 3:
     adjacent cubes share a bond of dimension 2).
  2. Time-first contraction (Sec. III): every qubit's gates are contracted along
     time into one world-line tensor whose indices are its bond bits (in time
     order) and its output bit; the network becomes a 2D grid.
  3. Slicing (Sec. III-A): the cut bond bits are fixed to one value per slice;
     each slice is an independent network ("path"), and the amplitude is the
     sum over all slices.
  4. Fast sampling (Sec. III-B): open output qubits keep their output index, so
     the last tensor holds all completions of a prefix.
  5. Pairwise contraction in the plan's order (Sec. III-A, III-D); each pair is
     one numpy.tensordot over the shared bond bits.
Labels: ('b', q0, q1, j) is bond bit j (j-th two-qubit gate in time order) of
edge (q0, q1); ('x', q) is the open output bit of qubit q.
"""
from __future__ import annotations

from typing import Dict, List, Optional, Sequence

import numpy as np

from .parse import OracleCircuit, check_plan, read_circuit


def world_lines(circ: OracleCircuit):
    """Per qubit: (tensor, labels) with the output bit as the last axis."""
    n = circ.n
    tens = [np.array([1.0, 0.0], dtype=np.complex128) for _ in range(n)]
    labels: List[List[tuple]] = [[] for _ in range(n)]
    count: Dict[tuple, int] = {}
    for (_, _, qs), val in zip(circ.ops, circ.values):
        if len(qs) == 1:
            q = qs[0]
            # W[..., s] -> sum_s W[..., s] G[t, s]
            tens[q] = np.tensordot(tens[q], val, axes=([tens[q].ndim - 1], [1]))
            continue
        q0, q1 = qs
        j = count.get((q0, q1), 0)
        count[(q0, q1)] = j + 1
        lab = ("b", q0, q1, j)
        # projector side: F0[k, s] = delta(k, s); diagonal side: F1[k, s] = D[2k + s]
        f0 = np.eye(2, dtype=np.complex128)
        f1 = np.asarray(val, dtype=np.complex128).reshape(2, 2)
        for q, f in ((q0, f0), (q1, f1)):
            w = tens[q]
            # W'[..., k, s] = W[..., s] * F[k, s]
            tens[q] = w[..., None, :] * f
            labels[q].append(lab)
    return tens, labels


def _cut_values(cuts: Sequence[Sequence[int]], s: int) -> Dict[tuple, int]:
    total = sum(c[3] for c in cuts)
    vals = {}
    off = total
    for q0, q1, lo, nb in cuts:
        off -= nb
        v = (s >> off) & ((1 << nb) - 1)
        for i in range(nb):
            vals[(min(q0, q1), max(q0, q1), lo + i)] = (v >> (nb - 1 - i)) & 1
    return vals


def _leaf(t: np.ndarray, labs: List[tuple], q: int, bit: Optional[int], cutv: Dict[tuple, int]):
    idx = []
    out_labs = []
    for lab in labs:
        key = lab[1:]
        if key in cutv:
            idx.append(cutv[key])
        else:
            idx.append(slice(None))
            out_labs.append(lab)
    if bit is None:
        idx.append(slice(None))
        out_labs.append(("x", q))
    else:
        idx.append(bit)
    return t[tuple(idx)], out_labs


def _contract(a, la, b, lb):
    shared = [l for l in la if l in lb]
    ia = [la.index(l) for l in shared]
    ib = [lb.index(l) for l in shared]
    c = np.tensordot(a, b, axes=(ia, ib))
    lc = [l for l in la if l not in shared] + [l for l in lb if l not in shared]
    return c, lc


def chain_plan(n: int) -> dict:
    steps = [[0, 1]] + [[n + i - 1, i + 1] for i in range(1, n - 1)]
    return {"steps": steps, "cuts": [], "open": []}


def slice_amplitudes(circ, bits_row: np.ndarray, plan: dict, s: int, wl=None) -> np.ndarray:
    """Contribution of slice s to the 2^k amplitudes of one prefix."""
    if isinstance(circ, str):
        circ = read_circuit(circ)
    n = circ.n
    tens, labels = wl if wl is not None else world_lines(circ)
    open_q = list(plan.get("open", []))
    cutv = _cut_values(plan.get("cuts", []), s)
    nodes = []
    for q in range(n):
        bit = None if q in open_q else int(bits_row[q])
        nodes.append(_leaf(tens[q], labels[q], q, bit, cutv))
    for a, b in plan["steps"]:
        (ta, la), (tb, lb) = nodes[a], nodes[b]
        nodes.append(_contract(ta, la, tb, lb))
        nodes[a] = nodes[b] = None
    root, lr = nodes[-1]
    want = [("x", q) for q in open_q]
    if sorted(lr) != sorted(want):
        raise ValueError(f"root has labels {lr}, expected open legs {want}")
    perm = [lr.index(l) for l in want]
    return np.transpose(root, perm).reshape(-1) if want else np.asarray(root).reshape(1)


def amplitudes(circ, bits: np.ndarray, plan: Optional[dict] = None, slices=None) -> np.ndarray:
    """Amplitudes (B, 2^k) summed over `slices` (default: all slices)."""
    if isinstance(circ, str):
        circ = read_circuit(circ)
    n = circ.n
    if plan is None:
        plan = chain_plan(n)
    check_plan(n, plan)
    n_cut = sum(c[3] for c in plan.get("cuts", []))
    if slices is None:
        slices = range(2 ** n_cut)
    wl = world_lines(circ)
    k = len(plan.get("open", []))
    bits = np.asarray(bits)
    out = np.zeros((bits.shape[0], 2 ** k), dtype=np.complex128)
    for bi in range(bits.shape[0]):
        for s in slices:
            out[bi] += slice_amplitudes(circ, bits[bi], plan, s, wl)
    return out


def partial_contract(circ, bits_row: np.ndarray, plan: dict, s: int, n_steps: int = None, subset=None):
    """Run only some contractions of slice s (used to time a bounded sample of a large
    workload): the first n_steps, or the step indices in `subset` (ascending; each step's
    inputs must be leaves or results of earlier listed steps).  Returns the last result."""
    if isinstance(circ, str):
        circ = read_circuit(circ)
    n = circ.n
    tens, labels = world_lines(circ)
    open_q = list(plan.get("open", []))
    cutv = _cut_values(plan.get("cuts", []), s)
    nodes = {}
    for q in range(n):
        bit = None if q in open_q else int(bits_row[q])
        nodes[q] = _leaf(tens[q], labels[q], q, bit, cutv)
    idx = list(range(n_steps)) if subset is None else list(subset)
    last = None
    for i in idx:
        a, b = plan["steps"][i]
        (ta, la), (tb, lb) = nodes.pop(a), nodes.pop(b)
        last = _contract(ta, la, tb, lb)
        nodes[n + i] = last
    return last
