"""Writes the FP64 reference values that the GPU parity tests compare against.

Every stored value is computed here by the oracle package (plain FP64 numpy code written from
the paper) on the seeded synthetic inputs of the workloads package; nothing comes from the HIP
library, and this script imports nothing from it.  Run from the repository root:

    python tests/golden/make_goldens.py c4   # 7x7 (1+40+1): one slice of one prefix, 64 amplitudes
    python tests/golden/make_goldens.py c5   # 8x9 minus 2 corners (1+24+1): 16 whole amplitudes
    python tests/golden/make_goldens.py c2   # 6x6 (1+24+1): 64 amplitudes and 16 gradient entries
    python tests/golden/make_goldens.py c3   # 7x7 (1+32+1): whole amplitudes of 2 prefixes

Long runs keep per-part results in --scratch (default /tmp/qfmi_goldens) and resume from them.
Each output is a numpy .npz (no pickled objects) next to this file.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import grad, tn  # noqa: E402
from workloads.bitstrings import random_bitstrings  # noqa: E402
from workloads.circuits import generate  # noqa: E402
from workloads.plans import (PlanBuilder, C5_REMOVED, nonvanishing_slices, plan_7x7,  # noqa: E402
                             sweep_plan)


def _say(msg):
    print(f"[{time.strftime('%H:%M:%S')}] {msg}", flush=True)


def plan_cost(circ, plan):
    """(peak bits, flops of one slice as 8 sqrt(v0 v1 v2) summed over steps) of a plan."""
    pb = PlanBuilder(circ, plan.get("cuts", []), plan.get("open", []))
    for a, b in plan["steps"]:
        pb.contract(a, b)
    peak, fl = 0, 0.0
    for i, (a, b) in enumerate(plan["steps"]):
        va, vb, vc = (pb.bits_of(pb.members[x]) for x in (a, b, pb.n + i))
        peak = max(peak, va, vb, vc)
        fl += 8 * 2.0 ** ((va + vb + vc) / 2)
    return peak, fl


def _part(scratch, name, fn):
    """Cached evaluation of one part of a long run."""
    path = os.path.join(scratch, name + ".npy")
    if os.path.exists(path):
        return np.load(path)
    v = fn()
    np.save(path + ".tmp.npy", v)
    os.replace(path + ".tmp.npy", path)
    return v


# 7x7 (1+40+1), bond 32: the benchmark's region plan (two whole corner cuts, 1024 slices, six open
# qubits).  One slice of its 2^30-element tensors does not fit host memory in complex128, so the
# slice is split further by three more cut bond bits (one on each of the bonds (2,0)-(3,0),
# (5,2)-(5,3) and (0,2)-(0,3), their first gates in time) and the eight finer slices are summed:
# summing a cut bit over both values reproduces the uncut contraction exactly (Sec. III-A).
C4_EXTRA_SITES = (((2, 0), (3, 0)), ((5, 2), (5, 3)), ((0, 2), (0, 3)))


def make_c4(args):
    circ = generate(7, 7, 40, 0)
    text = circ.to_text()
    plan, _ = plan_7x7(circ, 40)
    bits = random_bitstrings(64, 49, 1)
    row = bits[:1]
    s = nonvanishing_slices(circ, plan, bits[0], 1)[0]
    qid = circ.qubit_of()
    extra = [[min(qid[a], qid[b]), max(qid[a], qid[b]), 0, 1] for a, b in C4_EXTRA_SITES]
    fine = dict(plan, cuts=[list(c) for c in plan["cuts"]] + extra)
    peak, fl = plan_cost(circ, fine)
    _say(f"c4: slice {s} of prefix 0 as 8 finer slices, peak 2^{peak}, {8 * fl:.3e} flop")
    total = np.zeros((1, 64), dtype=np.complex128)
    for e in range(8):
        t0 = time.perf_counter()
        part = _part(args.scratch, f"c4_s{s}_e{e}",
                     lambda: tn.amplitudes(text, row, fine, slices=[(s << 3) | e]))
        total += part
        _say(f"c4: finer slice {e} done ({time.perf_counter() - t0:.0f} s), |part| {np.linalg.norm(part):.3e}")
    np.savez(os.path.join(HERE, "c4_slice.npz"), amps=total[0], bits=bits[0], slice=np.int64(s),
             extra_cuts=np.array(extra, dtype=np.int64), peak_bits=np.int64(peak), flops=np.float64(8 * fl),
             note=np.array("7x7 (1+40+1) seed 0, bitstrings seed 1 row 0, region plan with cuts "
                           "(2,6)-(3,6) and (6,2)-(6,3), first nonvanishing slice; FP64 oracle-TN"))
    _say(f"c4: wrote c4_slice.npz, |amps| {np.linalg.norm(total):.6e}")


def make_c5(args):
    circ = generate(8, 9, 24, 0, C5_REMOVED)
    text = circ.to_text()
    bits = random_bitstrings(16, 70, 1)
    plan = sweep_plan(circ, by="col")
    peak, fl = plan_cost(circ, plan)
    _say(f"c5: column sweep, peak 2^{peak}, {fl:.3e} flop per bitstring")
    amps = []
    for b in range(16):
        t0 = time.perf_counter()
        amps.append(_part(args.scratch, f"c5_b{b}", lambda: tn.amplitudes(text, bits[b:b + 1], plan))[0, 0])
        _say(f"c5: bitstring {b} done ({time.perf_counter() - t0:.0f} s)")
    np.savez(os.path.join(HERE, "c5_amplitudes.npz"), amps=np.array(amps), bits=bits, peak_bits=np.int64(peak),
             flops_per_bitstring=np.float64(fl),
             note=np.array("8x9 minus (0,0),(7,8), (1+24+1) seed 0, 16 bitstrings seed 1; whole amplitudes by "
                           "an unsliced column sweep; FP64 oracle-TN"))
    _say("c5: wrote c5_amplitudes.npz")


def make_c2(args):
    circ = generate(6, 6, 24, 0)
    text = circ.to_text()
    bits = random_bitstrings(64, 36, 1)
    plan = sweep_plan(circ)
    peak, fl = plan_cost(circ, plan)
    _say(f"c2: row sweep, peak 2^{peak}, {fl:.3e} flop per bitstring")
    amps = _part(args.scratch, "c2_amps", lambda: tn.amplitudes(text, bits, plan))[:, 0]
    # 16 seeded gate entries: 8 of one-qubit gates (the H layers included), 8 diagonal entries of CZs
    one_q = [i for i, op in enumerate(circ.ops) if len(op.qubits) == 1]
    two_q = [i for i, op in enumerate(circ.ops) if len(op.qubits) == 2]
    rng = np.random.default_rng(7)
    ops = list(rng.choice(one_q, 8, replace=False)) + list(rng.choice(two_q, 8, replace=False))
    entries = list(rng.integers(0, 4, 16))
    g = []
    for k, (op, ent) in enumerate(zip(ops, entries)):
        t0 = time.perf_counter()
        v = _part(args.scratch, f"c2_g{op}_{ent}",
                  lambda: np.array(grad.fd_norm_loss_tn(text, bits, plan, int(op), int(ent), h=0.25)))
        g.append(complex(v))
        _say(f"c2: entry {k} (op {op}, entry {ent}) = {complex(v):.6e} ({time.perf_counter() - t0:.0f} s)")
    np.savez(os.path.join(HERE, "c2_grad.npz"), amps=amps, bits=bits, ops=np.array(ops, dtype=np.int64),
             entries=np.array(entries, dtype=np.int64), grad=np.array(g),
             note=np.array("6x6 (1+24+1) seed 0, 64 bitstrings seed 1; gradient of sum |a|^2 by exact central "
                           "differences (h = 0.25) through FP64 oracle-TN (row sweep); dL/dRe + i dL/dIm"))
    _say("c2: wrote c2_grad.npz")


def make_c3(args):
    circ = generate(7, 7, 32, 0)
    text = circ.to_text()
    plan, _ = plan_7x7(circ, 32)
    bits = random_bitstrings(256, 49, 1)
    peak, fl = plan_cost(circ, plan)
    _say(f"c3: region plan, 16 slices, peak 2^{peak}, {16 * fl:.3e} flop per prefix")
    amps = []
    for b in range(2):
        t0 = time.perf_counter()
        amps.append(_part(args.scratch, f"c3_b{b}", lambda: tn.amplitudes(text, bits[b:b + 1], plan))[0])
        _say(f"c3: prefix {b} done ({time.perf_counter() - t0:.0f} s)")
    np.savez(os.path.join(HERE, "c3_prefixes.npz"), amps=np.array(amps), bits=bits[:2], peak_bits=np.int64(peak),
             note=np.array("7x7 (1+32+1) seed 0, prefixes 0 and 1 of 256 bitstrings seed 1, region plan with "
                           "the cut (6,2)-(6,3): whole amplitudes (all 16 slices); FP64 oracle-TN"))
    _say("c3: wrote c3_prefixes.npz")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("which", choices=["c4", "c5", "c2", "c3"])
    ap.add_argument("--scratch", default="/tmp/qfmi_goldens")
    args = ap.parse_args()
    os.makedirs(args.scratch, exist_ok=True)
    {"c4": make_c4, "c5": make_c5, "c2": make_c2, "c3": make_c3}[args.which](args)


if __name__ == "__main__":
    main()
