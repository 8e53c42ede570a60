"""Properties of the seeded circuit generator and the benchmark plans."""
from collections import Counter

import pytest

from workloads.circuits import generate, circuit_from_text, edge_class, grid_edges
from workloads.plans import plan_7x7, sweep_plan, PlanBuilder


@pytest.mark.parametrize("rows,cols,depth,removed", [(4, 4, 16, ()), (6, 6, 24, ()), (7, 7, 40, ()),
                                                     (8, 9, 24, ((0, 0), (7, 8)))])
def test_every_edge_gets_one_cz_per_8_cycles(rows, cols, depth, removed):
    c = generate(rows, cols, depth, 0, removed)
    cnt = Counter(op.qubits for op in c.ops if op.name == "cz")
    assert len(cnt) == len(grid_edges(rows, cols, removed))
    assert set(cnt.values()) == {depth // 8}
    # gates in one cycle act on disjoint qubits
    by_cycle = {}
    for op in c.ops:
        seen = by_cycle.setdefault(op.cycle, set())
        assert not (seen & set(op.qubits))
        seen.update(op.qubits)


def test_single_qubit_rules_and_seed():
    a = generate(5, 5, 24, 7)
    b = generate(5, 5, 24, 7)
    assert a.to_text() == b.to_text()
    assert a.to_text() != generate(5, 5, 24, 8).to_text()
    last = {}
    for op in a.ops:
        if op.name in ("t", "x_1_2", "y_1_2"):
            q = op.qubits[0]
            if q not in last:
                assert op.name == "t"
            else:
                assert op.name != last[q]
            last[q] = op.name


def test_text_roundtrip():
    c = generate(8, 9, 8, 0, ((0, 0), (7, 8)))
    d = circuit_from_text(c.to_text())
    assert d.to_text() == c.to_text()
    assert d.n_qubits == 70


def test_7x7_plan_shapes():
    c = generate(7, 7, 40, 0)
    plan, pb = plan_7x7(c, 40)
    assert max(pb.sizes()) == 30
    assert sum(cut[3] for cut in plan["cuts"]) == 10
    assert len(plan["open"]) == 6
    c3 = generate(7, 7, 32, 0)
    plan3, pb3 = plan_7x7(c3, 32)
    assert max(pb3.sizes()) == 28


def test_structurally_vanishing_slices_are_zero_in_the_oracle():
    """Slices the gate-name rules declare vanishing are zero in the FP64 oracle (up to rounding),
    over many seeds, depths and bonds so that both rules fire."""
    import numpy as np
    from oracle import tn
    from workloads.bitstrings import random_bitstrings
    from workloads.plans import slice_vanishes, _cut_rules, sweep_plan
    fired = {"tie": 0, "tail": 0}
    for depth in (8, 16):
        for seed in range(16):
            c = generate(3, 3, depth, seed)
            qid = c.qubit_of()
            for (a, b) in (((0, 0), (0, 1)), ((0, 1), (0, 2)), ((1, 1), (1, 2)), ((0, 2), (1, 2)),
                           ((1, 0), (2, 0)), ((1, 1), (2, 1))):
                q0, q1 = sorted((qid[a], qid[b]))
                ties, tail = _cut_rules(c, q0, q1)
                if not (ties or tail):
                    continue
                nb = depth // 8
                plan = sweep_plan(c, cuts=[[q0, q1, 0, nb]])
                bits = random_bitstrings(2, 9, seed)
                for row in bits:
                    for s in range(2 ** nb):
                        if slice_vanishes(c, plan, row, s):
                            v = tn.amplitudes(c.to_text(), row[None], plan, slices=[s])
                            assert np.abs(v).max() < 1e-14, (depth, seed, a, b, s)
                            fired["tie" if ties else "tail"] += 1
    assert fired["tie"] > 0 and fired["tail"] > 0, fired
