"""Pins of the tensor-network oracle: it must reproduce the state-vector
definition for every plan, every cut choice and every open-qubit set, and the
sum over slices must equal the unsliced contraction."""
import numpy as np
import pytest

from oracle import sv, tn
from oracle.parse import read_circuit
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate, identity_cz
from workloads.plans import sweep_plan, region_plan, PlanBuilder


@pytest.mark.parametrize("rows,cols,depth", [(2, 2, 8), (3, 3, 8), (3, 4, 16), (4, 4, 16)])
def test_chain_matches_sv(rows, cols, depth):
    c = generate(rows, cols, depth, 3)
    text = c.to_text()
    bits = random_bitstrings(5, c.n_qubits, 9)
    ref = sv.amplitudes(text, bits)
    got = tn.amplitudes(text, bits)[:, 0]
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.max(np.abs(ref)))


def test_region_plan_with_cuts_and_open_matches_sv():
    c = generate(4, 4, 16, 5)
    text = c.to_text()
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 1]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 3), (2, 2)])
    bits = random_bitstrings(3, 16, 2)
    got = tn.amplitudes(text, bits, plan)
    ref = sv.open_amplitudes(text, bits, plan["open"])
    assert np.allclose(got, ref, atol=1e-12)


def test_slices_sum_to_unsliced():
    c = generate(3, 4, 16, 8)
    text = c.to_text()
    qid = c.qubit_of()
    bits = random_bitstrings(2, 12, 4)
    cuts = [[qid[(0, 1)], qid[(0, 2)], 0, 2], [qid[(1, 1)], qid[(2, 1)], 1, 1]]
    sliced = tn.amplitudes(text, bits, sweep_plan(c, cuts=cuts))
    whole = tn.amplitudes(text, bits, sweep_plan(c))
    assert np.allclose(sliced, whole, atol=1e-12)
    # and the slices are genuinely different partial sums
    parts = [tn.amplitudes(text, bits, sweep_plan(c, cuts=cuts), slices=[s]) for s in range(8)]
    assert np.allclose(sum(parts), whole, atol=1e-12)
    assert np.std([abs(p[0, 0]) for p in parts]) > 0


def test_plan_invariance_column_vs_row():
    c = generate(3, 4, 24, 6)
    text = c.to_text()
    bits = random_bitstrings(3, 12, 5)
    a = tn.amplitudes(text, bits, sweep_plan(c, by="row"))
    b = tn.amplitudes(text, bits, sweep_plan(c, by="col"))
    assert np.allclose(a, b, atol=1e-12)


def test_product_circuit_factorises():
    """With every CZ replaced by the identity, a(x) = prod_q <x_q| W_q |0>."""
    from oracle import gates
    c = identity_cz(generate(3, 3, 16, 1))
    text = c.to_text()
    bits = random_bitstrings(4, 9, 3)
    got = tn.amplitudes(text, bits, sweep_plan(c))[:, 0]
    circ = read_circuit(text)
    per_q = []
    for q in range(9):
        v = np.array([1, 0], dtype=np.complex128)
        for (_, name, qs), val in zip(circ.ops, circ.values):
            if qs == (q,):
                v = val @ v
        per_q.append(v)
    want = np.array([np.prod([per_q[q][b[q]] for q in range(9)]) for b in bits])
    assert np.allclose(got, want, atol=1e-13)


def test_plan_checker_rejects_bad_plans():
    from oracle.parse import check_plan
    with pytest.raises(ValueError):
        check_plan(3, {"steps": [[0, 1], [0, 2]]})
    with pytest.raises(ValueError):
        check_plan(3, {"steps": [[0, 1]]})
    with pytest.raises(ValueError):
        check_plan(3, {"steps": [[0, 4], [1, 2]]})
