"""Pins of the oracle's helper functions against closed forms and against the state vector:
partial contractions (a prefix or a subset of a plan's steps), the Porter-Thomas statistics, and
the finite-difference gradient through the tensor-network route."""
import numpy as np
import pytest

from oracle import grad, sv, tn
from oracle.metrics import porter_thomas, rel_err
from workloads.bitstrings import random_bitstrings, all_bitstrings
from workloads.circuits import Circuit, Op, generate
from workloads.plans import region_plan, sweep_plan


def _rows_decoupled(rows, cols, depth, seed):
    """A generated circuit without its vertical CZs: the rows never interact, so a row's part of
    the network contracts to the amplitude of that row alone."""
    c = generate(rows, cols, depth, seed)
    ops = [op for op in c.ops if len(op.qubits) == 1 or op.qubits[0] // cols == op.qubits[1] // cols]
    return Circuit(rows, cols, (), ops)


def _row_circuit(c, r):
    """Row r of a rows-decoupled circuit as a 1 x cols circuit."""
    lo = r * c.cols
    ops = [Op(op.cycle, op.name, tuple(q - lo for q in op.qubits)) for op in c.ops
           if all(lo <= q < lo + c.cols for q in op.qubits)]
    return Circuit(1, c.cols, (), ops)


def test_partial_contract_every_step_is_the_slice():
    c = generate(4, 4, 16, 5)
    text = c.to_text()
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 1]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 3), (2, 2)])
    bits = random_bitstrings(2, 16, 2)
    for b in range(2):
        for s in (0, 5):
            root, labels = tn.partial_contract(text, bits[b], plan, s, n_steps=len(plan["steps"]))
            want = [("x", q) for q in plan["open"]]
            got = np.transpose(root, [labels.index(l) for l in want]).reshape(-1)
            assert np.array_equal(got, tn.slice_amplitudes(text, bits[b], plan, s))


@pytest.mark.parametrize("open_q", [[], [2]])
def test_partial_contract_prefix_is_the_first_row(open_q):
    c = _rows_decoupled(2, 3, 16, 4)
    plan = sweep_plan(c, open_qubits=open_q)  # row-major chain: its first two steps hold row 0
    bits = random_bitstrings(3, 6, 1)
    row0 = _row_circuit(c, 0).to_text()
    for b in range(3):
        t, labels = tn.partial_contract(c.to_text(), bits[b], plan, 0, n_steps=2)
        assert labels == [("x", q) for q in open_q]
        if open_q:
            want = sv.open_amplitudes(row0, bits[b:b + 1, :3], open_q)[0]
        else:
            want = sv.amplitudes(row0, bits[b:b + 1, :3])
        assert np.allclose(np.asarray(t).reshape(-1), want, rtol=0, atol=1e-13)


def test_partial_contract_subset_is_the_second_row():
    c = _rows_decoupled(2, 3, 16, 6)
    # row 0 -> node 7, row 1 -> node 9, then the two rows
    plan = {"steps": [[0, 1], [6, 2], [3, 4], [8, 5], [7, 9]], "cuts": [], "open": []}
    bits = random_bitstrings(4, 6, 3)
    row1 = _row_circuit(c, 1).to_text()
    for b in range(4):
        t, labels = tn.partial_contract(c.to_text(), bits[b], plan, 0, subset=[2, 3])
        assert labels == []
        want = sv.amplitudes(row1, bits[b:b + 1, 3:])[0]
        assert abs(complex(t) - want) <= 1e-13
        # and the whole plan gives the product of the two rows' amplitudes
        row0 = _row_circuit(c, 0).to_text()
        whole = tn.amplitudes(c.to_text(), bits[b:b + 1], plan)[0, 0]
        assert abs(whole - want * sv.amplitudes(row0, bits[b:b + 1, :3])[0]) <= 1e-13


def test_porter_thomas_exact_exponential_quantiles():
    """N p at the midpoint quantiles of Exp(1): the empirical CDF steps straddle 1 - e^-x by
    exactly 1/(2m), and the moments are midpoint sums of int_0^1 (-ln(1-u))^k du = k!."""
    m, n = 1 << 20, 30
    x = -np.log1p(-(np.arange(m) + 0.5) / m)
    rng = np.random.default_rng(0)
    amps = np.sqrt(x / 2.0 ** n) * np.exp(2j * np.pi * rng.random(m))  # phases do not matter
    m1, m2, ks = porter_thomas(rng.permutation(amps), n)
    assert abs(ks - 0.5 / m) <= 1e-9
    assert abs(m1 - 1.0) <= 1e-5
    assert abs(m2 - 2.0) <= 2e-4


def test_porter_thomas_uniform_and_point_mass():
    """N p uniform on [0, 2]: KS = sup |x/2 - (1 - e^-x)| = 1/2 - ln(2)/2 at x = ln 2, moments
    1 and 4/3.  N p = 1 for every bitstring: KS = max(e^-1, 1 - e^-1), moments 1 and 1."""
    m, n = 1 << 18, 20
    x = 2.0 * (np.arange(m) + 0.5) / m
    m1, m2, ks = porter_thomas(np.sqrt(x / 2.0 ** n), n)
    assert abs(ks - (0.5 - 0.5 * np.log(2.0))) <= 2.0 / m
    assert abs(m1 - 1.0) <= 1e-9 and abs(m2 - 4.0 / 3.0) <= 1e-9
    m1, m2, ks = porter_thomas(np.full(1000, 2.0 ** -(n / 2)), n)
    assert abs(ks - (1.0 - np.exp(-1.0))) <= 1e-12
    assert abs(m1 - 1.0) <= 1e-12 and abs(m2 - 1.0) <= 1e-12


def test_rel_err_is_normwise():
    ref = np.array([3.0, 4.0j])
    assert rel_err(ref + np.array([0.3, 0.4j]), ref) == pytest.approx(0.1, rel=1e-14)
    assert rel_err(np.array([1e-3, 0.0]), np.zeros(2)) == pytest.approx(1e-3, rel=1e-14)


def test_fd_through_tensor_network_matches_adjoint():
    """The finite-difference gradient of sum |a|^2 through oracle-TN (with a cut and an open qubit)
    equals the adjoint state-vector gradient with cotangent 2a over every completion."""
    c = generate(2, 3, 16, 3)
    text = c.to_text()
    qid = c.qubit_of()
    plan = sweep_plan(c, open_qubits=[5], cuts=[[qid[(0, 1)], qid[(1, 1)], 0, 1]])
    bits = random_bitstrings(3, 6, 4)
    full = np.repeat(bits, 2, axis=0)
    full[:, 5] = np.tile([0, 1], 3)
    a = sv.amplitudes(text, full)
    ref = grad.adjoint_gradient(text, full, 2 * a)
    one_q = [i for i, op in enumerate(c.ops) if len(op.qubits) == 1]
    two_q = [i for i, op in enumerate(c.ops) if len(op.qubits) == 2]
    for op in (one_q[0], one_q[len(one_q) // 2], one_q[-1], two_q[0], two_q[-1]):
        for e in range(4):
            got = grad.fd_norm_loss_tn(text, bits, plan, op, e, h=0.3)
            assert abs(got - np.asarray(ref[op]).reshape(-1)[e]) <= 1e-12, (op, e)
