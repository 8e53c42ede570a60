"""Pins of the state-vector oracle against things other than itself:
algebraic identities of the gate table, brute-force Kronecker products of the
full unitaries, closed-form small circuits, unitarity and Porter-Thomas."""
import numpy as np
import pytest

from oracle import gates, sv
from oracle.parse import read_circuit
from oracle.metrics import porter_thomas
from workloads.circuits import generate, mirror, Circuit, Op


def test_gate_table_algebra():
    I = np.eye(2)
    H, T, S = gates.one_qubit("h"), gates.one_qubit("t"), gates.one_qubit("s")
    X = np.array([[0, 1], [1, 0]])
    Y = np.array([[0, -1j], [1j, 0]])
    assert np.allclose(H @ H, I)
    assert np.allclose(T @ T, S)
    assert np.allclose(np.linalg.matrix_power(T, 8), I)
    assert np.allclose(gates.one_qubit("x_1_2") @ gates.one_qubit("x_1_2"), X)
    assert np.allclose(gates.one_qubit("y_1_2") @ gates.one_qubit("y_1_2"), Y)
    for name in ("h", "t", "s", "x_1_2", "y_1_2"):
        g = gates.one_qubit(name)
        assert np.allclose(g.conj().T @ g, I)
        assert np.allclose(gates.one_qubit(name + "dg") @ g, I)
    # principal square roots: eigenvalues in {1, i}
    for name in ("x_1_2", "y_1_2"):
        ev = np.sort_complex(np.linalg.eigvals(gates.one_qubit(name)))
        assert np.allclose(ev, np.sort_complex(np.array([1, 1j])))
    assert np.allclose(gates.two_qubit_diag("cz"), [1, 1, 1, -1])


def _full_unitary(circ):
    """Brute force: product of 2^n x 2^n matrices built with np.kron."""
    n = circ.n
    U = np.eye(2 ** n, dtype=np.complex128)
    for (_, _, qs), val in zip(circ.ops, circ.values):
        if len(qs) == 1:
            q = qs[0]
            M = np.kron(np.kron(np.eye(2 ** q), val), np.eye(2 ** (n - q - 1)))
        else:
            q0, q1 = qs
            if q1 == q0 + 1:
                M = np.kron(np.kron(np.eye(2 ** q0), np.diag(val)), np.eye(2 ** (n - q1 - 1)))
            else:
                # D = sum_{k} P_k(q0) (x) diag(val[2k], val[2k+1])(q1), built from krons
                M = np.zeros((2 ** n, 2 ** n), dtype=np.complex128)
                for k in range(2):
                    P = np.zeros((2, 2))
                    P[k, k] = 1
                    ops = [np.eye(2)] * n
                    ops[q0] = P
                    ops[q1] = np.diag(val[2 * k:2 * k + 2])
                    term = np.array([[1.0]])
                    for o in ops:
                        term = np.kron(term, o)
                    M = M + term
        U = M @ U
    return U


@pytest.mark.parametrize("rows,cols,depth,seed", [(2, 2, 8, 0), (2, 3, 8, 3), (3, 3, 12, 5), (2, 4, 16, 7)])
def test_sv_matches_kronecker_unitary(rows, cols, depth, seed):
    circ = read_circuit(generate(rows, cols, depth, seed).to_text())
    U = _full_unitary(circ)
    assert np.allclose(U.conj().T @ U, np.eye(2 ** circ.n), atol=1e-12)
    psi = sv.final_state(circ)
    assert np.allclose(psi, U[:, 0], atol=1e-12)


def test_unit_norm_and_probability_sum():
    circ = read_circuit(generate(4, 4, 16, 0).to_text())
    psi = sv.final_state(circ)
    assert abs(np.sum(np.abs(psi) ** 2) - 1) < 1e-12


def test_depth_zero_is_delta():
    circ = generate(3, 3, 0, 0)  # H layer then H layer
    psi = sv.final_state(circ.to_text())
    want = np.zeros(2 ** 9)
    want[0] = 1
    assert np.allclose(psi, want, atol=1e-14)


@pytest.mark.parametrize("q", [0, 3, 5])
def test_bit_order_qubit0_is_msb(q):
    n = 6
    c = Circuit(2, 3, (), [Op(0, "x_1_2", (q,)), Op(1, "x_1_2", (q,))])
    a = sv.amplitudes(c.to_text(), np.eye(n, dtype=np.uint8)[[q]])
    assert abs(abs(a[0]) - 1) < 1e-14
    psi = sv.final_state(c.to_text())
    assert abs(abs(psi[2 ** (n - 1 - q)]) - 1) < 1e-14


def test_cz_makes_bell_pair():
    # H(x)H, CZ, H on qubit 1  ->  (|00> + |11>)/sqrt 2
    c = Circuit(1, 2, (), [Op(0, "h", (0,)), Op(0, "h", (1,)), Op(1, "cz", (0, 1)), Op(2, "h", (1,))])
    psi = sv.final_state(c.to_text())
    assert np.allclose(psi, np.array([1, 0, 0, 1]) / np.sqrt(2), atol=1e-14)


def test_mirror_circuit_is_identity():
    base = generate(3, 3, 16, 4)
    m = mirror(base, 16, 4)
    psi = sv.final_state(m.to_text())
    want = np.zeros(2 ** 9)
    want[0] = 1
    assert np.allclose(psi, want, atol=1e-12)


def test_porter_thomas_deep_4x4():
    circ = generate(4, 4, 32, 11)
    psi = sv.final_state(circ.to_text())
    mean, second, ks = porter_thomas(psi, 16)
    assert abs(mean - 1) < 1e-9  # exact: all 2^n amplitudes
    assert abs(second - 2) < 0.1
    assert ks < 0.02


def test_open_amplitudes_enumerates_completions():
    circ = generate(3, 3, 8, 2).to_text()
    psi = sv.final_state(circ)
    bits = np.zeros((1, 9), dtype=np.uint8)
    bits[0, 0] = 1
    out = sv.open_amplitudes(circ, bits, [8, 4])
    # completions j: qubit 8 is the MSB of j, qubit 4 the LSB
    for j in range(4):
        b = bits[0].copy()
        b[8], b[4] = j >> 1, j & 1
        assert out[0, j] == psi[sv.bit_index(b)]
