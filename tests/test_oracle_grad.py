"""Pin of the adjoint gradient: central finite differences of a loss that is
linear in every gate entry, so the differences carry no truncation error."""
import numpy as np

from oracle import grad, sv
from oracle.parse import read_circuit
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate


def test_adjoint_matches_exact_finite_differences():
    c = generate(2, 3, 8, 2)
    circ = read_circuit(c.to_text())
    bits = random_bitstrings(4, 6, 1)
    rng = np.random.default_rng(0)
    cot = rng.normal(size=4) + 1j * rng.normal(size=4)
    g = grad.adjoint_gradient(circ, bits, cot)
    two_q = [i for i, (_, _, qs) in enumerate(circ.ops) if len(qs) == 2]
    one_q = [i for i, (_, _, qs) in enumerate(circ.ops) if len(qs) == 1]
    for i in one_q[:3] + one_q[-2:] + two_q[:3]:
        fd = grad.fd_gradient(circ, bits, cot, i, h=0.37)
        assert np.allclose(g[i], fd, atol=1e-11), i


def test_norm_loss_gradient_is_2a():
    # for L = sum |a|^2 the cotangent is 2a; the gradient of the last H layer
    # gate on qubit q equals sum_b 2 a_b conj(d a_b / d H)
    c = generate(2, 2, 8, 5)
    circ = read_circuit(c.to_text())
    bits = random_bitstrings(3, 4, 2)
    a = sv.amplitudes(circ, bits)
    g = grad.adjoint_gradient(circ, bits, 2 * a)
    # L = sum |a|^2 is quadratic; central FD of it is exact too
    i = len(circ.ops) - 1
    h = 0.1
    fd = np.zeros((2, 2), dtype=np.complex128)
    for idx in np.ndindex(2, 2):
        for step, w in ((h, 1), (1j * h, 1j)):
            vp = [v.copy() for v in circ.values]
            vm = [v.copy() for v in circ.values]
            vp[i][idx] += step
            vm[i][idx] -= step
            lp = np.sum(np.abs(sv.amplitudes(circ.with_values(vp), bits)) ** 2)
            lm = np.sum(np.abs(sv.amplitudes(circ.with_values(vm), bits)) ** 2)
            fd[idx] += w * (lp - lm) / (2 * h)
    assert np.allclose(g[i], fd, atol=1e-12)
