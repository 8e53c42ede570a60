"""Frugal rejection sampling and XEB scoring on exact amplitudes of a deep 4x4 circuit."""
import numpy as np

from oracle import sv
from paper_1905_00444_amd.sampling import frugal_rejection_sample, xeb_linear, xeb_log, complete
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate


def _setup():
    c = generate(4, 4, 32, 3).to_text()
    psi = sv.final_state(c)
    return c, psi


def test_complete_orders_open_qubits_msb_first():
    x = complete(np.zeros(6, dtype=np.uint8), [4, 1], 2)
    assert list(x) == [0, 0, 0, 0, 1, 0]


def test_rejection_samples_score_like_ideal_samples():
    c, psi = _setup()
    n = 16
    open_q = list(range(10, 16))
    prefixes = random_bitstrings(3000, n, 5)
    amps = sv.open_amplitudes(c, prefixes, open_q)
    samples, ok = frugal_rejection_sample(amps, prefixes, open_q, n, M=10.0, rng=np.random.default_rng(0))
    assert ok.mean() > 0.9
    p = np.abs(psi[sv.bit_index(samples[ok])]) ** 2
    # ideal (Porter-Thomas) sampling gives linear XEB ~ 1 and log XEB ~ 1
    assert abs(xeb_linear(p, n) - 1.0) < 0.15
    assert abs(xeb_log(p, n) - 1.0) < 0.15
    # uniformly drawn bitstrings score ~ 0
    pu = np.abs(psi[sv.bit_index(random_bitstrings(3000, n, 9))]) ** 2
    assert abs(xeb_linear(pu, n)) < 0.1
    assert abs(xeb_log(pu, n)) < 0.1


def test_exact_distribution_when_one_try_per_pass():
    """With one candidate per pass the accepted samples follow p exactly (small circuit)."""
    c = generate(2, 3, 16, 1).to_text()
    psi = sv.final_state(c)
    n = 6
    open_q = [0, 1, 2, 3, 4, 5]
    prefixes = np.zeros((40000, n), dtype=np.uint8)
    amps = np.tile(psi, (40000, 1))
    samples, ok = frugal_rejection_sample(amps, prefixes, open_q, n, M=12.0, rng=np.random.default_rng(1),
                                          tries_per_pass=1)
    idx = sv.bit_index(samples[ok])
    counts = np.bincount(idx, minlength=64) / ok.sum()
    p = np.abs(psi) ** 2
    assert np.max(np.abs(counts - p)) < 5 * np.sqrt(p.max() / ok.sum()) + 1e-3
