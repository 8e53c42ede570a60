"""Noisy simulation by partial path sums (paper Sec. III-C): the oracle's per-path states are
pinned against the full evolution and the tensor-network slices, the fidelity ~ f property is
checked on the oracle, and the host bookkeeping of the package's fidelity module is checked on
closed forms."""
import numpy as np
import pytest

from oracle import sv, tn
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import region_plan


def _setup(seed, depth=32):
    c = generate(4, 4, depth, seed)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 3), (2, 3)])
    return c, plan


def test_sliced_states_sum_to_final_state():
    c, plan = _setup(2)
    text = c.to_text()
    psi = sv.final_state(text)
    acc = sum(sv.sliced_state(text, plan["cuts"], s) for s in range(16))
    assert np.max(np.abs(acc - psi)) <= 1e-13
    # each path is a genuine part: none is the whole state or zero
    one = sv.sliced_state(text, plan["cuts"], 5)
    assert 1e-3 < np.linalg.norm(one) < 0.9


def test_sliced_state_matches_tensor_network_slice():
    """Two routes to one path: direct evolution with the split gate's term, and the sliced
    world-line contraction."""
    c, plan = _setup(3)
    text = c.to_text()
    bits = random_bitstrings(2, 16, 9)
    opn = plan["open"]
    for s in (0, 6, 15):
        psi_s = sv.sliced_state(text, plan["cuts"], s)
        for b in range(2):
            want = tn.slice_amplitudes(text, bits[b], plan, s)
            x = bits[b].astype(np.int64).copy()
            got = np.empty(4, dtype=np.complex128)
            for j in range(4):
                x[opn[0]], x[opn[1]] = (j >> 1) & 1, j & 1
                got[j] = psi_s[sv.bit_index(x)]
            assert np.max(np.abs(got - want)) <= 1e-14 + 1e-11 * np.max(np.abs(want))


def test_sliced_state_rejects_nothing_when_no_cuts():
    c, _ = _setup(2)
    text = c.to_text()
    assert np.array_equal(sv.sliced_state(text, [], 0), sv.final_state(text))


@pytest.mark.parametrize("seed,depth", [(2, 32), (4, 40), (7, 24)])
def test_fraction_of_paths_has_fidelity_f(seed, depth):
    """Random circuits: the first m of 16 paths give overlap and norm fidelities close to m/16."""
    from paper_1905_00444_amd.fidelity import overlap_fidelity, norm_fidelity
    c, plan = _setup(seed, depth)
    text = c.to_text()
    psi = sv.final_state(text)
    states = [sv.sliced_state(text, plan["cuts"], s) for s in range(16)]
    for m in (1, 2, 4, 8, 12):
        part = sum(states[:m])
        assert abs(overlap_fidelity(part, psi) - m / 16) <= 0.03, m
        assert abs(norm_fidelity(part, psi) - m / 16) <= 0.03, m


def test_fidelity_host_bookkeeping():
    from paper_1905_00444_amd.fidelity import (paths_for_fidelity, slice_runs, overlap_fidelity,
                                               norm_fidelity, sampling_fidelity)
    assert paths_for_fidelity(1024, 0.005) == 6
    assert paths_for_fidelity(16, 1.0) == 16
    assert paths_for_fidelity(16, 1e-9) == 1
    with pytest.raises(ValueError):
        paths_for_fidelity(16, 0.0)
    assert slice_runs([5, 3, 4, 9, 10, 3]) == [(3, 6), (9, 11)]
    assert slice_runs([]) == []
    rng = np.random.default_rng(0)
    a = rng.normal(size=64) + 1j * rng.normal(size=64)
    assert overlap_fidelity(0.25 * a, a) == pytest.approx(0.25, abs=1e-15)
    assert norm_fidelity(0.5 * a, a) == pytest.approx(0.25, abs=1e-15)
    assert sampling_fidelity(0.1, 0.5) == pytest.approx(0.05)
