"""Partial path sums through the HIP path (paper Sec. III-C): parity with the oracle's per-path
states, and the fidelity of a quarter of the paths measured on all 2^16 amplitudes."""
import numpy as np
import pytest

from oracle import sv
from oracle.metrics import rel_err
from workloads.bitstrings import all_bitstrings, random_bitstrings
from workloads.circuits import generate
from workloads.plans import sweep_plan

pytestmark = pytest.mark.gpu


def _setup():
    c = generate(4, 4, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    return c, cuts


def test_noisy_amplitudes_match_oracle_paths():
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan
    from paper_1905_00444_amd.fidelity import noisy_amplitudes
    print("noisy amplitudes vs oracle paths", flush=True)
    ctx = Context(0)
    c, cuts = _setup()
    plan = sweep_plan(c, open_qubits=[14, 15], cuts=cuts)
    bits = random_bitstrings(8, 16, 3)
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, "fp32")
    got = noisy_amplitudes(p, bits, 0.25, paths=[0, 1, 2, 9, 7])  # first two of five -> 0, 1
    torch.cuda.synchronize()
    text = c.to_text()
    part = sv.sliced_state(text, cuts, 0) + sv.sliced_state(text, cuts, 1)
    ref = np.empty((8, 4), dtype=np.complex128)
    for b in range(8):
        x = bits[b].astype(np.int64).copy()
        for j in range(4):
            x[14], x[15] = (j >> 1) & 1, j & 1
            ref[b, j] = part[sv.bit_index(x)]
    assert rel_err(got.cpu().numpy(), ref) <= 1e-5


def test_quarter_of_paths_has_fidelity_quarter_on_all_amplitudes():
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan
    from paper_1905_00444_amd.fidelity import noisy_amplitudes, overlap_fidelity, norm_fidelity
    print("fidelity of 4 of 16 paths, all 2^16 amplitudes", flush=True)
    ctx = Context(0)
    c, cuts = _setup()
    plan = sweep_plan(c, open_qubits=list(range(8, 16)), cuts=cuts)
    prefixes = np.zeros((256, 16), dtype=np.uint8)
    prefixes[:, :8] = all_bitstrings(8)
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, "bf16x3", batch=64)
    got = noisy_amplitudes(p, prefixes, 0.25)
    torch.cuda.synchronize()
    a_f = got.cpu().numpy().reshape(-1)
    psi = sv.final_state(c.to_text())
    assert abs(overlap_fidelity(a_f, psi) - 0.25) <= 0.03
    assert abs(norm_fidelity(a_f, psi) - 0.25) <= 0.03
