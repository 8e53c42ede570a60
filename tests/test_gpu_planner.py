"""Plans from the automatic search run through the HIP path: exact against the state vector on
a small grid, and on the 70-qubit (8x9 minus two corners, 1+24+1) workload the searched plan
(no cuts needed at 2^27) gives the same full amplitudes as the hand plan's 256-slice sum."""
import numpy as np
import pytest

from oracle import sv
from oracle.metrics import rel_err
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import plan_8x9, C5_REMOVED

pytestmark = pytest.mark.gpu


def test_searched_plan_with_cuts_vs_state_vector():
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, planner
    print("searched plan 4x5", flush=True)
    c = generate(4, 5, 32, 2)
    text = c.to_text()
    free = planner.search(text, 40)
    best = planner.search(text, free.peak_bits - 3, [(3, 4), (2, 4)])
    assert best.n_slices > 1
    ctx = Context(0)
    bits = random_bitstrings(4, 20, 12)
    got = Plan(ctx, Circuit(ctx, text), best.plan, "fp32").amplitudes(bits)
    torch.cuda.synchronize()
    assert rel_err(got.cpu().numpy(), sv.open_amplitudes(text, bits, best.plan["open"])) <= 1e-5


def test_70_qubit_searched_plan_equals_hand_plan_path_sum():
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, planner
    print("70 qubits: searched plan vs 256-slice hand plan", flush=True)
    c = generate(8, 9, 24, 0, C5_REMOVED)
    text = c.to_text()
    hand, _ = plan_8x9(c)
    best = planner.search(text, 27)
    assert best.peak_bits <= 27
    ctx = Context(0)
    circ = Circuit(ctx, text)
    bits = random_bitstrings(2, 70, 1)
    a = Plan(ctx, circ, best.plan, "fp32").amplitudes(bits)
    b = Plan(ctx, circ, hand, "fp32").amplitudes(bits)
    torch.cuda.synchronize()
    a, b = a.cpu().numpy(), b.cpu().numpy()
    assert np.all(np.abs(b) > 0)
    assert rel_err(a, b) <= 2e-5
