"""The HIP path through the C-ABI against FP64 values of the tensor-network oracle, stored in
tests/golden by tests/golden/make_goldens.py (which calls only the oracle package), at the full
sizes of the benchmark configurations:
  * 7x7 (1+40+1), bond 32: one nonvanishing slice of prefix 0 of the region plan with its two
    corner cuts (64 amplitudes, tensors up to 2^30 elements), in FP32, split-BF16 and FP16;
  * 8x9 minus two corners (70 qubits, 1+24+1): 16 whole amplitudes, through the 256-slice hand
    plan (batched chains, captured graph) and through the searched uncut plan;
  * 6x6 (1+24+1): 64 amplitudes and 16 entries of the gradient of sum |a|^2, the oracle's by exact
    central differences.
Bounds: FP32 1e-5 and split-BF16 1e-4 norm-wise; FP16 n 2^-11 for n contractions (each rounds
its operands to an 11-bit significand once), the analogue of the split-BF16 drift reading."""
import os

import numpy as np
import pytest

from oracle.metrics import rel_err
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import plan_7x7, plan_8x9, sweep_plan, C5_REMOVED

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _say(msg):
    print(msg, flush=True)


def _golden(name):
    path = os.path.join(GOLDEN, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated yet (tests/golden/make_goldens.py)")
    return np.load(path)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
def test_7x7_d40_slice_vs_fp64_oracle(ctx, precision):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    g = _golden("c4_slice.npz")
    circ = generate(7, 7, 40, 0)
    plan, _ = plan_7x7(circ, 40)
    bits = random_bitstrings(64, 49, 1)[:1]
    assert np.array_equal(g["bits"], bits[0])
    s = int(g["slice"])
    _say(f"7x7 d40 slice {s} of prefix 0 vs FP64 oracle, {precision}")
    p = Plan(ctx, Circuit(ctx, circ.to_text()), plan, precision)
    got = p.amplitudes(bits, s, s + 1)
    torch.cuda.synchronize()
    bound = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16": len(plan["steps"]) * 2.0 ** -11}[precision]
    err = rel_err(got.cpu().numpy()[0], g["amps"])
    _say(f"  rel err {err:.3e} (bound {bound:.1e})")
    assert err <= bound


def test_70_qubit_hand_plan_path_sums_vs_fp64_oracle():
    """All 256 slices of the two-halves hand plan for 4 of the 16 bitstrings (1024 chains in launch
    groups of 256 slices of one bitstring, the benchmark's configuration; one captured graph on a
    side stream), split-BF16."""
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan
    _say("70 qubits, hand plan, 4 bitstrings x 256 slices vs FP64 oracle")
    ctx = Context(0, stream=torch.cuda.Stream())
    g = _golden("c5_amplitudes.npz")
    circ = generate(8, 9, 24, 0, C5_REMOVED)
    bits = random_bitstrings(16, 70, 1)
    assert np.array_equal(g["bits"], bits)
    hand, _ = plan_8x9(circ)
    p = Plan(ctx, Circuit(ctx, circ.to_text()), hand, "bf16x3", batch=256, graph=True)
    with torch.cuda.stream(p.ctx.stream):
        bt = torch.from_numpy(bits[:4]).to(p.ctx.device)
    got = p.amplitudes(bt)
    p.ctx.synchronize()
    assert p.graph_info()[0] == 1
    assert rel_err(got.cpu().numpy()[:, 0], g["amps"][:4]) <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_70_qubit_searched_plan_vs_fp64_oracle(ctx, precision):
    """The 16 whole amplitudes through the uncut plan that the search finds (peak 2^27)."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan, planner
    _say(f"70 qubits, searched plan, 16 amplitudes vs FP64 oracle, {precision}")
    g = _golden("c5_amplitudes.npz")
    circ = generate(8, 9, 24, 0, C5_REMOVED)
    text = circ.to_text()
    best = planner.search(text, 27)
    p = Plan(ctx, Circuit(ctx, text), best.plan, precision)
    got = p.amplitudes(g["bits"])
    torch.cuda.synchronize()
    assert rel_err(got.cpu().numpy()[:, 0], g["amps"]) <= {"fp32": 1e-5, "bf16x3": 1e-4}[precision]


def test_6x6_d24_gradient_vs_fp64_finite_differences(ctx):
    """64 amplitudes and the gradient of L = sum |a|^2 (cotangent 2a) on 16 seeded gate entries
    (8 of one-qubit gates, 8 diagonal entries of CZs), FP32, against the oracle's exact central
    differences through its own tensor-network contraction."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("6x6 d24 gradient vs FP64 finite differences")
    g = _golden("c2_grad.npz")
    circ = generate(6, 6, 24, 0)
    bits = random_bitstrings(64, 36, 1)
    assert np.array_equal(g["bits"], bits)
    p = Plan(ctx, Circuit(ctx, circ.to_text()), sweep_plan(circ), "fp32", backward=True)
    a = p.amplitudes(bits)
    gr = p.backward(bits, 2 * a)
    torch.cuda.synchronize()
    assert rel_err(a.cpu().numpy()[:, 0], g["amps"]) <= 1e-5
    sel = gr.cpu().numpy()[g["ops"], g["entries"]]
    assert rel_err(sel, g["grad"]) <= 1e-4
