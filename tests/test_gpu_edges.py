"""Edge cases of the amplitude path on the GPU, through the C-ABI: empty bitstring batches and
empty slice ranges (no-ops that leave the caller's accumulator untouched), slice ranges past the
plan's slices (errors), the depth-0 circuit (an H layer then an H layer: no bonds at all, every
contraction an outer product with K = 1; a(x) = 1 at x = 0 and 0 elsewhere, exactly), and the
smallest grids (two qubits, one bond)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

PRECISIONS = ["fp32", "bf16x3", "fp16"]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


def _say(msg):
    print(msg, flush=True)


def _cut_plan():
    """4x4 (1+16+1), bond 4: a 2-bit cut on one bond (4 slices), two open qubits."""
    from workloads.circuits import generate
    from workloads.plans import region_plan
    c = generate(4, 4, 16, 3)
    qid = c.qubit_of()
    q0, q1 = sorted((qid[(1, 1)], qid[(1, 2)]))
    plan, _ = region_plan(c, 2, 2, [[q0, q1, 0, 2]], [(3, 2), (3, 3)])
    return c, plan


def test_empty_batch_and_empty_slice_range_leave_the_accumulator_untouched(ctx):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    from workloads.bitstrings import random_bitstrings
    _say("empty batch / empty slice range")
    c, plan = _cut_plan()
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, "bf16x3")
    assert p.info()["n_slices"] == 4
    bits = random_bitstrings(3, 16, 5)
    sentinel = torch.full((3, 4), 0.25 - 0.5j, dtype=torch.complex128, device="cuda")
    out = sentinel.clone()
    p.amplitudes(bits, 2, 2, out=out)          # empty slice range
    p.amplitudes(bits[:0], 0, 4, out=out[:0])  # empty batch
    torch.cuda.synchronize()
    assert torch.equal(out, sentinel)
    # and a non-empty call still accumulates on top of what is there
    ref = p.amplitudes(bits)
    p.amplitudes(bits, out=out)
    torch.cuda.synchronize()
    assert torch.equal(out - sentinel, ref)


def test_slice_range_past_the_plan_is_an_error(ctx):
    from paper_1905_00444_amd import Circuit, Plan
    from workloads.bitstrings import random_bitstrings
    _say("slice range errors")
    c, plan = _cut_plan()
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, "fp32")
    bits = random_bitstrings(2, 16, 6)
    for s_begin, s_end in ((0, 5), (3, 2), (-1, 2)):
        with pytest.raises(RuntimeError):
            p.amplitudes(bits, s_begin, s_end)


@pytest.mark.parametrize("precision", PRECISIONS)
def test_depth_zero_circuit_is_a_delta(ctx, precision):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    from workloads.circuits import generate
    from workloads.plans import sweep_plan
    from workloads.bitstrings import random_bitstrings
    _say(f"depth-0 circuit {precision}")
    c = generate(4, 4, 0, 0)
    plan = sweep_plan(c, open_qubits=[15, 14, 13])
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, precision)
    bits = random_bitstrings(8, 16, 2)
    bits[0, :] = 0
    got = p.amplitudes(bits)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    ref = np.zeros_like(got)
    for b in range(bits.shape[0]):
        if not bits[b, :13].any():
            ref[b, 0] = 1.0  # open qubits 15, 14, 13 all 0 is column 0
    # H H = I in every precision: the H entries 1/sqrt(2) multiply to 1/2 exactly in FP32 only
    # up to rounding, so compare to a tight bound rather than bitwise
    tol = {"fp32": 1e-6, "bf16x3": 1e-5, "fp16": 2e-3}[precision]
    assert np.max(np.abs(got - ref)) <= tol


@pytest.mark.parametrize("shape", [(1, 2), (2, 1)])
@pytest.mark.parametrize("precision", PRECISIONS)
def test_two_qubit_grids_match_the_state_vector(ctx, shape, precision):
    import torch
    from oracle import sv
    from paper_1905_00444_amd import Circuit, Plan
    from workloads.circuits import generate
    from workloads.plans import sweep_plan
    _say(f"two-qubit grid {shape} {precision}")
    c = generate(shape[0], shape[1], 16, 4)
    plan = sweep_plan(c)
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, precision)
    bits = np.array([[0, 0], [0, 1], [1, 0], [1, 1]], dtype=np.uint8)
    got = p.amplitudes(bits)
    torch.cuda.synchronize()
    ref = sv.amplitudes(c.to_text(), bits)
    tol = {"fp32": 1e-6, "bf16x3": 1e-5, "fp16": 2e-3}[precision]
    assert np.max(np.abs(got.cpu().numpy()[:, 0] - ref)) <= tol
    # the four amplitudes of a two-qubit state have unit norm
    assert abs(np.sum(np.abs(got.cpu().numpy()) ** 2) - 1.0) <= 10 * tol
