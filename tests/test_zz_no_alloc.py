"""qf_amplitudes_static (the entry point that allocates nothing: every tensor of the plan in the
library's own device array) against qf_amplitudes on the same plans and inputs, through the
C-ABI: two calls in a row, the second with a smaller input, and against the FP64 oracle."""
import ctypes as C

import numpy as np
import pytest

from oracle import sv
from oracle.metrics import rel_err
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import region_plan, sweep_plan

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


def _4x5(ctx, precision, batch=1):
    from paper_1905_00444_amd import Circuit, Plan
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4), (3, 3)])
    return c, plan, Plan(ctx, Circuit(ctx, c.to_text()), plan, precision, batch=batch)


def test_static_scratch_size_is_reported(ctx):
    from paper_1905_00444_amd import _lib
    n = C.c_size_t()
    assert _lib.load().qf_static_scratch_bytes(C.byref(n)) == 0
    assert n.value == 64 << 20


@pytest.mark.parametrize("precision,batch", [("fp32", 1), ("bf16x3", 1), ("bf16x3", 2)])
def test_static_entry_equals_qf_amplitudes_two_calls(ctx, precision, batch):
    """4x5 (1+32+1) with two cuts (16 slices) and three open qubits: a first call over 6 prefixes
    and every slice, then a smaller one (2 prefixes, slices 3..8); both bitwise equal to
    qf_amplitudes on the context's workspace and within the FP64 bounds of the oracle."""
    import torch
    _say(f"static scratch vs qf_amplitudes, 4x5 regions, {precision}, {batch} chains per launch")
    c, plan, p = _4x5(ctx, precision, batch)
    bits1 = random_bitstrings(6, 20, 3)
    bits2 = random_bitstrings(2, 20, 4)
    for bits, rng in ((bits1, (0, 16)), (bits2, (3, 9))):
        ref = p.amplitudes(bits, *rng)
        got = p.amplitudes_static(torch.from_numpy(bits).cuda(), *rng)
        torch.cuda.synchronize()
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
    full = sv.open_amplitudes(c.to_text(), bits1, plan["open"])
    got = p.amplitudes_static(torch.from_numpy(bits1).cuda())
    torch.cuda.synchronize()
    assert rel_err(got.cpu().numpy(), full) <= {"fp32": 1e-5, "bf16x3": 1e-4}[precision]


def test_static_entry_across_plans_and_after_the_workspace_path(ctx):
    """The 6x6 (1+24+1) sweep (49 MiB of the 64) then the smaller 4x4 (1+16+1) plan in the same
    array, then the first plan again on its own workspace: each result equals qf_amplitudes."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("static scratch across plans")
    c6 = generate(6, 6, 24, 0)
    p6 = Plan(ctx, Circuit(ctx, c6.to_text()), sweep_plan(c6), "fp32")
    assert p6.info()["workspace_bytes"] > 32 << 20
    c4 = generate(4, 4, 16, 0)
    p4 = Plan(ctx, Circuit(ctx, c4.to_text()), sweep_plan(c4, open_qubits=[15, 14]), "bf16x3")
    b6 = random_bitstrings(8, 36, 1)
    b4 = random_bitstrings(3, 16, 2)
    g6 = p6.amplitudes_static(torch.from_numpy(b6).cuda())
    g4 = p4.amplitudes_static(torch.from_numpy(b4).cuda())
    r6 = p6.amplitudes(b6)
    r4 = p4.amplitudes(b4)
    torch.cuda.synchronize()
    assert np.array_equal(g6.cpu().numpy(), r6.cpu().numpy())
    assert np.array_equal(g4.cpu().numpy(), r4.cpu().numpy())
    assert rel_err(g4.cpu().numpy(), sv.open_amplitudes(c4.to_text(), b4, [15, 14])) <= 1e-4


def test_static_entry_refuses_plans_beyond_the_array_and_graph_plans(ctx):
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, _lib
    _say("static scratch refusals")
    c = generate(4, 4, 40, 0)
    plan, _ = region_plan(c, 2, 2, [], [(3, 2), (3, 3)])
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, "fp32")
    assert p.info()["workspace_bytes"] > 64 << 20
    bits = torch.zeros((1, 16), dtype=torch.uint8, device="cuda")
    out = torch.zeros((1, 4), dtype=torch.complex128, device="cuda")
    st = ctx.lib.qf_amplitudes_static(p.h, 1, C.c_void_p(bits.data_ptr()), 0, 1, C.c_void_p(out.data_ptr()))
    assert st == _lib.QF_ERR_WORKSPACE
    gctx = Context(0, stream=torch.cuda.Stream())
    _, plan5, _ = _4x5(ctx, "fp32")
    c5 = generate(4, 5, 32, 2)
    g = Plan(gctx, Circuit(gctx, c5.to_text()), plan5, "fp32", batch=2, graph=True)
    bits = torch.zeros((1, 20), dtype=torch.uint8, device="cuda")
    out = torch.zeros((1, 8), dtype=torch.complex128, device="cuda")
    st = gctx.lib.qf_amplitudes_static(g.h, 1, C.c_void_p(bits.data_ptr()), 0, 1, C.c_void_p(out.data_ptr()))
    assert st == _lib.QF_ERR_UNSUPPORTED
