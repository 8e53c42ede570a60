"""Batched chains (G bitstring x slice pairs per launch) and their hipGraph replay: identical
to the one-chain-at-a-time path, and correct against the oracle and closed forms, including
the 70-qubit (8x9 minus two corners, 1+24+1) workload's shapes."""
import numpy as np
import pytest

from oracle import sv
from oracle.metrics import rel_err
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate, identity_cz
from workloads.plans import region_plan, plan_8x9, C5_REMOVED

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


@pytest.fixture(scope="module")
def gctx():
    """A context on a non-default stream (graph capture needs one)."""
    import torch
    from paper_1905_00444_amd import Context
    return Context(0, stream=torch.cuda.Stream())


def _setup_4x5():
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    return c, plan


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("G", [2, 8])
def test_batched_equals_sequential_bitwise(ctx, precision, G):
    """With group hoisting off, the batched path runs every step of every chain with the same
    kernels and shapes as the one-chain path: bitwise equal."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say(f"batched G={G} {precision}")
    c, plan = _setup_4x5()
    bits = random_bitstrings(3, 20, 5)  # 3 x 16 = 48 chains: 48 / 8 leaves no tail, 48 / 32 would
    circ = Circuit(ctx, c.to_text())
    seq = Plan(ctx, circ, plan, precision, hoist=False).amplitudes(bits)
    bat = Plan(ctx, circ, plan, precision, batch=G, hoist=False).amplitudes(bits)
    torch.cuda.synchronize()
    assert np.array_equal(seq.cpu().numpy(), bat.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
@pytest.mark.parametrize("G", [2, 8, 32])
def test_group_hoisting_matches_sequential_and_state_vector(ctx, precision, G):
    """Batched plans with cuts (default): the steps that depend on no cut run once per launch
    group, a shared operand is taken as B and the group's chains stack along M.  Different GEMM
    shapes and operand roles accumulate in another order and split their operands in other
    kernels, so the comparison with the one-chain path is within rounding: FP32 2e-6 norm-wise,
    split-BF16 2e-5 (each operand is represented to about 2^-17 relative, and the two paths
    round their splits independently); both meet the state-vector bounds."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say(f"group hoisting G={G} {precision}")
    c, plan = _setup_4x5()
    bits = random_bitstrings(3, 20, 5)
    circ = Circuit(ctx, c.to_text())
    seq = Plan(ctx, circ, plan, precision).amplitudes(bits)
    bp = Plan(ctx, circ, plan, precision, batch=G)
    bat = bp.amplitudes(bits)
    torch.cuda.synchronize()
    seq, bat = seq.cpu().numpy(), bat.cpu().numpy()
    assert rel_err(bat, seq) <= {"fp32": 2e-6, "bf16x3": 2e-5}[precision]
    ref = sv.open_amplitudes(c.to_text(), bits, plan["open"])
    bound = 1e-5 if precision == "fp32" else 1e-4
    assert rel_err(seq, ref) <= bound and rel_err(bat, ref) <= bound
    # the executed flops count each group's cut-independent steps once
    S = bp.info()["n_slices"]
    assert bp.flops(0, S) < S * bp.info()["flops_per_slice"]


def test_batched_tail_and_slice_subrange(ctx):
    """Chains that do not fill the last group are masked; slice sub-ranges compose.  Group
    hoisting puts each bitstring's slices in groups of their own (7 slices of 3 bitstrings in
    groups of 8: one partly idle group per bitstring)."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("batched tail")
    c, plan = _setup_4x5()
    bits = random_bitstrings(3, 20, 6)
    circ = Circuit(ctx, c.to_text())
    seq = Plan(ctx, circ, plan, "fp32", hoist=False).amplitudes(bits, 3, 10)  # 21 chains
    bat = Plan(ctx, circ, plan, "fp32", batch=8, hoist=False).amplitudes(bits, 3, 10)
    hst = Plan(ctx, circ, plan, "fp32", batch=8).amplitudes(bits, 3, 10)
    torch.cuda.synchronize()
    assert np.array_equal(seq.cpu().numpy(), bat.cpu().numpy())
    assert rel_err(hst.cpu().numpy(), seq.cpu().numpy()) <= 2e-6
    ref = sv.open_amplitudes(c.to_text(), bits, plan["open"])
    full = Plan(ctx, circ, plan, "fp32", batch=8)
    parts = full.amplitudes(bits, 0, 5)
    full.amplitudes(bits, 5, 16, out=parts)
    whole = full.amplitudes(bits)
    torch.cuda.synchronize()
    assert rel_err(whole.cpu().numpy(), ref) <= 1e-5
    assert rel_err(parts.cpu().numpy(), whole.cpu().numpy()) <= 2e-6


def test_graph_replays_match_eager(gctx):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("graph replay")
    c, plan = _setup_4x5()
    bits = random_bitstrings(4, 20, 7)
    circ = Circuit(gctx, c.to_text())
    eager = Plan(gctx, circ, plan, "bf16x3", batch=4)
    graph = Plan(gctx, circ, plan, "bf16x3", batch=4, graph=True)
    ref = eager.amplitudes(bits)
    gctx.synchronize()
    ref = ref.cpu().numpy()
    bits_t = torch.from_numpy(bits).to(gctx.device)
    with torch.cuda.stream(gctx.stream):
        out = torch.zeros((4, 4), dtype=torch.complex128, device=gctx.device)
    n_chains = 4 * graph.info()["n_slices"]
    assert n_chains // 4 >= 8  # several groups of 4 chains per call
    for rep in range(4):
        with torch.cuda.stream(gctx.stream):
            out.zero_()
        graph.amplitudes(bits_t, out=out)  # same pointers every time: the captured graph is replayed
        gctx.synchronize()
        assert np.array_equal(out.cpu().numpy(), ref), rep
        # the whole call, every group of 4 chains, is one graph launch
        launches, nodes = graph.graph_info()
        assert launches == rep + 1
        assert nodes > n_chains // 4
        # eager work between replays
        eager.amplitudes(bits)
        gctx.synchronize()


def _product_slice(circ, plan, bits_row, s):
    from oracle import gates
    total = sum(x[3] for x in plan["cuts"])
    fixed = {}
    off = total
    for q0, q1, lo, nb in plan["cuts"]:
        off -= nb
        v = (s >> off) & ((1 << nb) - 1)
        for i in range(nb):
            fixed[(q0, q1, lo + i)] = (v >> (nb - 1 - i)) & 1
    vecs = [np.array([1, 0], dtype=np.complex128) for _ in range(circ.n_qubits)]
    seen = {}
    for op in circ.ops:
        if len(op.qubits) == 1:
            vecs[op.qubits[0]] = gates.one_qubit(op.name) @ vecs[op.qubits[0]]
        else:
            j = seen.get(op.qubits, 0)
            seen[op.qubits] = j + 1
            if op.qubits + (j,) in fixed:
                q0 = op.qubits[0]
                vecs[q0] = vecs[q0] * (np.arange(2) == fixed[op.qubits + (j,)])
    return np.prod([vecs[q][bits_row[q]] for q in range(circ.n_qubits)])


def _clifford_batch(base, plan, n, seed):
    """Clifford product circuit (CZ -> identity, T -> S) and n bitstrings with nonzero slice-0
    amplitudes: the larger component of every qubit, then random flips of the qubits whose two
    components are equal in magnitude (see the 7x7 product test for why split-BF16 needs it)."""
    from test_gpu_amplitudes import _product_vectors
    from workloads.circuits import clifford_substitute
    c = clifford_substitute(identity_cz(base))
    vecs = _product_vectors(c, plan, 0)
    first = np.array([int(np.argmax(np.abs(v))) for v in vecs], dtype=np.uint8)
    cut_q = {q for cut in plan["cuts"] for q in cut[:2]}
    free = [q for q, v in enumerate(vecs) if q not in cut_q and abs(abs(v[0]) - abs(v[1])) < 1e-12]
    rng = np.random.default_rng(seed)
    bits = np.tile(first, (n, 1))
    for b in range(1, n):
        bits[b, free] ^= rng.integers(0, 2, len(free)).astype(np.uint8)
    return c, bits


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_70_qubit_product_circuit_batched_graph(gctx, precision):
    """8x9 minus two corners, (1+24+1), every CZ -> identity: each chain has a closed form.
    16 bitstrings x slices 0..7 run as 128 chains, 32 per launch, through the captured graph.
    Split-BF16 runs the Clifford variant."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say(f"70 qubits product circuit {precision}")
    base = generate(8, 9, 24, 0, C5_REMOVED)
    plan, _ = plan_8x9(base)
    if precision == "bf16x3":
        c, bits = _clifford_batch(base, plan, 16, 1)
    else:
        c = identity_cz(base)
        bits = random_bitstrings(16, 70, 1)
    p = Plan(gctx, Circuit(gctx, c.to_text()), plan, precision, batch=32, graph=True)
    got = p.amplitudes(bits, 0, 8)
    gctx.synchronize()
    ref = np.array([sum(_product_slice(c, plan, bits[b], s) for s in range(8)) for b in range(16)])
    assert np.count_nonzero(ref) >= 8
    assert rel_err(got.cpu().numpy()[:, 0], ref) <= (1e-5 if precision == "fp32" else 1e-4)


def test_70_qubit_random_circuit_batched_vs_oracle_one_chain(gctx):
    """One chain (bitstring 0, slice 5) of the random 70-qubit circuit against the FP64
    tensor-network oracle, through the batched graph path."""
    import torch
    from oracle import tn
    from paper_1905_00444_amd import Circuit, Plan
    _say("70 qubits random, one chain vs oracle")
    c = generate(8, 9, 24, 0, C5_REMOVED)
    plan, _ = plan_8x9(c)
    bits = random_bitstrings(1, 70, 1)
    p = Plan(gctx, Circuit(gctx, c.to_text()), plan, "fp32", batch=2, graph=True)
    got = p.amplitudes(bits, 5, 6)
    gctx.synchronize()
    ref = tn.amplitudes(c.to_text(), bits, plan, slices=[5])
    assert rel_err(got.cpu().numpy(), ref) <= 1e-5
