"""Backward pass (environment tensors through the contraction tree, then through every
world-line) against the FP64 adjoint state-vector gradient and exact finite differences."""
import numpy as np
import pytest

from oracle import grad as ograd
from oracle import sv
from oracle.metrics import rel_err
from oracle.parse import read_circuit
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import sweep_plan, region_plan

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


def _oracle_grad(text, bits_full, cot_full):
    g = ograd.adjoint_gradient(read_circuit(text), bits_full, cot_full)
    return np.stack([np.asarray(x).reshape(4) for x in g])


def _expand_open(bits, open_q, cot):
    """Prefix rows x 2^k completions -> full bitstrings and their cotangents."""
    k = len(open_q)
    rows, cots = [], []
    for b in range(bits.shape[0]):
        for j in range(2 ** k):
            r = bits[b].copy()
            for t, q in enumerate(open_q):
                r[q] = (j >> (k - 1 - t)) & 1
            rows.append(r)
            cots.append(cot[b, j])
    return np.array(rows, dtype=np.uint8), np.array(cots)


def test_grad_4x4_d16_norm_loss_vs_adjoint_oracle(ctx):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("grad 4x4 d16")
    c = generate(4, 4, 16, 0)
    text = c.to_text()
    bits = random_bitstrings(16, 16, 1)
    p = Plan(ctx, Circuit(ctx, text), sweep_plan(c), "fp32", backward=True)
    a = p.amplitudes(bits)
    g = p.backward(bits, 2 * a)
    torch.cuda.synchronize()
    ref = _oracle_grad(text, bits, 2 * sv.amplitudes(text, bits))
    assert rel_err(g.cpu().numpy(), ref) <= 1e-4


def test_grad_4x5_d32_cuts_open_random_cotangent(ctx):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("grad 4x5 d32 cuts + open")
    c = generate(4, 5, 32, 2)
    text = c.to_text()
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 1]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    bits = random_bitstrings(3, 20, 7)
    rng = np.random.default_rng(3)
    cot = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    p = Plan(ctx, Circuit(ctx, text), plan, "fp32", backward=True)
    g = p.backward(bits, cot)
    torch.cuda.synchronize()
    fb, fc = _expand_open(bits, plan["open"], cot)
    ref = _oracle_grad(text, fb, fc)
    assert rel_err(g.cpu().numpy(), ref) <= 1e-4


@pytest.mark.parametrize("precision", ["bf16x3", "fp16"])
def test_grad_reduced_precision_vs_adjoint_oracle(ctx, precision):
    """The backward pass in split-BF16 and FP16 (the same permute and GEMM kernels as the forward,
    without renormalisation: backward plans keep true scales, and FP16 scales each GEMM's operands
    from their largest magnitudes).  Bound: the drift reading for n contractions, applied to the
    forward and reverse sweeps (2 n steps): 2 n 2^-16 for split-BF16, 2 n 2^-11 for FP16."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say(f"grad 4x5 d32 cuts + open, {precision}")
    c = generate(4, 5, 32, 2)
    text = c.to_text()
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 1]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    bits = random_bitstrings(3, 20, 7)
    rng = np.random.default_rng(3)
    cot = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    p = Plan(ctx, Circuit(ctx, text), plan, precision, backward=True)
    g = p.backward(bits, cot)
    torch.cuda.synchronize()
    fb, fc = _expand_open(bits, plan["open"], cot)
    ref = _oracle_grad(text, fb, fc)
    n = len(plan["steps"])
    bound = 2 * n * 2.0 ** (-16 if precision == "bf16x3" else -11)
    err = rel_err(g.cpu().numpy(), ref)
    _say(f"  rel err {err:.2e} (bound {bound:.1e})")
    assert err <= bound


def test_grad_6x6_d24_64_bitstrings_exact_finite_differences(ctx):
    """L = sum_b |a_b|^2 is quadratic in each gate entry: central differences are exact."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("grad 6x6 d24 vs finite differences")
    c = generate(6, 6, 24, 0)
    text = c.to_text()
    bits = random_bitstrings(64, 36, 1)
    circ = Circuit(ctx, text)
    plan = sweep_plan(c)
    p = Plan(ctx, circ, plan, "fp32", backward=True)
    a = p.amplitudes(bits)
    g = p.backward(bits, 2 * a).cpu().numpy()
    base = circ.values.copy()

    def loss(vals):
        circ.set_values(vals)
        out = p.amplitudes(bits)
        torch.cuda.synchronize()
        return float(torch.sum(torch.abs(out) ** 2).item())

    ops = circ.ops
    two = [i for i, (_, _, qs) in enumerate(ops) if len(qs) == 2]
    one = [i for i, (_, _, qs) in enumerate(ops) if len(qs) == 1]
    picks = [(two[5], 3), (two[-7], 1), (one[3], 2), (one[len(one) // 2], 0), (one[-1], 1)]
    h = 0.5
    for i, e in picks:
        fd = 0j
        for step, w in ((h, 1.0), (1j * h, 1j)):
            vp, vm = base.copy(), base.copy()
            vp[i, e] += step
            vm[i, e] -= step
            fd += w * (loss(vp) - loss(vm)) / (2 * h)
        scale = np.max(np.abs(g))
        assert abs(g[i, e] - fd) <= 2e-4 * scale, (i, e, g[i, e], fd)
    circ.set_values(base)


def test_autograd_function_matches_direct_backward(ctx):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    from paper_1905_00444_amd.autograd import QFlexAmplitudes
    _say("autograd.Function")
    c = generate(3, 4, 16, 4)
    text = c.to_text()
    bits = random_bitstrings(8, 12, 2)
    circ = Circuit(ctx, text)
    p = Plan(ctx, circ, sweep_plan(c, open_qubits=[11]), "fp32", backward=True)
    vals = torch.tensor(circ.values, dtype=torch.complex64, device="cuda", requires_grad=True)
    amps = QFlexAmplitudes.apply(vals, p, bits)
    loss = (amps.abs() ** 2).sum()
    loss.backward()
    direct = p.backward(bits, 2 * amps.detach())
    torch.cuda.synchronize()
    assert torch.allclose(vals.grad, direct, rtol=0, atol=1e-6 * float(direct.abs().max()))
    fb, fc = _expand_open(bits, [11], 2 * amps.detach().cpu().numpy())
    ref = _oracle_grad(text, fb, fc)
    assert rel_err(vals.grad.cpu().numpy(), ref) <= 1e-4


def test_autograd_interleaved_forwards_get_their_own_gradients(ctx):
    """Two forwards with different gate values, then one backward through both: each branch's
    gradient is the adjoint oracle's at that branch's values (the plan's circuit holds one set of
    values at a time, so each backward writes its forward's values back first)."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    from paper_1905_00444_amd.autograd import QFlexAmplitudes
    from oracle.parse import read_circuit
    _say("autograd.Function, two interleaved forwards")
    c = generate(3, 4, 16, 4)
    text = c.to_text()
    bits = random_bitstrings(6, 12, 3)
    circ = Circuit(ctx, text)
    p = Plan(ctx, circ, sweep_plan(c, open_qubits=[11]), "fp32", backward=True)
    base = torch.tensor(circ.values, dtype=torch.complex64)
    rng = np.random.default_rng(12)
    other = base + 0.3 * torch.from_numpy((rng.normal(size=base.shape) + 1j * rng.normal(size=base.shape))
                                          .astype(np.complex64))
    v1 = base.clone().cuda().requires_grad_(True)
    v2 = other.clone().cuda().requires_grad_(True)
    a1 = QFlexAmplitudes.apply(v1, p, bits)
    a2 = QFlexAmplitudes.apply(v2, p, bits)
    loss = (a1.abs() ** 2).sum() + (a2.abs() ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    oc = read_circuit(text)
    for v, a, g in ((base, a1, v1.grad), (other, a2, v2.grad)):
        vals = [np.asarray(x).reshape(-1) for x in v.numpy().astype(np.complex128)]
        ov = oc.with_values([x.reshape(np.shape(y)) for x, y in zip(vals, oc.values)])
        fb, fc = _expand_open(bits, [11], 2 * a.detach().cpu().numpy())
        ref = np.stack([np.asarray(x).reshape(4) for x in ograd.adjoint_gradient(ov, fb, fc)])
        assert rel_err(g.cpu().numpy(), ref) <= 1e-4
    assert rel_err(v1.grad.cpu().numpy(), v2.grad.cpu().numpy()) > 1e-2  # the two really differ


@pytest.mark.parametrize("G", [4, 8])
def test_batched_backward_matches_sequential_and_oracle(ctx, G):
    """Backward with G chains per launch (chains = bitstrings x slices, 3 x 8 here): equal to the
    one-chain-at-a-time backward up to the order in which chains add into the world-line
    environments (atomic additions), and to the FP64 adjoint oracle.  Cuts and open qubits as in
    the test above."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say(f"batched backward G={G}")
    c = generate(4, 5, 32, 2)
    text = c.to_text()
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 1]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    bits = random_bitstrings(3, 20, 7)
    rng = np.random.default_rng(3)
    cot = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    seq = Plan(ctx, Circuit(ctx, text), plan, "fp32", backward=True).backward(bits, cot)
    bat = Plan(ctx, Circuit(ctx, text), plan, "fp32", backward=True, batch=G).backward(bits, cot)
    torch.cuda.synchronize()
    seq, bat = seq.cpu().numpy(), bat.cpu().numpy()
    assert rel_err(bat, seq) <= 1e-5
    fb, fc = _expand_open(bits, plan["open"], cot)
    assert rel_err(bat, _oracle_grad(text, fb, fc)) <= 1e-4


def test_batched_backward_ragged_last_group_and_slice_subrange(ctx):
    """5 bitstrings x slices [1, 6) = 25 chains in groups of 8 (the last holds one chain): the
    gradient equals the one-at-a-time backward over the same chains."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say("batched backward ragged")
    c = generate(4, 5, 32, 2)
    text = c.to_text()
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 1]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    bits = random_bitstrings(5, 20, 9)
    rng = np.random.default_rng(4)
    cot = rng.normal(size=(5, 4)) + 1j * rng.normal(size=(5, 4))
    seq = Plan(ctx, Circuit(ctx, text), plan, "fp32", backward=True).backward(bits, cot, 1, 6)
    bat = Plan(ctx, Circuit(ctx, text), plan, "fp32", backward=True, batch=8).backward(bits, cot, 1, 6)
    torch.cuda.synchronize()
    assert rel_err(bat.cpu().numpy(), seq.cpu().numpy()) <= 1e-5
