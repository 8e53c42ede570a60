"""End-to-end parity of the HIP path (through the C-ABI) with the FP64 oracle and with
closed forms, at the benchmark configurations' shapes."""
import os

import numpy as np
import pytest

from oracle import sv, tn
from oracle.metrics import rel_err
from workloads.bitstrings import random_bitstrings, all_bitstrings
from workloads.circuits import generate, identity_cz, mirror
from workloads.plans import sweep_plan, region_plan, plan_7x7, plan_11x11, nonvanishing_slices

pytestmark = pytest.mark.gpu

# norm-wise relative error bounds against FP64 (FP32 and split-BF16 targets; FP16 stated)
BOUND = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16": 3e-2}


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1905_00444_amd import Context
    assert torch.cuda.is_available()
    return Context(0)


def _amps(ctx, circ, plan, bits, precision="fp32", s_begin=0, s_end=None, hoist=True, renorm=True):
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    c = Circuit(ctx, circ.to_text())
    p = Plan(ctx, c, plan, precision, hoist=hoist, renorm=renorm)
    out = p.amplitudes(bits, s_begin, s_end)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
def test_4x4_d16_64_bitstrings_vs_state_vector(ctx, precision):
    _say(f"4x4 d16 64 bitstrings {precision}")
    c = generate(4, 4, 16, 0)
    bits = random_bitstrings(64, 16, 1)
    got = _amps(ctx, c, sweep_plan(c), bits, precision)[:, 0]
    ref = sv.amplitudes(c.to_text(), bits)
    assert rel_err(got, ref) <= BOUND[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_open_qubits_on_both_sides_with_operands_listed_small_first(ctx, precision):
    """Every step of a row sweep written as (new cell, running tensor), so the library's roles
    (the larger operand as A) are the reverse of the listed order, with open qubits in the first
    and the last cell: the open output legs of both sides of the final contraction land where the
    state vector has them."""
    _say(f"open qubits on both sides, operands listed small first, {precision}")
    c = generate(4, 4, 16, 3)
    plan = sweep_plan(c, open_qubits=[0, 1, 14, 15])
    plan = dict(plan, steps=[[b, a] for a, b in plan["steps"]])
    bits = random_bitstrings(6, 16, 5)
    ref = sv.open_amplitudes(c.to_text(), bits, plan["open"])
    got = _amps(ctx, c, plan, bits, precision)
    assert rel_err(got, ref) <= BOUND[precision]


def test_4x4_d16_all_amplitudes_unit_norm(ctx):
    _say("4x4 d16 all 2^16 amplitudes")
    c = generate(4, 4, 16, 0)
    open_q = list(range(8, 16))
    prefixes = np.zeros((256, 16), dtype=np.uint8)
    prefixes[:, :8] = all_bitstrings(8)
    got = _amps(ctx, c, sweep_plan(c, open_qubits=open_q), prefixes)
    psi = sv.final_state(c.to_text())
    assert rel_err(got.reshape(-1), psi) <= 1e-5
    assert abs(np.sum(np.abs(got) ** 2) - 1.0) <= 1e-5


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
def test_4x5_d32_regions_cuts_open_vs_state_vector(ctx, precision):
    _say(f"4x5 d32 regions {precision}")
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4), (3, 3)])
    bits = random_bitstrings(4, 20, 3)
    got = _amps(ctx, c, plan, bits, precision)
    ref = sv.open_amplitudes(c.to_text(), bits, plan["open"])
    assert rel_err(got, ref) <= BOUND[precision]


def test_6x6_d24_vs_tensor_network_oracle(ctx):
    _say("6x6 d24 vs oracle-TN")
    c = generate(6, 6, 24, 0)
    bits = random_bitstrings(3, 36, 1)
    plan = sweep_plan(c)
    got = _amps(ctx, c, plan, bits, "fp32")[:, 0]
    ref = tn.amplitudes(c.to_text(), bits, plan)[:, 0]
    assert rel_err(got, ref) <= 1e-5
    got16 = _amps(ctx, c, plan, bits, "bf16x3")[:, 0]
    assert rel_err(got16, ref) <= 1e-4


def test_hoisting_and_slice_ranges_are_exact(ctx):
    """Reusing slice-independent subtrees, and splitting the slice range, change nothing."""
    _say("hoist / slice range")
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4)])
    bits = random_bitstrings(2, 20, 4)
    a = _amps(ctx, c, plan, bits, "fp32")
    b = _amps(ctx, c, plan, bits, "fp32", hoist=False)
    assert np.array_equal(a, b)
    part = _amps(ctx, c, plan, bits, "fp32", 0, 5)
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    cc = Circuit(ctx, c.to_text())
    p = Plan(ctx, cc, plan, "fp32")
    out = p.amplitudes(bits, 0, 5)
    p.amplitudes(bits, 5, 16, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), a)
    assert not np.allclose(part, a)


def test_fault_injection_and_resume(ctx, monkeypatch):
    import torch
    from paper_1905_00444_amd import Circuit, Plan, _lib
    _say("fault injection")
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    plan, _ = region_plan(c, 2, 2, [[qid[(1, 3)], qid[(2, 3)], 0, 3]], [(3, 4)])
    bits = random_bitstrings(1, 20, 4)
    full = _amps(ctx, c, plan, bits, "fp32")
    cc = Circuit(ctx, c.to_text())
    p = Plan(ctx, cc, plan, "fp32")
    monkeypatch.setenv("QFMI_FAULT_AFTER_SLICES", "3")
    with pytest.raises(_lib.QfError) as e:
        out = torch.zeros((1, 2), dtype=torch.complex128, device="cuda")
        p.amplitudes(bits, 0, 8, out=out)
    assert e.value.status == _lib.QF_ERR_INJECTED
    monkeypatch.delenv("QFMI_FAULT_AFTER_SLICES")
    p.amplitudes(bits, 3, 8, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), full)


def _product_vectors(circ, plan, s):
    """Per-qubit final 2-vectors of one slice when every CZ is the identity: the network
    factorises per qubit; a cut bond bit k fixes the q0-side projector |k><k| at that gate's time."""
    from oracle import gates
    cuts = plan["cuts"]
    total = sum(c[3] for c in cuts)
    fixed = {}
    off = total
    for q0, q1, lo, nb in cuts:
        off -= nb
        v = (s >> off) & ((1 << nb) - 1)
        for i in range(nb):
            fixed[(q0, q1, lo + i)] = (v >> (nb - 1 - i)) & 1
    vecs = [np.array([1, 0], dtype=np.complex128) for _ in range(circ.n_qubits)]
    seen = {}
    for op in circ.ops:
        if len(op.qubits) == 1:
            q = op.qubits[0]
            vecs[q] = gates.one_qubit(op.name) @ vecs[q]
        else:
            q0, q1 = op.qubits
            j = seen.get((q0, q1), 0)
            seen[(q0, q1)] = j + 1
            if (q0, q1, j) in fixed:
                k = fixed[(q0, q1, j)]
                vecs[q0] = vecs[q0] * (np.arange(2) == k)
    return vecs


def _product_slice_closed_form(circ, plan, bits_row, s):
    """Closed form of one slice of a product circuit (see _product_vectors)."""
    vecs = _product_vectors(circ, plan, s)
    opn = plan["open"]
    closed = [vecs[q][bits_row[q]] for q in range(circ.n_qubits) if q not in opn]
    amp = np.prod(closed)
    out = np.array([amp], dtype=np.complex128)
    for q in opn:
        out = np.outer(out, vecs[q]).reshape(-1)
    return out


def _clifford_case(base, plan, n_slices):
    """A Clifford product circuit (CZ -> identity, T -> S) and a bitstring whose first n_slices
    non-vanishing slices are all nonzero: each output bit is the larger component of its qubit.
    Its tensors hold entries within a bounded range of magnitudes (products of 0, 1 and 2^-1/2
    factors), unlike product circuits with T gates, whose tensors span more than 2^150."""
    from workloads.circuits import clifford_substitute
    c = clifford_substitute(identity_cz(base))
    bits = np.zeros((1, base.n_qubits), dtype=np.uint8)
    for _ in range(3):
        s0 = nonvanishing_slices(base, plan, bits[0], 1)[0]
        vecs = _product_vectors(c, plan, s0)
        bits[0] = [int(np.argmax(np.abs(v))) for v in vecs]
    sl = nonvanishing_slices(base, plan, bits[0], n_slices)
    return c, bits, sl


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
def test_product_circuit_full_7x7_d40_shape_one_slice(ctx, precision):
    """Every tensor of the 7x7 (1+40+1) workload at full size (peak 2^30), CZ -> identity.
    Split-BF16 runs the Clifford variant: with T gates a product circuit's tensors hold entries
    over more than 2^150 of range, and the low BF16 halves of entries far below a tensor's
    largest fall under the smallest normal number (random circuits stay far from that)."""
    _say(f"7x7 d40 product circuit, one slice, {precision}")
    base = generate(7, 7, 40, 0)
    plan, _ = plan_7x7(base, 40)
    if precision == "bf16x3":
        c, bits, sl = _clifford_case(base, plan, 1)
        s = sl[0]
    else:
        c = identity_cz(base)
        bits = random_bitstrings(1, 49, 1)
        s = nonvanishing_slices(base, plan, bits[0], 3)[-1]
    ref = _product_slice_closed_form(c, plan, bits[0], s)
    assert np.linalg.norm(ref) > 1e-20
    got = _amps(ctx, c, plan, bits, precision, s, s + 1)[0]
    assert rel_err(got, ref) <= BOUND[precision]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_mirror_circuit_7x7_bond16_all_slices(ctx, precision):
    """V^dagger V on 7x7 with 16+16 cycles has bond dimension 16 (the 7x7 (1+32+1) shape):
    a(0...0) = 1 and every other amplitude 0, summed over all 16 slices."""
    _say(f"7x7 mirror, 16 slices, {precision}")
    base = generate(7, 7, 32, 0)
    plan, _ = plan_7x7(base, 32)
    m = mirror(base, 16, 5)
    bits = np.zeros((1, 49), dtype=np.uint8)
    got = _amps(ctx, m, plan, bits, precision)[0]
    want = np.zeros(64, dtype=np.complex128)
    want[0] = 1.0
    assert np.max(np.abs(got - want)) <= (2e-5 if precision == "fp32" else 2e-4)


def test_product_circuit_7x7_d40_bench_launch_configuration(ctx):
    """The benchmark's exact call: one prefix, slices 0..5 with reuse of the subtrees that do not
    depend on the second cut, split-BF16; every slice has a closed form when CZ -> identity."""
    _say("7x7 d40 Clifford product circuit, six slices (bench configuration)")
    base = generate(7, 7, 40, 0)
    plan, _ = plan_7x7(base, 40)
    c, bits, sl = _clifford_case(base, plan, 6)
    assert sl == list(range(sl[0], sl[0] + 6))
    got = _amps(ctx, c, plan, bits, "bf16x3", sl[0], sl[0] + 6)[0]
    ref = sum(_product_slice_closed_form(c, plan, bits[0], s) for s in sl)
    assert np.linalg.norm(ref) > 1e-20
    assert rel_err(got, ref) <= 1e-4


def test_7x7_d32_random_slice_vs_tensor_network_oracle(ctx):
    """A random 7x7 (1+32+1) circuit (bond 16, peak 2^28): one slice of one prefix (64
    amplitudes) against the FP64 tensor-network oracle, in all three precisions."""
    _say("7x7 d32 random slice vs oracle-TN")
    c = generate(7, 7, 32, 0)
    plan, _ = plan_7x7(c, 32)
    bits = random_bitstrings(1, 49, 1)
    s = nonvanishing_slices(c, plan, bits[0], 4)[-1]
    ref = tn.amplitudes(c.to_text(), bits, plan, slices=[s])
    assert np.linalg.norm(ref) > 1e-20
    for prec, bound in (("fp32", 1e-5), ("bf16x3", 1e-4), ("fp16", 5e-3)):
        got = _amps(ctx, c, plan, bits, prec, s, s + 1)
        assert rel_err(got, ref) <= bound, prec


def test_7x7_d40_random_slice_precisions_agree(ctx):
    """The benchmark's random 7x7 (1+40+1) circuit at full size (peak 2^30): one nonvanishing
    slice of one prefix (64 amplitudes) in split-BF16 and FP16 against FP32 on the same slice.
    No FP64 reference reaches this size in a test (one slice is 7.5e14 flop); FP32 itself is
    pinned to the FP64 oracles on the 7x7 (1+32+1) slice above and on the 4x4 (1+40+1) circuit
    (bond 32, as here) of the benchmark's sub-check."""
    _say("7x7 d40 random slice, split-BF16 and FP16 vs FP32")
    c = generate(7, 7, 40, 0)
    plan, _ = plan_7x7(c, 40)
    bits = random_bitstrings(1, 49, 1)
    s = nonvanishing_slices(c, plan, bits[0], 1)[0]
    ref = _amps(ctx, c, plan, bits, "fp32", s, s + 1)
    assert np.linalg.norm(ref) > 1e-20
    for prec, bound in (("bf16x3", 1e-4), ("fp16", 5e-3)):
        got = _amps(ctx, c, plan, bits, prec, s, s + 1)
        assert rel_err(got, ref) <= bound, prec


def test_11x11_d24_random_slice_precisions_agree(ctx):
    """The 121-qubit random circuit (peak 2^30, 120 contractions; amplitudes about 2^-60, kept in
    range by the renormalisation): one slice of one prefix in split-BF16 against FP32, held to the
    split-BF16 target of 1e-4 over its 120 contractions (the worst-case drift n 2^-16 would allow
    1.8e-3)."""
    _say("11x11 d24 random slice, split-BF16 vs FP32")
    c = generate(11, 11, 24, 0)
    plan, _ = plan_11x11(c)
    bits = random_bitstrings(1, 121, 1)
    s = nonvanishing_slices(c, plan, bits[0], 1)[0]
    ref = _amps(ctx, c, plan, bits, "fp32", s, s + 1)
    assert np.linalg.norm(ref) > 0
    got = _amps(ctx, c, plan, bits, "bf16x3", s, s + 1)
    err = rel_err(got, ref)
    _say(f"  split-BF16 vs FP32 rel err {err:.2e} (bound 1.0e-04)")
    assert err <= 1e-4


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_renormalisation_is_exact(ctx, precision):
    """Power-of-two renormalisation only moves exponents: FP32 and split-BF16 results with and
    without it are bitwise identical on a workload whose values stay in range."""
    _say(f"renormalisation exact {precision}")
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    bits = random_bitstrings(3, 20, 8)
    a = _amps(ctx, c, plan, bits, precision)
    b = _amps(ctx, c, plan, bits, precision, renorm=False)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision", ["fp32", "bf16x3", "fp16"])
def test_11x11_d24_scaled_product_circuit_full_shape(ctx, precision):
    """121 qubits, (1+24+1), peak 2^30, one slice of the 64.  A Clifford product circuit (CZ ->
    identity, T -> S; product circuits with T gates are ill-conditioned at this size: their paths
    cancel to 2^-190) whose Hadamard gate values are scaled by 1/4, so the amplitudes are about
    2^-530, far below the FP32 and FP16 ranges: only the renormalised path can return them.
    Closed form: the unscaled product times 4^-(number of Hadamards).  FP32 and split-BF16 are held
    to their targets (1e-5, 1e-4) over the 120 contractions; FP16 to 3e-2."""
    import torch
    from paper_1905_00444_amd import Circuit, Plan
    _say(f"11x11 d24 scaled Clifford product circuit {precision}")
    base = generate(11, 11, 24, 0)
    plan, pb = plan_11x11(base)
    assert max(pb.sizes()) == 30
    c, bits, sl = _clifford_case(base, plan, 1)
    s = sl[0]
    n_h = sum(1 for op in c.ops if op.name == "h")
    ref = _product_slice_closed_form(c, plan, bits[0], s) * 0.25 ** n_h
    assert np.linalg.norm(ref) > 1e-300
    circ = Circuit(ctx, c.to_text())
    vals = circ.values.copy()
    vals[[i for i, op in enumerate(c.ops) if op.name == "h"]] *= 0.25
    circ.set_values(vals)
    bound = {"fp32": 1e-5, "bf16x3": 1e-4, "fp16": 3e-2}[precision]
    got = Plan(ctx, circ, plan, precision).amplitudes(bits, s, s + 1)
    torch.cuda.synchronize()
    err = rel_err(got.cpu().numpy()[0], ref)
    _say(f"  rel err {err:.2e} (bound {bound:.1e})")
    assert err <= bound
    if precision == "fp32":
        flat = Plan(ctx, circ, plan, precision, renorm=False).amplitudes(bits, s, s + 1)
        torch.cuda.synchronize()
        assert rel_err(flat.cpu().numpy()[0], ref) > 0.5  # underflows at true scale


def test_one_call_amplitudes_function():
    import torch
    from paper_1905_00444_amd import amplitudes
    _say("one-call amplitudes")
    c = generate(4, 4, 16, 0)
    bits = random_bitstrings(8, 16, 2)
    got = amplitudes(c.to_text(), sweep_plan(c), bits, "fp32")
    torch.cuda.synchronize()
    assert got.dtype == torch.complex128 and got.shape == (8, 1)
    assert rel_err(got.cpu().numpy()[:, 0], sv.amplitudes(c.to_text(), bits)) <= 1e-5
