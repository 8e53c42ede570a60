"""CPU-side checks of the C-ABI library: it loads, exports every declared symbol, and its
host logic (circuit and plan validation, shapes, flop counts, slice bookkeeping) is right.
No compute call is made here: there is no GPU on this side."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1905_00444_amd import _lib
from workloads.circuits import generate
from workloads.plans import plan_7x7, sweep_plan, PlanBuilder

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "qfmi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qf_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in _lib.EXPORTS, f"binding lacks {name}"


def _host_ctx():
    lib = _lib.load()
    h = C.c_void_p()
    assert lib.qf_ctx_create(0, None, None, 0, C.byref(h)) == 0
    return lib, h


def _circuit(lib, ctx, circ):
    from paper_1905_00444_amd.gates import gate_entries
    ops = circ.ops
    arr = (_lib.qf_op * len(ops))()
    for i, op in enumerate(ops):
        arr[i].cycle = op.cycle
        if len(op.qubits) == 1:
            arr[i].kind, arr[i].q0, arr[i].q1 = 1, op.qubits[0], -1
        else:
            arr[i].kind, arr[i].q0, arr[i].q1 = 2, op.qubits[0], op.qubits[1]
        e = gate_entries(op.name)
        for j in range(4):
            arr[i].values[2 * j], arr[i].values[2 * j + 1] = e[j].real, e[j].imag
    pres = circ.present_mask
    h = C.c_void_p()
    st = lib.qf_circuit_create(ctx, circ.rows, circ.cols, pres.ctypes.data_as(C.c_void_p), len(ops), arr, C.byref(h))
    return st, h


def _plan(lib, ctx, ch, plan, precision=0):
    steps = np.ascontiguousarray(np.asarray(plan["steps"], dtype=np.int32).reshape(-1))
    cuts = plan.get("cuts", [])
    carr = (_lib.qf_cut * max(1, len(cuts)))()
    for i, c in enumerate(cuts):
        carr[i].q0, carr[i].q1, carr[i].bit_lo, carr[i].nbits = c
    opn = np.ascontiguousarray(np.asarray(plan.get("open", []), dtype=np.int32))
    d = _lib.qf_plan_desc()
    d.n_steps = len(steps) // 2
    d.steps = steps.ctypes.data_as(C.POINTER(C.c_int32))
    d.n_cuts = len(cuts)
    d.cuts = carr
    d.n_open = len(opn)
    d.open = opn.ctypes.data_as(C.POINTER(C.c_int32)) if len(opn) else None
    d.precision = precision
    h = C.c_void_p()
    st = lib.qf_plan_create(ctx, ch, C.byref(d), C.byref(h))
    return st, h


def test_plan_info_matches_paper_flop_formula_7x7_d40():
    lib, ctx = _host_ctx()
    c = generate(7, 7, 40, 0)
    plan, pb = plan_7x7(c, 40)
    st, ch = _circuit(lib, ctx, c)
    assert st == 0
    st, ph = _plan(lib, ctx, ch, plan, precision=_lib.QF_BF16X3)
    assert st == 0, lib.qf_last_error(ctx)
    inf = _lib.qf_plan_info()
    assert lib.qf_plan_info_get(ph, C.byref(inf)) == 0
    assert inf.n_slices == 1024 and inf.n_open == 6 and inf.peak_bits == 30
    # F = 8 sqrt(v0 v1 v2) summed over steps, sizes from the plan builder
    want = 0.0
    for (a, b), vc in zip(plan["steps"], pb.sizes()):
        va, vb = pb.bits_of(pb.members[a]), pb.bits_of(pb.members[b])
        want += 8 * 2.0 ** ((va + vb + vc) / 2)
    assert abs(inf.flops_per_slice - want) / want < 1e-12
    # split-BF16 issues three MFMA products per complex product; the few SIMT steps issue none
    assert 2.99 * inf.flops_per_slice < inf.mfma_flops_per_slice <= 3.0 * inf.flops_per_slice
    # the A x B subtree does not depend on the second cut: later slices reuse it
    assert inf.flops_next_slice < inf.flops_first_slice
    f6 = C.c_double()
    assert lib.qf_plan_flops(ph, 0, 6, C.byref(f6)) == 0
    assert f6.value < 6 * inf.flops_per_slice
    assert inf.workspace_bytes > 4 * 8 * 2 ** 30  # several 2^30 complex64 tensors live at once
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)


def test_plan_validation_errors():
    lib, ctx = _host_ctx()
    c = generate(3, 3, 8, 0)
    st, ch = _circuit(lib, ctx, c)
    good = sweep_plan(c)
    st, ph = _plan(lib, ctx, ch, good)
    assert st == 0
    lib.qf_plan_destroy(ph)
    bad = {"steps": [[0, 1], [0, 2]] + good["steps"][2:], "cuts": [], "open": []}
    assert _plan(lib, ctx, ch, bad)[0] == _lib.QF_ERR_PLAN
    bad = {"steps": good["steps"][:-1], "cuts": [], "open": []}
    assert _plan(lib, ctx, ch, bad)[0] == _lib.QF_ERR_PLAN
    bad = dict(good, cuts=[[0, 4, 0, 1]])  # (0,0)-(1,1) is not a bond
    assert _plan(lib, ctx, ch, bad)[0] == _lib.QF_ERR_PLAN
    bad = dict(good, cuts=[[0, 1, 0, 2]])  # bond (0,1) has one bit at depth 8
    assert _plan(lib, ctx, ch, bad)[0] == _lib.QF_ERR_PLAN
    bad = dict(good, open=[3, 3])
    assert _plan(lib, ctx, ch, bad)[0] == _lib.QF_ERR_PLAN
    assert "open" in lib.qf_last_error(ctx).decode()
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)


def test_circuit_validation_errors():
    lib, ctx = _host_ctx()
    c = generate(3, 3, 8, 0)
    from workloads.circuits import Circuit, Op
    bad = Circuit(3, 3, (), list(c.ops) + [Op(9, "cz", (0, 4))])  # diagonal neighbours
    st, _ = _circuit(lib, ctx, bad)
    assert st == _lib.QF_ERR_ARG
    bad = Circuit(3, 3, (), list(c.ops) + [Op(9, "t", (9,))])
    st, _ = _circuit(lib, ctx, bad)
    assert st == _lib.QF_ERR_ARG
    lib.qf_ctx_destroy(ctx)


def test_workspace_required_before_compute():
    lib, ctx = _host_ctx()
    c = generate(3, 3, 8, 0)
    st, ch = _circuit(lib, ctx, c)
    st, ph = _plan(lib, ctx, ch, sweep_plan(c))
    out = C.c_void_p(16)
    bits = C.c_void_p(16)
    # no workspace: the call must refuse before touching the device
    assert lib.qf_amplitudes(ph, 1, bits, 0, 1, out) == _lib.QF_ERR_WORKSPACE
    assert lib.qf_amplitudes(ph, 1, bits, 0, 2, out) == _lib.QF_ERR_ARG  # 1 slice only
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)


def test_autotune_argument_checks_without_device():
    lib, ctx = _host_ctx()
    c = generate(3, 3, 8, 0)
    st, ch = _circuit(lib, ctx, c)
    st, ph = _plan(lib, ctx, ch, sweep_plan(c))
    assert lib.qf_autotune(None, ph, None) == _lib.QF_ERR_ARG
    assert lib.qf_autotune(ctx, None, None) == _lib.QF_ERR_ARG
    # no workspace: refused before any device call
    assert lib.qf_autotune(ctx, ph, None) == _lib.QF_ERR_WORKSPACE
    v = C.c_int(-1)
    assert lib.qf_tuned_variant(ctx, 1, 1 << 15, 1 << 15, 1 << 15, 1, C.byref(v)) == 0
    assert v.value == 0
    assert lib.qf_tuned_variant(None, 1, 1, 1, 1, 1, C.byref(v)) == _lib.QF_ERR_ARG
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)


def test_destroy_order_detaches_instead_of_dangling():
    """Objects may be released in any order (Python's collector does not order finalisers):
    destroying a context or a circuit detaches what was built on it."""
    lib, ctx = _host_ctx()
    c = generate(3, 3, 8, 0)
    st, ch = _circuit(lib, ctx, c)
    st, p1 = _plan(lib, ctx, ch, sweep_plan(c))
    st, p2 = _plan(lib, ctx, ch, sweep_plan(c))
    out = C.c_void_p(16)
    bits = C.c_void_p(16)
    lib.qf_circuit_destroy(ch)       # p1, p2 lose their circuit
    assert lib.qf_amplitudes(p1, 1, bits, 0, 1, out) == _lib.QF_ERR_ARG
    lib.qf_ctx_destroy(ctx)          # and their context
    assert lib.qf_amplitudes(p2, 1, bits, 0, 1, out) == _lib.QF_ERR_ARG
    inf = _lib.qf_plan_info()
    assert lib.qf_plan_info_get(p2, C.byref(inf)) == 0  # host-side description stays readable
    lib.qf_plan_destroy(p1)
    lib.qf_plan_destroy(p2)
    # a circuit of another context is refused
    lib, ctx_a = _host_ctx()
    lib, ctx_b = _host_ctx()
    st, ch = _circuit(lib, ctx_a, c)
    st, ph = _plan(lib, ctx_b, ch, sweep_plan(c))
    assert st == _lib.QF_ERR_ARG
    lib.qf_ctx_destroy(ctx_a)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx_b)


def test_cgemm_variant_argument_checks_without_device():
    """qf_cgemm_variant refuses unknown variants and variants that do not fit the shape before
    any device call (the pointers here are never dereferenced)."""
    lib, ctx = _host_ctx()
    p = C.c_void_p(256)
    tall = _lib.GEMM_VARIANTS.index("tall")
    assert lib.qf_cgemm_variant(ctx, 1, 99, 4096, 32, 32, p, p, p, 1, 0, 0, 0) == _lib.QF_ERR_ARG
    assert lib.qf_cgemm_variant(ctx, 1, -1, 4096, 32, 32, p, p, p, 1, 0, 0, 0) == _lib.QF_ERR_ARG
    # N = 4 and K = 4 are below the tall kernel's operand tiles; M = 100 is not a power of two
    assert lib.qf_cgemm_variant(ctx, 1, tall, 4096, 4, 32, p, p, p, 1, 0, 0, 0) == _lib.QF_ERR_UNSUPPORTED
    assert lib.qf_cgemm_variant(ctx, 1, tall, 4096, 32, 4, p, p, p, 1, 0, 0, 0) == _lib.QF_ERR_UNSUPPORTED
    assert lib.qf_cgemm_variant(ctx, 1, tall, 100, 32, 32, p, p, p, 1, 0, 0, 0) == _lib.QF_ERR_UNSUPPORTED
    assert lib.qf_cgemm_variant(ctx, 1, _lib.GEMM_VARIANTS.index("large"), 64, 64, 64, p, p, p, 1, 0, 0, 0) \
        == _lib.QF_ERR_UNSUPPORTED
    lib.qf_ctx_destroy(ctx)


def test_single_qubit_circuit_is_refused():
    """A one-qubit grid has no network to contract: the circuit is refused with a clear status."""
    lib, ctx = _host_ctx()
    st, ch = _circuit(lib, ctx, generate(1, 1, 8, 0))
    assert st == _lib.QF_ERR_UNSUPPORTED
    assert "2 qubits" in lib.qf_last_error(ctx).decode()
    lib.qf_ctx_destroy(ctx)


def test_plan_step_info_is_consistent_with_the_plan():
    """Per-step layout of the 7x7 (1+40+1) split-BF16 plan: sizes multiply to the step flops, the
    flops add up to the plan's, every leaf operand is gathered, the big steps run pre-split."""
    lib, ctx = _host_ctx()
    c = generate(7, 7, 40, 0)
    plan, _ = plan_7x7(c, 40)
    st, ch = _circuit(lib, ctx, c)
    st, ph = _plan(lib, ctx, ch, plan, precision=1)
    assert st == 0
    inf = _lib.qf_plan_info()
    assert lib.qf_plan_info_get(ph, C.byref(inf)) == 0
    n = inf.n_qubits
    steps = np.asarray(plan["steps"]).reshape(-1, 2)
    total = 0.0
    for i in range(inf.n_steps):
        si = _lib.qf_step_info()
        assert lib.qf_plan_step_info(ph, i, C.byref(si)) == 0
        assert (si.lhs, si.rhs) == tuple(int(x) for x in steps[i])
        assert {si.a_node, si.b_node} == {si.lhs, si.rhs}
        assert si.m_bits >= si.n_bits  # A has the larger free volume
        assert si.flops == 8.0 * 2.0 ** (si.m_bits + si.n_bits + si.k_bits)
        for node, permuted, reordered in ((si.a_node, si.a_permuted, si.a_reordered),
                                          (si.b_node, si.b_permuted, si.b_reordered)):
            if node < n:
                assert permuted  # world-line slices are gathered
            assert permuted or not reordered
        fits = si.m_bits >= 8 and si.n_bits >= 7 and si.k_bits >= 4
        assert si.presplit == fits
        if si.presplit:
            # the split happens in the permute, or the producing pre-split step wrote the operand
            for node, permuted in ((si.a_node, si.a_permuted), (si.b_node, si.b_permuted)):
                if not permuted:
                    prod = _lib.qf_step_info()
                    assert node >= n and lib.qf_plan_step_info(ph, node - n, C.byref(prod)) == 0
                    assert prod.presplit and prod.out_split
        else:
            assert not si.out_split
        total += si.flops
    assert total == pytest.approx(inf.flops_per_slice, rel=1e-12)
    si = _lib.qf_step_info()
    assert lib.qf_plan_step_info(ph, inf.n_steps, C.byref(si)) == _lib.QF_ERR_ARG
    assert lib.qf_plan_step_info(ph, -1, C.byref(si)) == _lib.QF_ERR_ARG
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)


def test_batched_plans_with_cuts_run_cut_independent_steps_once_per_group():
    """Batched plans with cuts group chains by bitstring: steps that depend on no cut run once per
    launch group, the others once per slice (qf_plan_flops counts the executed steps)."""
    from workloads.circuits import generate as gen
    from workloads.plans import plan_8x9, C5_REMOVED
    lib, ctx = _host_ctx()
    circ = gen(8, 9, 24, 0, C5_REMOVED)
    plan, _ = plan_8x9(circ)
    st, ch = _circuit(lib, ctx, circ)
    assert st == 0
    flops = {}
    for G in (1, 16, 256):
        steps = np.ascontiguousarray(np.asarray(plan["steps"], dtype=np.int32).reshape(-1))
        carr = (_lib.qf_cut * len(plan["cuts"]))()
        for i, c in enumerate(plan["cuts"]):
            carr[i].q0, carr[i].q1, carr[i].bit_lo, carr[i].nbits = c
        d = _lib.qf_plan_desc()
        d.n_steps, d.steps = len(steps) // 2, steps.ctypes.data_as(C.POINTER(C.c_int32))
        d.n_cuts, d.cuts, d.n_open, d.open, d.precision, d.batch = len(plan["cuts"]), carr, 0, None, 1, G
        h = C.c_void_p()
        assert lib.qf_plan_create(ctx, ch, C.byref(d), C.byref(h)) == 0
        inf = _lib.qf_plan_info()
        assert lib.qf_plan_info_get(h, C.byref(inf)) == 0
        f = C.c_double()
        assert lib.qf_plan_flops(h, 0, 256, C.byref(f)) == 0
        flops[G] = f.value
        if G == 256:
            # per slice, only the two 3-cell strips and the three joining contractions remain
            per_slice = inf.flops_per_slice
            f1 = C.c_double()
            assert lib.qf_plan_flops(h, 0, 1, C.byref(f1)) == 0
            assert f1.value == pytest.approx(per_slice)
            assert (f.value - per_slice) / 255 < 0.01 * per_slice
    assert flops[256] < flops[16] < 256 * inf.flops_per_slice


def test_output_order_lets_the_next_step_read_in_place():
    """The layout pass orders each result by the step that contracts its labels, lifting the top
    bits of N above the low bits of M where that order needs it: for the 70-qubit hand plan all but
    a few of the large operands are then read in place, and every output map keeps runs of at
    least 8 elements of N's low bits and stays within the step's bits."""
    from workloads.plans import plan_8x9, C5_REMOVED
    lib, ctx = _host_ctx()
    circ = generate(8, 9, 24, 0, C5_REMOVED)
    plan, _ = plan_8x9(circ)
    st, ch = _circuit(lib, ctx, circ)
    assert st == 0
    st, ph = _plan(lib, ctx, ch, plan, precision=1)
    assert st == 0
    info = _lib.qf_plan_info()
    assert lib.qf_plan_info_get(ph, C.byref(info)) == 0
    big = permuted = mapped = 0
    for i in range(info.n_steps):
        si = _lib.qf_step_info()
        assert lib.qf_plan_step_info(ph, i, C.byref(si)) == 0
        if si.out_nh:
            mapped += 1
            assert 0 < si.out_q <= si.m_bits and si.n_bits - si.out_nh >= 3
        for perm, bits in ((si.a_permuted, si.m_bits + si.k_bits), (si.b_permuted, si.n_bits + si.k_bits)):
            if bits >= 24:
                big += 1
                permuted += perm
    assert big == 50 and permuted <= 10 and mapped >= 20
    assert info.permute_bytes < 2e10
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)


def test_time_ceiling_argument_checks_without_device():
    """qf_time_ceiling refuses unknown kinds and precisions, copy sizes that are not positive
    multiples of 32 KiB, loops without trips, reps < 1 and null outputs before any device call
    (the buffer pointer here is never dereferenced)."""
    lib, ctx = _host_ctx()
    p = C.c_void_p(256)
    ms, work = C.c_float(), C.c_double()
    ARG = _lib.QF_ERR_ARG
    assert lib.qf_time_ceiling(ctx, 7, 1, p, 1 << 20, 1, C.byref(ms), C.byref(work)) == ARG  # kind
    assert lib.qf_time_ceiling(ctx, 0, 1, p, 3 << 10, 1, C.byref(ms), C.byref(work)) == ARG  # copy size
    assert lib.qf_time_ceiling(ctx, 0, 1, p, 0, 1, C.byref(ms), C.byref(work)) == ARG
    assert lib.qf_time_ceiling(ctx, 1, 9, p, 100, 1, C.byref(ms), C.byref(work)) == ARG      # precision
    assert lib.qf_time_ceiling(ctx, 1, 1, p, 0, 1, C.byref(ms), C.byref(work)) == ARG        # no trips
    assert lib.qf_time_ceiling(ctx, 1, 1, p, 100, 0, C.byref(ms), C.byref(work)) == ARG      # reps
    assert lib.qf_time_ceiling(ctx, 1, 1, None, 100, 1, C.byref(ms), C.byref(work)) == ARG   # buffer
    assert lib.qf_time_ceiling(ctx, 1, 1, p, 100, 1, None, C.byref(work)) == ARG
    assert b"qf_time_ceiling" in lib.qf_last_error(ctx)
    lib.qf_ctx_destroy(ctx)


@pytest.mark.parametrize("name", ["7x7-d40-bf16x3", "7x7-d40-fp32", "11x11-bf16x3"])
def test_layout_invariants_and_permute_traffic(name):
    """On the benchmark plans every output map stays within its step and keeps runs of at least 8
    elements of N's low bits, every split output feeds a pre-split consumer that reads it without
    a permute, and the permute traffic per slice stays at the level of the in-place layouts
    (it was 487 GB for 7x7 (1+40+1) and 778 GB for 11x11 (1+24+1) with every large operand
    permuted)."""
    from workloads.plans import plan_11x11
    lib, ctx = _host_ctx()
    if name.startswith("7x7"):
        circ = generate(7, 7, 40, 0)
        plan, _ = plan_7x7(circ, 40)
    else:
        circ = generate(11, 11, 24, 0)
        plan, _ = plan_11x11(circ)
    precision = 0 if name.endswith("fp32") else 1
    limit = {"7x7-d40-bf16x3": 2e11, "7x7-d40-fp32": 1.5e11, "11x11-bf16x3": 1.6e11}[name]
    st, ch = _circuit(lib, ctx, circ)
    assert st == 0
    st, ph = _plan(lib, ctx, ch, plan, precision=precision)
    assert st == 0
    info = _lib.qf_plan_info()
    assert lib.qf_plan_info_get(ph, C.byref(info)) == 0
    n = info.n_qubits
    steps = []
    for i in range(info.n_steps):
        si = _lib.qf_step_info()
        assert lib.qf_plan_step_info(ph, i, C.byref(si)) == 0
        steps.append(si)
    consumed_split = set()
    for si in steps:
        if si.out_nh:
            assert 0 < si.out_q <= si.m_bits and si.n_bits - si.out_nh >= 3
        for node, permuted in ((si.a_node, si.a_permuted), (si.b_node, si.b_permuted)):
            if node >= n and steps[node - n].out_split:
                assert si.presplit and not permuted
                consumed_split.add(node - n)
    assert consumed_split == {i for i, si in enumerate(steps) if si.out_split}
    if precision == 0:
        assert not consumed_split
    assert info.permute_bytes < limit
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)
