"""Automatic cut and order search (paper Sec. III-D): its plans are valid and exact (oracle),
its time model's reuse rule and sizes agree with the library's own bookkeeping, and on the 7x7
(1+40+1) workload it finds a plan at least as good as the hand-built one."""
import ctypes as C
import json

import numpy as np
import pytest

from paper_1905_00444_amd import _lib, planner
from workloads.circuits import generate
from workloads.plans import plan_7x7, C4_OPEN_SITES

from test_capi_host import _host_ctx, _circuit, _plan


def _library_figures(circ, plan):
    lib, ctx = _host_ctx()
    st, ch = _circuit(lib, ctx, circ)
    assert st == 0
    st, ph = _plan(lib, ctx, ch, plan)
    assert st == 0, lib.qf_last_error(ctx)
    inf = _lib.qf_plan_info()
    assert lib.qf_plan_info_get(ph, C.byref(inf)) == 0
    f = C.c_double()
    assert lib.qf_plan_flops(ph, 0, inf.n_slices, C.byref(f)) == 0
    out = (inf.peak_bits, inf.n_slices, f.value)
    lib.qf_plan_destroy(ph)
    lib.qf_circuit_destroy(ch)
    lib.qf_ctx_destroy(ctx)
    return out


def test_search_7x7_d40_matches_or_beats_hand_plan_and_library_agrees():
    c = generate(7, 7, 40, 0)
    text = c.to_text()
    hand, _ = plan_7x7(c, 40)
    ref = planner.evaluate(text, hand)
    best = planner.search(text, 30, C4_OPEN_SITES)
    assert best.peak_bits <= 30
    assert best.seconds <= ref.seconds
    for choice in (ref, best):
        peak, S, flops = _library_figures(c, choice.plan)
        assert peak == choice.peak_bits and S == choice.n_slices
        assert abs(flops - choice.flops) <= 1e-12 * flops


def test_search_prefers_no_cuts_when_everything_fits():
    c = generate(4, 4, 16, 0)
    best = planner.search(c.to_text(), 40)
    assert best.n_slices == 1 and best.plan["cuts"] == []


def test_search_respects_the_size_limit_with_cuts():
    from oracle import sv, tn
    from oracle.metrics import rel_err
    from workloads.bitstrings import random_bitstrings
    c = generate(4, 5, 32, 2)
    text = c.to_text()
    free = planner.search(text, 40)
    best = planner.search(text, free.peak_bits - 3, [(3, 4), (2, 4)])
    assert best.peak_bits <= free.peak_bits - 3 and best.n_slices > 1
    peak, S, flops = _library_figures(c, best.plan)
    assert (peak, S) == (best.peak_bits, best.n_slices)
    bits = random_bitstrings(2, 20, 4)
    got = tn.amplitudes(text, bits, best.plan)
    want = sv.open_amplitudes(text, bits, best.plan["open"])
    assert rel_err(got, want) <= 1e-12


def test_search_reports_infeasible_limits():
    c = generate(4, 5, 32, 2)
    with pytest.raises(ValueError):
        planner.search(c.to_text(), 8, max_cuts=1, max_cut_bits=2)


def test_cost_model_takes_measured_gemm_times(tmp_path):
    path = tmp_path / "tune.json"
    doc = {"device": "x", "entries": [
        {"precision": 1, "M": 1024, "N": 2048, "K": 512, "batch": 1, "variant": "large",
         "us": {"tiled4x4": 900.0, "large": 500.0}},
        {"precision": 0, "M": 1024, "N": 2048, "K": 512, "batch": 1, "variant": "tiled4x4",
         "us": {"tiled4x4": 7.0}}]}
    path.write_text(json.dumps(doc))
    m = planner.CostModel.from_autotune(str(path), "bf16x3")
    assert m.measured == {(10, 11, 9): 500e-6}
    base = planner.CostModel(precision="bf16x3")
    extra = m.step_seconds(10, 11, 9) - base.step_seconds(10, 11, 9)
    gemm_model = max(8.0 * 2.0 ** 30 / base.gemm_rate["bf16x3"],
                     8.0 * (2.0 ** 19 + 2.0 ** 20 + 2.0 ** 21) / base.bandwidth) + base.launch
    assert extra == pytest.approx(500e-6 - gemm_model)
    v = m.steps_seconds(np.array([10, 3]), np.array([11, 3]), np.array([9, 3]))
    assert v[0] == pytest.approx(m.step_seconds(10, 11, 9)) and v[1] == pytest.approx(m.step_seconds(3, 3, 3))
