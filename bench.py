"""Benchmark: amplitudes/s and complex Tflop/s of the 7x7 (1+40+1) random circuit (bond 32),
split-BF16 (3 products) beside plain FP32, on one MI355X.

One step = one bitstring prefix with 6 open output qubits (64 amplitudes, paper Sec. III-B)
contracted over 6 of the 1024 slices (the paper's fidelity 6/1024 per amplitude, Sec. V).
Prints one JSON line.  Inputs are seeded synthetic circuits from the workloads package
(the paper's circuit files are not used).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_BF16 = 2516.6  # TFLOP/s, dense BF16 MFMA, MI355X
PEAK_FP32 = 157.3   # TFLOP/s, FP32 MFMA / vector, MI355X


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--slices", type=int, default=6, help="slices per step (fidelity slices/1024)")
    ap.add_argument("--fp32-steps", type=int, default=3)
    ap.add_argument("--fp16-steps", type=int, default=3)
    ap.add_argument("--whole-prefixes", type=int, default=1,
                    help="prefixes whose whole path sum (every contributing slice) is timed in split-BF16")
    ap.add_argument("--c5-slices", type=int, default=256,
                    help="8x9-d24: slices per bitstring of the hand plan's 256")
    ap.add_argument("--c5-batch", type=int, default=256, help="8x9-d24: chains per launch group (a power of two)")
    ap.add_argument("--cpu-reps", type=int, default=10, help="prefixes in the CPU oracle sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-subcheck", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="skip timing the GEMM kernel variants of the plans' shapes before the warmup")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip measuring the card's MFMA-loop and streaming-copy ceilings")
    ap.add_argument("--calib-copy", action="store_true",
                    help="launch one plain 1 GiB device copy first (HBM counter calibration)")
    ap.add_argument("--workload", default="7x7-d40", choices=["7x7-d40", "7x7-d32", "8x9-d24", "6x6-d24-grad", "11x11-d24", "vendor-gemm"],
                    help="7x7-d40: the benchmark line (default); 8x9-d24: 70 qubits, batched chains through a "
                         "captured graph, beside the searched plan; 6x6-d24-grad: forward and backward of 64 "
                         "amplitudes; 7x7-d32: whole 16-slice path sums in FP32 beside split-BF16; 11x11-d24: 121 qubits, a run of slices of the 64-slice region plan; vendor-gemm: the vendor real BF16 / FP32 GEMM on the same GPU (context for "
                         "the roofline: what the matrix cores sustain under the power limit)")
    return ap.parse_args()


def measure_ceilings(ctx):
    """What this card sustains, beside the nominal peaks: register-only MFMA loops (BF16, FP16,
    FP32 instructions, about 0.2 s per launch so that the clock settles under the power limit) and
    a streaming copy of 4 GiB (8 GiB read plus written per launch)."""
    from paper_1905_00444_amd import time_ceiling
    out = {"mfma_loop_tflops": {}, "unit_mfma": "TFLOP/s (real, dense)", "unit_copy": "TB/s (read + written)"}
    for prec, trips in (("bf16x3", 100000), ("fp16", 100000), ("fp32", 60000)):
        ms, flops = time_ceiling(ctx, "mfma", prec, trips, reps=3)
        out["mfma_loop_tflops"]["bf16" if prec == "bf16x3" else prec] = flops / ms / 1e9
    ms, nbytes = time_ceiling(ctx, "copy", size=8 << 30, reps=10)
    out["copy_tbps"] = nbytes / ms / 1e9
    return out


def bench_8x9(args):
    """70 qubits (8x9 minus two corners, 1+24+1, bond 8): 16 bitstrings x all 256 slices (or the
    first --c5-slices) of the two-halves plan as 4096 chains in launch groups of --c5-batch slices
    of one bitstring (the steps that no cut touches run once per group), one captured hipGraph per
    call; and the whole amplitudes of the same 16 bitstrings with the plan the search finds (no
    cut at 2^27)."""
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, planner, autotune
    from workloads.bitstrings import random_bitstrings
    from workloads.circuits import generate
    from workloads.plans import plan_8x9, C5_REMOVED
    circ = generate(8, 9, 24, 0, C5_REMOVED)
    text = circ.to_text()
    hand, _ = plan_8x9(circ)
    bits = random_bitstrings(16, 70, 1)
    ctx = Context(0, stream=torch.cuda.Stream())
    cobj = Circuit(ctx, text)
    rec = {"metric": "70-qubit (8x9 - 2, 1+24+1) amplitudes", "n_gpus": 1, "data": "synthetic, seeded",
           "dtype": "bf16x3 (FP32 accumulate)"}
    G, S = args.c5_batch, max(1, min(256, args.c5_slices))
    p = Plan(ctx, cobj, hand, "bf16x3", batch=G, graph=True)
    ctx.ensure_workspace(p.info()["workspace_bytes"])
    if not args.no_autotune:
        t0 = time.perf_counter()
        autotune(p)
        ctx.synchronize()
        print(f"bench: 8x9 autotune {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    with torch.cuda.stream(ctx.stream):
        bits_t = torch.from_numpy(bits).to(ctx.device)  # one device copy: the captured graph keys on it
    out = p.amplitudes(bits_t, 0, S)  # captures the graph, warms up
    ctx.synchronize()
    print("bench: 8x9 graph captured, warm-up pass done", file=sys.stderr, flush=True)
    with torch.cuda.stream(ctx.stream):
        out.zero_()
    ctx.synchronize()
    t0 = time.perf_counter()
    p.amplitudes(bits_t, 0, S, out=out)
    ctx.synchronize()
    dt = time.perf_counter() - t0
    launches, nodes = p.graph_info()
    chains = 16 * S
    fl = 16 * p.flops(0, S)  # executed: cut-independent steps once per launch group
    rec["batched_graph"] = {"chains": chains, "chains_per_launch_group": G, "slices": S, "seconds": dt,
                            "amplitudes_per_s": 16 / dt if S == 256 else None,
                            "chains_per_s": chains / dt, "complex_tflops": fl / dt / 1e12, "flops_executed": fl,
                            "flops_without_reuse": chains * p.info()["flops_per_slice"],
                            "graph_launches_per_call": 1, "graph_nodes": nodes,
                            "plan": "two halves, cuts (0,4)-(0,5) 3 bits, (1,4)-(1,5) 3 bits, (2,4)-(2,5) 2 bits; "
                                    "the cells carrying the cuts absorbed last as two 3-cell strips"}
    hand_amps = out.cpu().numpy()
    print(f"bench: 8x9 timed pass {dt:.2f} s", file=sys.stderr, flush=True)
    del p
    best = planner.search(text, 27)
    q = Plan(ctx, cobj, best.plan, "bf16x3")
    q.amplitudes(bits[:1])
    ctx.synchronize()
    t0 = time.perf_counter()
    full = q.amplitudes(bits)
    ctx.synchronize()
    dt = time.perf_counter() - t0
    f32 = Plan(ctx, cobj, best.plan, "fp32").amplitudes(bits)
    ctx.synchronize()
    from numpy.linalg import norm
    a, b = full.cpu().numpy(), f32.cpu().numpy()
    rec["searched_plan"] = {"amplitudes": 16, "seconds": dt, "amplitudes_per_s": 16 / dt,
                            "complex_tflops": 16 * q.info()["flops_per_slice"] / dt / 1e12,
                            "plan": repr(best), "rel_err_bf16x3_vs_fp32": float(norm(a - b) / norm(b)),
                            # all 256 slices of the hand plan sum to the same amplitudes (plan invariance)
                            "rel_diff_vs_hand_plan_path_sum": (float(norm(hand_amps - a) / norm(a))
                                                               if S == 256 else None)}
    print(json.dumps(rec), flush=True)
    return 0


def bench_vendor_gemm(args):
    """Real square GEMMs through torch (hipBLASLt / rocBLAS) in BF16 and FP32 on this GPU."""
    import torch
    out = {"metric": "vendor real GEMM TFLOP/s (torch matmul)", "n_gpus": 1}
    for dt, name in ((torch.bfloat16, "bf16"), (torch.float32, "fp32")):
        for n in (8192, 16384):
            a = torch.randn(n, n, device="cuda", dtype=dt)
            b = torch.randn(n, n, device="cuda", dtype=dt)
            for _ in range(3):
                c = a @ b
            torch.cuda.synchronize()
            reps = 10 if n == 8192 else 4
            t0 = time.perf_counter()
            for _ in range(reps):
                c = a @ b
            torch.cuda.synchronize()
            sec = (time.perf_counter() - t0) / reps
            out[f"{name}_{n}"] = {"ms": sec * 1e3, "tflops": 2.0 * n ** 3 / sec / 1e12}
            del a, b, c
    print(json.dumps(out), flush=True)
    return 0


def bench_6x6_grad(args):
    """6x6 (1+24+1), bond 8, 64 bitstrings: forward amplitudes and the gradient of sum |a|^2 with
    respect to every gate entry (FP32, row sweep, no cuts)."""
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan
    from workloads.bitstrings import random_bitstrings
    from workloads.circuits import generate
    from workloads.plans import sweep_plan
    circ = generate(6, 6, 24, 0)
    plan = sweep_plan(circ)
    bits = random_bitstrings(64, 36, 1)
    ctx = Context(0)
    p = Plan(ctx, Circuit(ctx, circ.to_text()), plan, "fp32", backward=True)
    a = p.amplitudes(bits)
    g = p.backward(bits, 2 * a)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = p.amplitudes(bits)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        g = p.backward(bits, 2 * a)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fwd, bwd = (t1 - t0) / args.steps, (t2 - t1) / args.steps
    fl = 64 * p.info()["flops_per_slice"]
    # the same forward with all 64 bitstrings as chains of one batched launch sequence
    pb = Plan(ctx, Circuit(ctx, circ.to_text()), plan, "fp32", batch=64)
    bits_t = torch.from_numpy(bits).to(ctx.device)
    ab = pb.amplitudes(bits_t)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    for _ in range(args.steps):
        ab = pb.amplitudes(bits_t)
    torch.cuda.synchronize()
    fwd_b = (time.perf_counter() - t3) / args.steps
    diff = float((torch.linalg.vector_norm(ab - a) / torch.linalg.vector_norm(a)).item())
    # and the backward with the 64 chains per launch
    pg = Plan(ctx, Circuit(ctx, circ.to_text()), plan, "fp32", backward=True, batch=64)
    gb = pg.backward(bits_t, 2 * a)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    for _ in range(args.steps):
        gb = pg.backward(bits_t, 2 * a)
    torch.cuda.synchronize()
    bwd_b = (time.perf_counter() - t4) / args.steps
    gdiff = float((torch.linalg.vector_norm(gb - g) / torch.linalg.vector_norm(g)).item())
    print(json.dumps({"metric": "6x6 (1+24+1) forward and backward, 64 bitstrings", "n_gpus": 1, "dtype": "fp32",
                      "forward_s": fwd, "backward_s": bwd, "forward_amplitudes_per_s": 64 / fwd,
                      "forward_complex_tflops": fl / fwd / 1e12, "backward_over_forward": bwd / fwd,
                      "forward_batched_s": fwd_b, "forward_batched_amplitudes_per_s": 64 / fwd_b,
                      "forward_batched_rel_diff": diff, "backward_batched_s": bwd_b,
                      "backward_batched_rel_diff": gdiff,
                      "gates": int(g.shape[0]), "data": "synthetic, seeded"}), flush=True)
    return 0


def bench_7x7_d32(args):
    """7x7 (1+32+1), bond 16: the region plan with one cut (16 slices, peak 2^28), 6 open qubits
    (64 amplitudes per prefix), whole path sums of seeded prefixes in plain FP32; beside it the
    same in split-BF16, and FP32 with the renormalisation off (its cost)."""
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, autotune
    from workloads.bitstrings import random_bitstrings
    from workloads.circuits import generate
    from workloads.plans import plan_7x7
    circ = generate(7, 7, 32, 0)
    plan, _ = plan_7x7(circ, 32)
    P = max(1, args.steps)
    bits = random_bitstrings(P, 49, 1)
    ctx = Context(0)
    cobj = Circuit(ctx, circ.to_text())
    res = {}
    for name, prec, renorm in (("fp32", "fp32", True), ("bf16x3", "bf16x3", True), ("fp32_no_renorm", "fp32", False)):
        p = Plan(ctx, cobj, plan, prec, renorm=renorm)
        if not args.no_autotune:
            autotune(p)
        p.amplitudes(bits[:1], 0, 1)  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        out = p.amplitudes(bits)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fl = P * p.flops(0, p.info()["n_slices"])
        res[name] = {"seconds": dt, "amplitudes_per_s": 64 * P / dt, "complex_tflops": fl / dt / 1e12}
        res[name + "_out"] = out
    rel = float((torch.linalg.vector_norm(res["bf16x3_out"] - res["fp32_out"])
                 / torch.linalg.vector_norm(res["fp32_out"])).item())
    # frugal rejection sampling (paper Sec. III-B) fed by split-BF16 path sums of fresh prefixes
    from paper_1905_00444_amd import sampling
    passes = 8 * P
    pre = random_bitstrings(passes, 49, 2)
    ps = Plan(ctx, cobj, plan, "bf16x3")
    t0 = time.perf_counter()
    amps = ps.amplitudes(pre).cpu().numpy()
    smp, acc = sampling.frugal_rejection_sample(amps, pre, plan["open"], 49, M=10.0,
                                                rng=np.random.default_rng(5))
    t_s = time.perf_counter() - t0
    probs = []
    for i in np.flatnonzero(acc):
        j = 0
        for t, q in enumerate(plan["open"]):
            j |= int(smp[i, q]) << (len(plan["open"]) - 1 - t)
        probs.append(abs(amps[i, j]) ** 2)
    sample_rec = {"passes": passes, "accepted": int(acc.sum()), "seconds": t_s,
                  "samples_per_s": float(acc.sum()) / t_s,
                  "xeb_linear": sampling.xeb_linear(np.array(probs), 49) if probs else None,
                  "xeb_linear_all_completions": sampling.xeb_linear(np.abs(amps.reshape(-1)) ** 2, 49)}
    same = bool(torch.equal(res["fp32_out"], res["fp32_no_renorm_out"]))
    print(json.dumps({"metric": "7x7 (1+32+1) amplitudes, 16-slice path sums", "n_gpus": 1, "prefixes": P,
                      "amplitudes": 64 * P, "fp32": res["fp32"], "bf16x3": res["bf16x3"],
                      "fp32_no_renorm": res["fp32_no_renorm"], "rel_err_bf16x3_vs_fp32": rel,
                      "renorm_bitwise_equal": same, "sampling": sample_rec, "data": "synthetic, seeded"}),
          flush=True)
    return 0


def bench_11x11(args):
    """121 qubits, 11x11 (1+24+1), bond 8: the region plan with two 3-bit corner cuts (64 slices,
    peak 2^30), 8 amplitudes (3 open qubits) of one bitstring prefix, split-BF16 with the
    renormalisation on (amplitudes are about 2^-60, below FP32's normal range).  Times a run of
    consecutive slices and extrapolates to the 64-slice path sum."""
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, autotune
    from workloads.bitstrings import random_bitstrings
    from workloads.circuits import generate
    from workloads.plans import plan_11x11
    circ = generate(11, 11, 24, 0)
    plan, _ = plan_11x11(circ)
    bits = random_bitstrings(1, 121, 1)
    ctx = Context(0)
    p = Plan(ctx, Circuit(ctx, circ.to_text()), plan, "bf16x3")
    if not args.no_autotune:
        autotune(p)
    info = p.info()
    n_slices = int(info["n_slices"])
    S = min(max(args.steps, 1) * 2, n_slices)
    out = p.amplitudes(bits, 0, 1)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = p.amplitudes(bits, 0, S)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    fl = p.flops(0, S)  # executed: subtrees that no cut bit changes run once per call
    full = p.flops(0, n_slices)
    est = dt * full / fl  # the whole path sum at the measured rate
    norm = float(torch.linalg.vector_norm(out).item())
    print(json.dumps({"metric": "11x11 (1+24+1) amplitudes, split-BF16", "n_gpus": 1, "dtype": "bf16x3 (FP32 accumulate)",
                      "slices_timed": S, "slices_per_amplitude": n_slices, "seconds": dt,
                      "complex_tflops": fl / dt / 1e12, "flops_timed": fl, "flops_full_path_sum": full,
                      "amplitudes_per_s_full_path_sum": 8 / est, "open_qubits": 3,
                      "partial_amplitude_norm": norm, "data": "synthetic, seeded"}), flush=True)
    return 0


def sub_check(ctx):
    """Relative amplitude error against the FP64 state vector on a 4x4 (1+40+1) circuit
    (bond 32, as in the 7x7 workload), per precision."""
    import torch
    from oracle import sv
    from oracle.metrics import rel_err
    from paper_1905_00444_amd import Circuit, Plan
    from workloads.bitstrings import random_bitstrings
    from workloads.circuits import generate
    from workloads.plans import region_plan
    c = generate(4, 4, 40, 0)
    plan, _ = region_plan(c, 2, 2, [], [(3, 2), (3, 3)])
    bits = random_bitstrings(64, 16, 1)
    ref = sv.open_amplitudes(c.to_text(), bits, plan["open"])
    out = {}
    for prec in ("fp32", "bf16x3", "fp16"):
        p = Plan(ctx, Circuit(ctx, c.to_text()), plan, prec)
        got = p.amplitudes(bits)
        torch.cuda.synchronize()
        out[prec] = rel_err(got.cpu().numpy(), ref)
    return out


def cpu_sample_steps(plan, pb, max_bits=25):
    """Plan steps whose operands and result all stay at or below 2^max_bits elements and whose
    inputs are leaves or other such steps (a bounded, representative part of the workload)."""
    n = pb.n
    ok = set(range(n))
    sel = []
    for i, ((a, b), vc) in enumerate(zip(plan["steps"], pb.sizes())):
        va, vb = pb.bits_of(pb.members[a]), pb.bits_of(pb.members[b])
        if a in ok and b in ok and max(va, vb, vc) <= max_bits:
            ok.add(n + i)
            sel.append(i)
    return sel


def host_cores():
    """(physical cores from lscpu, logical CPUs from os.cpu_count())."""
    import subprocess
    phys = None
    try:
        out = subprocess.run(["lscpu", "-p=core,socket"], capture_output=True, text=True, timeout=10).stdout
        phys = len({ln for ln in out.splitlines() if ln and not ln.startswith("#")})
    except Exception:
        pass
    return phys, os.cpu_count()


def cpu_baseline(circ, plan, pb, bits, step_info, flops_per_step, n_amp, reps):
    """Time the FP64 oracle on a bounded sample of the same workload and scale to one bench step:
    (1) the plan's steps whose tensors stay at or below 2^25 elements, slice 0, `reps` prefixes
    (tn.partial_contract); (2) the oracle's pairwise contraction (tn._contract, numpy tensordot in
    complex128) on one 2^13 x 2^13 x 2^13 complex product, the form of the plan's large steps.  A
    bench step's flops split into the small-step class (1) and the rest (2) as in one slice of the
    plan; its time is each class's flops over that class's measured rate."""
    import numpy as np
    from oracle import tn
    text = circ.to_text()
    sel = cpu_sample_steps(plan, pb)
    fl_small = 0.0
    for i in sel:
        (a, b), vc = plan["steps"][i], pb.sizes()[i]
        va, vb = pb.bits_of(pb.members[a]), pb.bits_of(pb.members[b])
        fl_small += 8 * 2.0 ** ((va + vb + vc) / 2)
    t0 = time.perf_counter()
    for r in range(reps):
        tn.partial_contract(text, bits[r], plan, 0, subset=sel)
    dt_small = time.perf_counter() - t0
    rate_small = fl_small * reps / dt_small
    # dominant class: A[m bits | k bits] x B[k bits | n bits] over the k bits, 2^13 each
    h = 13
    rng = np.random.default_rng(0)
    la = [("m", i) for i in range(h)] + [("k", i) for i in range(h)]
    lb = [("k", i) for i in range(h)] + [("n", i) for i in range(h)]
    a = (rng.standard_normal(2 ** (2 * h)) + 1j * rng.standard_normal(2 ** (2 * h))).reshape((2,) * (2 * h))
    b = (rng.standard_normal(2 ** (2 * h)) + 1j * rng.standard_normal(2 ** (2 * h))).reshape((2,) * (2 * h))
    t0 = time.perf_counter()
    tn._contract(a, la, b, lb)
    dt_big = time.perf_counter() - t0
    fl_big = 8.0 * 2.0 ** (3 * h)
    rate_big = fl_big / dt_big
    # flops of one slice of the plan by class (all steps, no reuse)
    slice_small = sum(st["flops"] for k, st in enumerate(step_info) if k in set(sel))
    slice_all = sum(st["flops"] for st in step_info)
    f_small = slice_small / slice_all
    t_step = flops_per_step * (f_small / rate_small + (1.0 - f_small) / rate_big)
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = None
    phys, logical = host_cores()
    return {"value": n_amp / t_step, "unit": "amplitudes/s", "cores": threads, "kind": "oracle",
            "sample": f"FP64 numpy oracle: (1) {len(sel)} of the {len(plan['steps'])} contractions of the 7x7 "
                      f"(1+40+1) plan (tensors <= 2^25 elements), slice 0, {reps} prefixes: "
                      f"{fl_small * reps:.3e} flop in {dt_small:.1f} s = {rate_small / 1e9:.1f} GFLOP/s; (2) the "
                      f"oracle's contraction on one 2^13-cubed complex product (the large steps' form): "
                      f"{fl_big:.3e} flop in {dt_big:.1f} s = {rate_big / 1e9:.1f} GFLOP/s; one step "
                      f"({flops_per_step:.3e} flop, {n_amp} amplitudes) at {100 * f_small:.2f}% class (1) and the "
                      f"rest class (2) flops",
            "fp64_gflops_small_steps": rate_small / 1e9, "fp64_gflops_large_product": rate_big / 1e9,
            "threads": threads, "physical_cores": phys, "os_cpu_count": logical}


PROFILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "profiles", "cgemm_pingpong_presplit_7x7_d40.md")
GEMM_SRC = [os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1905_00444_amd", "csrc", f)
            for f in ("cgemm_presplit.hip", "cgemm_common.h")]


def measured_traffic():
    """HBM bytes per dispatch of the dominant kernel from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or None when the kernel source has
    changed since the counters were taken."""
    import hashlib
    import re
    try:
        text = open(PROFILE).read()
        src = hashlib.sha256(b"".join(open(f, "rb").read() for f in GEMM_SRC)).hexdigest()
    except OSError:
        return None
    m = re.search(r"traffic_bytes_per_dispatch: ([0-9.e+]+) ; kernel source cgemm_presplit.hip \+ cgemm_common.h "
                  r"sha256: ([0-9a-f]+)", text)
    if not m or m.group(2) != src:
        return None
    return float(m.group(1))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: only --gpus 1 is supported; slices shard across GPUs "
                                   "with no communication but that path is not built"}))
        return 2
    if args.workload == "8x9-d24":
        return bench_8x9(args)
    if args.workload == "11x11-d24":
        return bench_11x11(args)
    if args.workload == "7x7-d32":
        return bench_7x7_d32(args)
    if args.workload == "6x6-d24-grad":
        return bench_6x6_grad(args)
    if args.workload == "vendor-gemm":
        return bench_vendor_gemm(args)
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, profile_enable, profile_read, autotune
    from workloads.bitstrings import random_bitstrings
    from workloads.circuits import generate
    from workloads.plans import plan_7x7, nonvanishing_slices

    print("bench: building 7x7 (1+40+1) workload", file=sys.stderr, flush=True)
    circ = generate(7, 7, 40, 0)
    plan, pb = plan_7x7(circ, 40)
    bits = random_bitstrings(64, 49, 1)
    ctx = Context(0)
    cobj = Circuit(ctx, circ.to_text())
    legs = [("bf16x3", args.steps), ("fp32", args.fp32_steps), ("fp16", args.fp16_steps)]
    plans = {prec: Plan(ctx, cobj, plan, prec) for prec, k in legs if k > 0 or prec == "bf16x3"}
    info = plans["bf16x3"].info()
    S = args.slices
    n_amp = 2 ** info["n_open"]
    ctx.ensure_workspace(info["workspace_bytes"])

    def runs_of(sl):
        r = []
        for x in sl:
            if r and r[-1][1] == x:
                r[-1][1] = x + 1
            else:
                r.append([x, x + 1])
        return r

    # the paths of each prefix: the first S slices not forced to zero by the gate pattern on the
    # cut qubits (for this circuit 128 of the 1024 paths of a prefix can be nonzero)
    n_free = len(nonvanishing_slices(circ, plan, bits[0], info["n_slices"]))
    runs = [runs_of(nonvanishing_slices(circ, plan, bits[b], S)) for b in range(len(bits))]
    step_flops = [sum(plans["bf16x3"].flops(a, e) for a, e in r) for r in runs]

    if not args.no_autotune:
        # per-shape kernel choice for the plans' GEMMs (held in the context; untimed set-up)
        for prec in plans:
            t0 = time.perf_counter()
            autotune(plans[prec])
            torch.cuda.synchronize()
            print(f"bench: autotune {prec} {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    ceil = None
    if not args.no_ceilings:
        ceil = measure_ceilings(ctx)
        print(f"bench: ceilings {ceil}", file=sys.stderr, flush=True)

    if args.calib_copy:
        x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    def run(prec, i, rr=None):
        b = i % len(bits)
        out = None
        for a, e in (rr if rr is not None else runs[b]):
            out = plans[prec].amplitudes(bits[b:b + 1], a, e, out=out)
        return out

    results = {}
    for prec, steps in legs:
        if steps <= 0:
            continue
        if prec == "bf16x3":
            for w in range(args.warmup):
                run(prec, w)
                torch.cuda.synchronize()
                print(f"bench: warmup {prec} {w} done", file=sys.stderr, flush=True)
        else:
            # one slice: workspace, kernels and tuning choices in place before the timed steps
            run(prec, 0, [[runs[0][0][0], runs[0][0][0] + 1]])
            torch.cuda.synchronize()
        profile_enable(ctx, True)
        profile_read(ctx, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        amps = []
        for i in range(steps):
            amps.append(run(prec, i))
            torch.cuda.synchronize()
            print(f"bench: {prec} step {i} done", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        gms, glaunch, gflops = profile_read(ctx, reset=True)
        profile_enable(ctx, False)
        results[prec] = {"s": dt, "steps": steps, "amps": torch.cat(amps).cpu().numpy(),
                         "gemm_ms": gms, "gemm_launches": glaunch, "gemm_flops": gflops}
        print(f"bench: {prec} {steps} steps in {dt:.2f} s", file=sys.stderr, flush=True)

    from numpy.linalg import norm

    def leg(prec):
        r = results.get(prec)
        if not r:
            return None
        fl = sum(step_flops[i % len(bits)] for i in range(r["steps"]))
        return {"value": n_amp * r["steps"] / r["s"], "complex_tflops": fl / r["s"] / 1e12, "steps": r["steps"],
                "ms_per_step": r["s"] / r["steps"] * 1e3}

    def rel(prec):
        # norm-wise difference from FP32 on the same prefixes (same steps)
        a, f = results.get(prec), results.get("fp32")
        if not a or not f:
            return None
        k = min(len(a["amps"]), len(f["amps"]))
        den = norm(f["amps"][:k])
        return float(norm(a["amps"][:k] - f["amps"][:k]) / den) if den > 0 else None

    bf = results["bf16x3"]
    main_leg = leg("bf16x3")
    ms_step = main_leg["ms_per_step"]
    value = main_leg["value"]
    flops_step = sum(step_flops[i % len(bits)] for i in range(bf["steps"])) / bf["steps"]
    gemm_avg_ms = bf["gemm_ms"] / max(1, bf["gemm_launches"])
    per_launch = bf["gemm_flops"] / max(1, bf["gemm_launches"])
    achieved = per_launch / (gemm_avg_ms * 1e-3) / 1e12 if gemm_avg_ms > 0 else 0.0
    peak = PEAK_BF16 / 3.0
    fp_leg = leg("fp32")
    rec = {
        "metric": "amplitudes/s and complex Tflop/s, 7x7 (1+40+1) RQC; split-BF16 vs FP32 at stated rel err",
        "value": value,
        "unit": f"amplitudes/s ({S} paths per amplitude: fidelity {S}/{n_free} of the paths that can be nonzero, "
                f"{S}/1024 of all)",
        "n_gpus": 1, "steps": bf["steps"], "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3 (FP32 accumulate)",
        "data": "synthetic: seeded 7x7 (1+40+1) random circuit, seeded bitstring prefixes",
        "config": {"workload": "7x7 (1+40+1) RQC, bond 32, 2 cuts (1024 slices), 6 open qubits (64 amplitudes "
                               f"per prefix), {S} nonvanishing slices per step", "global_batch": n_amp,
                   "slices_per_step": S, "nonvanishing_slices_per_prefix": n_free, "parallelism": "single GPU"},
        "complex_tflops": main_leg["complex_tflops"],
        "fp32": fp_leg,
        "fp16": leg("fp16"),
        "speedup_bf16x3_vs_fp32": value / fp_leg["value"] if fp_leg else None,
        "rel_err_vs_fp32_same_prefixes": {"bf16x3": rel("bf16x3"), "fp16": rel("fp16")},
        "flops_per_step": flops_step,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
                     "traffic": measured_traffic(),
                     "traffic_unit": "bytes per dispatch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "cgemm_pingpong_presplit (split-BF16, operands split by the preceding permute) on "
                               "the 2^15 x 2^15 x 2^15 complex contractions",
                     "peak_note": "2516.6 TFLOP/s dense BF16 MFMA / 3 products per complex FP32 product; "
                                  "achieved counts algorithmic complex flops 8*M*N*K",
                     "launches": bf["gemm_launches"], "avg_ms": gemm_avg_ms},
    }
    if ceil:
        mpeak = ceil["mfma_loop_tflops"]["bf16"] / 3.0
        rec["roofline"]["measured_peak"] = mpeak
        rec["roofline"]["frac_of_measured"] = achieved / mpeak
        rec["roofline"]["measured_note"] = ("register-only loop of v_mfma_f32_16x16x32_bf16 on this card (no memory "
                                            "traffic, pseudo-random operands) / 3 products; the sustained rate "
                                            "depends on the operands through power, and the benchmark's operands "
                                            "draw less than random ones, so this fraction can exceed 1")
        rec["ceilings"] = ceil
    if args.whole_prefixes > 0:
        # whole amplitudes: every slice of the prefix that can be nonzero (the other 896 of the 1024
        # paths are identically zero for this circuit), split-BF16
        wr = [runs_of(nonvanishing_slices(circ, plan, bits[b], info["n_slices"])) for b in range(args.whole_prefixes)]
        wfl = sum(plans["bf16x3"].flops(a, e) for r in wr for a, e in r)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for b in range(args.whole_prefixes):
            run("bf16x3", b, wr[b])
            torch.cuda.synchronize()
            print(f"bench: whole path sum of prefix {b} done", file=sys.stderr, flush=True)
        dt = time.perf_counter() - t0
        rec["whole_amplitudes"] = {"value": n_amp * args.whole_prefixes / dt, "unit": "amplitudes/s",
                                   "paths_per_amplitude": n_free, "prefixes": args.whole_prefixes, "seconds": dt,
                                   "complex_tflops": wfl / dt / 1e12, "flops": wfl,
                                   "note": "every path that can be nonzero (fidelity 1); the remaining "
                                           f"{info['n_slices'] - n_free} slices are identically zero"}
    if not args.no_subcheck:
        print("bench: 4x4 (1+40+1) sub-check vs FP64 state vector", file=sys.stderr, flush=True)
        rec["rel_err_vs_fp64_4x4_d40"] = sub_check(ctx)
    if not args.no_cpu:
        print("bench: CPU oracle sample", file=sys.stderr, flush=True)
        rec["cpu_baseline"] = cpu_baseline(circ, plan, pb, bits, plans["bf16x3"].steps(), flops_step, n_amp,
                                           args.cpu_reps)
    print(json.dumps(rec), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
