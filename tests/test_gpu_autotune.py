"""GEMM autotuning through the C-ABI: the cache file it writes, the variants it installs, and
that amplitudes computed after tuning (with the plan's buffers overwritten by the timing runs)
still match the state vector."""
import json

import numpy as np
import pytest

from oracle import sv
from oracle.metrics import rel_err
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import region_plan

pytestmark = pytest.mark.gpu


def _setup():
    c = generate(4, 5, 32, 2)
    qid = c.qubit_of()
    cuts = [[qid[(1, 3)], qid[(2, 3)], 0, 2], [qid[(3, 1)], qid[(3, 2)], 1, 2]]
    plan, _ = region_plan(c, 2, 2, cuts, [(3, 4), (2, 4)])
    return c, plan


@pytest.mark.parametrize("precision,batch", [("fp32", 1), ("bf16x3", 4)])
def test_autotune_cache_and_results(tmp_path, precision, batch):
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, autotune, tuned_variant, _lib
    print(f"autotune {precision} batch {batch}", flush=True)
    c, plan = _setup()
    bits = random_bitstrings(4, 20, 11)
    ref = sv.open_amplitudes(c.to_text(), bits, plan["open"])
    ctx = Context(0)
    p = Plan(ctx, Circuit(ctx, c.to_text()), plan, precision, batch=batch)
    before = p.amplitudes(bits)
    torch.cuda.synchronize()
    path = tmp_path / "tune.json"
    autotune(p, str(path))
    doc = json.loads(path.read_text())
    assert doc["device"] and doc["entries"]
    # batched plans with cuts run the steps that depend on no cut once per launch group (batch 1)
    assert {e["batch"] for e in doc["entries"]} <= {1, batch}
    assert any(e["batch"] == batch for e in doc["entries"])
    for e in doc["entries"]:
        assert e["variant"] in _lib.GEMM_VARIANTS[1:]
        assert e["variant"] in e["us"] and all(t > 0 for t in e["us"].values())
        assert tuned_variant(ctx, precision, e["M"], e["N"], e["K"], e["batch"]) == e["variant"]
    after = p.amplitudes(bits)
    torch.cuda.synchronize()
    bound = 1e-5 if precision == "fp32" else 1e-4
    assert rel_err(before.cpu().numpy(), ref) <= bound
    assert rel_err(after.cpu().numpy(), ref) <= bound
    # a fresh context takes every entry from the file without timing; the file keeps its entries
    ctx2 = Context(0)
    p2 = Plan(ctx2, Circuit(ctx2, c.to_text()), plan, precision, batch=batch)
    autotune(p2, str(path))
    doc2 = json.loads(path.read_text())
    assert doc2["entries"] == doc["entries"]
    for e in doc["entries"]:
        assert tuned_variant(ctx2, precision, e["M"], e["N"], e["K"], e["batch"]) == e["variant"]


@pytest.mark.parametrize("precision", ["fp32", "bf16x3"])
def test_every_gemm_variant_writes_the_plans_output_order(tmp_path, precision):
    """Each GEMM variant, forced for every shape through the autotune cache (a variant that does not
    fit a shape leaves it to the default), runs the 6x6 (1+24+1) sweep plan, most of whose steps
    write their result with the top bits of N above the low bits of M so that the next step reads
    it in place.  The amplitudes match the FP64 tensor-network oracle's (committed golden)."""
    import re
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan, autotune, _lib
    from workloads.plans import sweep_plan
    import os
    print(f"every GEMM variant with output maps, {precision}", flush=True)
    g = np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c2_grad.npz"))
    circ = generate(6, 6, 24, 0)
    bits = random_bitstrings(64, 36, 1)
    assert np.array_equal(g["bits"], bits)
    plan = sweep_plan(circ)
    text = circ.to_text()
    ctx = Context(0)
    p = Plan(ctx, Circuit(ctx, text), plan, precision)
    assert sum(s["out_nh"] > 0 for s in p.steps()) >= 10
    path = tmp_path / "tune.json"
    autotune(p, str(path))
    lines = path.read_text()
    bound = 1e-5 if precision == "fp32" else 1e-4
    for name in _lib.GEMM_VARIANTS[1:]:
        forced = tmp_path / f"tune_{name}.json"
        forced.write_text(re.sub(r'"variant": "[a-z0-9]+"', f'"variant": "{name}"', lines))
        c2 = Context(0)
        p2 = Plan(c2, Circuit(c2, text), plan, precision)
        autotune(p2, str(forced))
        got = p2.amplitudes(bits)
        torch.cuda.synchronize()
        err = rel_err(got.cpu().numpy()[:, 0], g["amps"])
        print(f"  {name}: rel err {err:.2e}", flush=True)
        assert err <= bound, name
