"""Frugal rejection sampling (paper Sec. III-B) and XEB scoring (Sec. I-A) fed by amplitudes
that the HIP path contracts through the C-ABI, checked against the FP64 oracle's exact
probabilities of the same circuit."""
import numpy as np
import pytest

from oracle import sv
from oracle.metrics import rel_err
from paper_1905_00444_amd.sampling import frugal_rejection_sample, xeb_linear, xeb_log
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import sweep_plan

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision,batch", [("bf16x3", 1), ("fp32", 64)])
def test_rejection_sampling_on_gpu_amplitudes(precision, batch):
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan
    print(f"rejection sampling on HIP amplitudes, {precision}, {batch} chains per launch", flush=True)
    c = generate(4, 4, 32, 3)
    text = c.to_text()
    n = 16
    open_q = list(range(10, 16))
    plan = sweep_plan(c, open_qubits=open_q)
    prefixes = random_bitstrings(3000, n, 5)
    ctx = Context(0)
    p = Plan(ctx, Circuit(ctx, text), plan, precision, batch=batch)
    amps = p.amplitudes(prefixes)
    torch.cuda.synchronize()
    amps = amps.cpu().numpy()
    # every one of the 3000 x 64 probabilities the sampler sees, against the oracle
    ref = sv.open_amplitudes(text, prefixes, open_q)
    assert rel_err(amps, ref) <= 1e-4
    samples, ok = frugal_rejection_sample(amps, prefixes, open_q, n, M=10.0, rng=np.random.default_rng(0))
    assert ok.mean() > 0.9
    # scored with the oracle's exact probabilities of the accepted bitstrings
    psi = sv.final_state(text)
    pr = np.abs(psi[sv.bit_index(samples[ok])]) ** 2
    assert abs(xeb_linear(pr, n) - 1.0) < 0.15
    assert abs(xeb_log(pr, n) - 1.0) < 0.15
    # the same seeded draws over the oracle's amplitudes accept the same bitstrings, except where a
    # uniform draw falls within the amplitudes' rounding difference of its threshold
    s_ref, ok_ref = frugal_rejection_sample(ref, prefixes, open_q, n, M=10.0, rng=np.random.default_rng(0))
    same = (ok == ok_ref) & np.all(samples == s_ref, axis=1)
    assert same.mean() >= 0.995
    # uniformly drawn bitstrings score about 0 on the same probabilities
    pu = np.abs(psi[sv.bit_index(random_bitstrings(3000, n, 9))]) ** 2
    assert abs(xeb_linear(pu, n)) < 0.1
