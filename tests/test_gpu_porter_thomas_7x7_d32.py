"""The 7x7 (1+32+1) workload as configured: 256 seeded bitstring prefixes, 6 open qubits each
(16,384 whole amplitudes, all 16 slices of the one-cut region plan), plain FP32 through the
C-ABI.  Checked three ways:
  * prefixes 0 and 1 against FP64 amplitudes of the tensor-network oracle (tests/golden);
  * the paper's scale, mean |a|^2 = 2^-49 (Sec. III-E: about 1e-15 for 49 qubits);
  * Porter-Thomas statistics of a chaotic circuit (paper Sec. I-A: N p ~ Exp(1) for uniformly
    drawn bitstrings): mean of N p within 0.03 of 1, second moment within 0.15 of 2 (about 4
    standard errors at 16,384 samples), Kolmogorov-Smirnov distance below 1.36 / sqrt(B).
The prefixes run in blocks of 32, one test per block, so that progress shows between blocks."""
import os

import numpy as np
import pytest

from oracle.metrics import porter_thomas, rel_err
from workloads.bitstrings import random_bitstrings
from workloads.circuits import generate
from workloads.plans import plan_7x7

pytestmark = pytest.mark.gpu

N_PREFIX = 256
BLOCK = 32
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "c3_prefixes.npz")
_results = {}


@pytest.fixture(scope="module")
def c3():
    import torch
    from paper_1905_00444_amd import Context, Circuit, Plan
    assert torch.cuda.is_available()
    circ = generate(7, 7, 32, 0)
    plan, _ = plan_7x7(circ, 32)
    ctx = Context(0)
    p = Plan(ctx, Circuit(ctx, circ.to_text()), plan, "fp32")
    return p, random_bitstrings(N_PREFIX, 49, 1)


@pytest.mark.parametrize("block", range(N_PREFIX // BLOCK))
def test_c3_block_of_prefixes(c3, block):
    import torch
    p, bits = c3
    print(f"7x7 d32 FP32, prefixes {block * BLOCK}..{(block + 1) * BLOCK - 1}", flush=True)
    rows = bits[block * BLOCK:(block + 1) * BLOCK]
    got = p.amplitudes(rows)
    torch.cuda.synchronize()
    got = got.cpu().numpy()
    assert got.shape == (BLOCK, 64) and np.all(np.isfinite(got))
    _results[block] = got


def _all():
    if len(_results) != N_PREFIX // BLOCK:
        pytest.skip("needs every block of prefixes from this session")
    return np.concatenate([_results[b] for b in range(N_PREFIX // BLOCK)])


def test_c3_prefixes_match_fp64_oracle():
    amps = _all()
    if not os.path.exists(GOLDEN):
        pytest.skip("c3_prefixes.npz not generated yet (tests/golden/make_goldens.py)")
    g = np.load(GOLDEN)
    k = g["amps"].shape[0]
    assert np.array_equal(g["bits"], random_bitstrings(N_PREFIX, 49, 1)[:k])
    assert rel_err(amps[:k], g["amps"]) <= 1e-5


def test_c3_porter_thomas_16384_amplitudes():
    amps = _all()
    B = amps.size
    m1, m2, ks = porter_thomas(amps, 49)
    print(f"Porter-Thomas over {B} amplitudes: mean {m1:.4f}, second moment {m2:.4f}, KS {ks:.4f}", flush=True)
    assert 0.5e-15 < np.mean(np.abs(amps) ** 2) < 3e-15
    assert abs(m1 - 1.0) <= 0.03, m1
    assert abs(m2 - 2.0) <= 0.15, m2
    assert ks <= 1.36 / np.sqrt(B), ks
