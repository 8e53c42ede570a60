"""torch.autograd.Function over the library's forward (qf_amplitudes) and hand-written
backward (qf_backward): amplitudes as a differentiable function of every gate's entries."""
from __future__ import annotations

import torch


class QFlexAmplitudes(torch.autograd.Function):
    """values: (n_ops, 4) complex64 gate entries in circuit order; plan: a Plan created with
    backward=True; bits: (n_batch, n) uint8.  Returns (n_batch, 2^n_open) complex128.

    The plan's circuit holds one set of gate values at a time, so the values of each forward are
    kept and written back into the circuit just before that forward's backward runs: interleaved
    forwards with different values each get their own gradient."""

    @staticmethod
    def forward(fctx, values, plan, bits, s_begin=0, s_end=None):
        vals = values.detach().to("cpu", torch.complex64).numpy().copy()
        plan.circuit.set_values(vals)
        out = plan.amplitudes(bits, s_begin, s_end)
        fctx.plan, fctx.bits, fctx.range = plan, bits, (s_begin, s_end)
        fctx.values_host = vals
        fctx.values_device = values.device
        return out

    @staticmethod
    def backward(fctx, grad_out):
        plan = fctx.plan
        plan.circuit.set_values(fctx.values_host)
        g = plan.backward(fctx.bits, grad_out.detach().to(torch.complex128), *fctx.range)
        return g.to(fctx.values_device), None, None, None, None


def amplitudes(values, plan, bits, s_begin=0, s_end=None):
    return QFlexAmplitudes.apply(values, plan, bits, s_begin, s_end)
